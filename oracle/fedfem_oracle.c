/*
 * FED-FEM FP64 CPU oracle -- TEST INFRASTRUCTURE, not part of the product.
 *
 * Only the test suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this library.  It shares no code with the GPU library.
 *
 * It follows Zhang & Chauhan, "Real-time computation of bio-heat transfer in
 * the fast explicit dynamics finite element algorithm (FED-FEM) framework"
 * (arXiv 1909.05098), Algorithm 1, for four-node linear tetrahedra, in double
 * precision, with plain loops in the paper's order:
 *
 *   pre-computation  (Algorithm 1, pre-computation block; Eq 15-16, Sec 2.3.5)
 *     per element: Jacobian J, det J, V_tet = |det J|/6, gradient matrix B,
 *                  A = V_tet B^T B                                  (Eq 16)
 *     per node:    lumped volume V_i = sum_e V_e / 4 (mass shared equally
 *                  among element nodes, Sec 2.3.4), K_b,i = w_b c_b V_i,
 *                  Q_b,i = w_b c_b T_a V_i, Q_m,i = Q_m V_i         (Sec 2.3.5)
 *   time stepping    (Algorithm 1, time-stepping block)
 *     per element: k_e = mean of k(T_n) over its 4 nodes            (Eq 13)
 *                  F_e = k_e A T_e                                   (Eq 17)
 *     assembly:    F_i = sum of F_e rows over the elements of node i,
 *                  in ascending element order                       (Eq 11)
 *     per node:    T_i += dt / C_i(T) * (q_i + Q_m,i + Q_b,i - K_b,i T_i - F_i)
 *                                                                    (Eq 19)
 *                  Dirichlet nodes are held at T_Gamma              (Eq 3)
 *
 * Readings of the paper used here (each is listed with its reason in the
 * design notes):
 *   - Sign of the conduction term: F_e = k A T with A positive semi-definite
 *     (Eq 12, 15, 17) is the outflow of heat, so it enters Eq 19 with a minus
 *     sign; the printed "+F" of Eq 7-10, 18, 19 would be anti-diffusive.
 *   - C_i(T) = rho(T_i) c(T_i) V_i at the node's current temperature.
 *   - Properties are p(T) = p0 + dp/dT (clamp(T, T_lo, T_hi) - T_ref): the
 *     paper's two-point tables with linear interpolation and constant
 *     extension outside the tabulated range.  Eq 13 clamps each node, then
 *     averages.
 *   - w_b is a mass perfusion rate [kg/(m^3 s)] (Eq 1).
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

/* Material vector layout (13 doubles). */
enum {
    M_RHO0 = 0, M_C0, M_K0, M_DRHO, M_DC, M_DK, M_TREF, M_TLO, M_THI,
    M_WB, M_CB, M_TA, M_QM, M_COUNT
};

typedef struct {
    int64_t n_nodes;
    int64_t n_tets;
    const int32_t *tets;    /* [E][4] node ids                               */
    const double *A;        /* [E][4][4] element matrices A = V B^T B        */
    const double *Vi;       /* [N] lumped nodal volumes                      */
    const double *mat;      /* [13] material vector                         */
    const uint8_t *is_dir;  /* [N] 1 = Dirichlet node                        */
    const double *T_dir;    /* [N] prescribed value where is_dir             */
    const double *q;        /* [N] nodal heat flow Q_r,i [W]; NULL = none    */
    const int64_t *csr_off; /* [N+1] node -> incident (element, corner)      */
    const int64_t *csr_ec;  /* [4E]  entries e*4+corner, ascending e         */
    double dt;
    int n_threads;
    const double *tabs;     /* NULL, or property tables (see prop_table)     */
} oracle_problem;

/* Property tables: for property p (0 k, 1 rho, 2 c) the block
 * tabs[p * ORACLE_TAB_STRIDE ...] holds the point count n (0 = use the
 * linear law), then ORACLE_MAX_TAB temperatures, then ORACLE_MAX_TAB values. */
#define ORACLE_MAX_TAB 16
#define ORACLE_TAB_STRIDE (1 + 2 * ORACLE_MAX_TAB)

static double clamp_T(double T, const double *m)
{
    if (T < m[M_TLO]) return m[M_TLO];
    if (T > m[M_THI]) return m[M_THI];
    return T;
}

/* Linear interpolation in a table of n points (temperatures increasing),
 * constant beyond its first and last point; returns 0 for n = 0. */
static int prop_table(const double *tabs, int p, double T, double *out)
{
    if (!tabs) return 0;
    const double *b = tabs + p * ORACLE_TAB_STRIDE;
    int n = (int)b[0];
    const double *t = b + 1, *v = b + 1 + ORACLE_MAX_TAB;
    if (n <= 0) return 0;
    if (T <= t[0]) { *out = v[0]; return 1; }
    if (T >= t[n - 1]) { *out = v[n - 1]; return 1; }
    int k = 0;
    while (t[k + 1] <= T) k++;
    *out = v[k] + (v[k + 1] - v[k]) * (T - t[k]) / (t[k + 1] - t[k]);
    return 1;
}

/* p(T) = p0 + dp/dT (clamp(T) - T_ref), or the property's table */
static double prop_k(double T, const double *m, const double *tabs)
{
    double v;
    if (prop_table(tabs, 0, T, &v)) return v;
    return m[M_K0] + m[M_DK] * (clamp_T(T, m) - m[M_TREF]);
}

static double prop_rho_c(double T, const double *m, const double *tabs)
{
    double Tc = clamp_T(T, m) - m[M_TREF];
    double rho = m[M_RHO0] + m[M_DRHO] * Tc, c = m[M_C0] + m[M_DC] * Tc;
    prop_table(tabs, 1, T, &rho);
    prop_table(tabs, 2, T, &c);
    return rho * c;
}

static void set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

int oracle_max_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/*
 * Element pre-computation (Algorithm 1, element loop of the pre-computation
 * block; Eq 15-16).  Natural coordinates xi map to x = x0 + sum_k xi_k
 * (x_k - x0), so the Jacobian's columns are the edge vectors x_k - x0 and
 * grad N_k = row k of J^-1 for k = 1..3, grad N_0 = -(sum of the others).
 *
 * Outputs (any may be NULL): A [E][4][4], vol [E], detJ [E], gradN [E][4][3].
 * Returns -1, or the first element with |det J| <= 1e-12 * (longest edge)^3.
 */
int64_t oracle_geometry(int64_t n_tets, const double *xyz, const int32_t *tets,
                        double *A, double *vol, double *detJ, double *gradN,
                        int n_threads)
{
    int64_t bad = -1;
    set_threads(n_threads);
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < n_tets; e++) {
        const double *p[4];
        for (int a = 0; a < 4; a++) p[a] = xyz + 3 * (int64_t)tets[4 * e + a];
        double J[3][3];              /* J[i][k] = (x_{k+1} - x_0)_i */
        for (int i = 0; i < 3; i++)
            for (int k = 0; k < 3; k++) J[i][k] = p[k + 1][i] - p[0][i];
        double det = J[0][0] * (J[1][1] * J[2][2] - J[1][2] * J[2][1])
                   - J[0][1] * (J[1][0] * J[2][2] - J[1][2] * J[2][0])
                   + J[0][2] * (J[1][0] * J[2][1] - J[1][1] * J[2][0]);
        double lmax = 0.0;
        for (int a = 0; a < 4; a++)
            for (int b = a + 1; b < 4; b++) {
                double d0 = p[a][0] - p[b][0], d1 = p[a][1] - p[b][1],
                       d2 = p[a][2] - p[b][2];
                double l = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
                if (l > lmax) lmax = l;
            }
        if (!(fabs(det) > 1e-12 * lmax * lmax * lmax)) {
#pragma omp critical
            {
                if (bad < 0 || e < bad) bad = e;
            }
            continue;
        }
        /* inverse by the adjugate: Jinv[k][i] = cof(J)[i][k] / det */
        double Ji[3][3];
        Ji[0][0] = (J[1][1] * J[2][2] - J[1][2] * J[2][1]) / det;
        Ji[0][1] = (J[0][2] * J[2][1] - J[0][1] * J[2][2]) / det;
        Ji[0][2] = (J[0][1] * J[1][2] - J[0][2] * J[1][1]) / det;
        Ji[1][0] = (J[1][2] * J[2][0] - J[1][0] * J[2][2]) / det;
        Ji[1][1] = (J[0][0] * J[2][2] - J[0][2] * J[2][0]) / det;
        Ji[1][2] = (J[0][2] * J[1][0] - J[0][0] * J[1][2]) / det;
        Ji[2][0] = (J[1][0] * J[2][1] - J[1][1] * J[2][0]) / det;
        Ji[2][1] = (J[0][1] * J[2][0] - J[0][0] * J[2][1]) / det;
        Ji[2][2] = (J[0][0] * J[1][1] - J[0][1] * J[1][0]) / det;
        double B[3][4];              /* B[:, a] = grad N_a */
        for (int i = 0; i < 3; i++) {
            B[i][1] = Ji[0][i];
            B[i][2] = Ji[1][i];
            B[i][3] = Ji[2][i];
            B[i][0] = -(B[i][1] + B[i][2] + B[i][3]);
        }
        double V = fabs(det) / 6.0;
        if (vol) vol[e] = V;
        if (detJ) detJ[e] = det;
        if (gradN)
            for (int a = 0; a < 4; a++)
                for (int i = 0; i < 3; i++) gradN[12 * e + 3 * a + i] = B[i][a];
        if (A)
            for (int a = 0; a < 4; a++)
                for (int b = 0; b < 4; b++) {
                    double s = 0.0;
                    for (int i = 0; i < 3; i++) s += B[i][a] * B[i][b];
                    A[16 * e + 4 * a + b] = V * s;
                }
    }
    return bad;
}

/*
 * Node -> (element, corner) lists in ascending element order, built by a
 * counting sort.  off has N+1 entries, ec has 4E entries holding e*4+corner.
 */
void oracle_build_csr(int64_t n_nodes, int64_t n_tets, const int32_t *tets,
                      int64_t *off, int64_t *ec)
{
    memset(off, 0, sizeof(int64_t) * (size_t)(n_nodes + 1));
    for (int64_t s = 0; s < 4 * n_tets; s++) off[tets[s] + 1]++;
    for (int64_t i = 0; i < n_nodes; i++) off[i + 1] += off[i];
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n_nodes + 1));
    memcpy(fill, off, sizeof(int64_t) * (size_t)(n_nodes + 1));
    for (int64_t s = 0; s < 4 * n_tets; s++) ec[fill[tets[s]]++] = s;
    free(fill);
}

/* Lumped nodal volume V_i = sum over incident elements of V_e / 4. */
void oracle_lumped_volume(int64_t n_nodes, const double *vol,
                          const int64_t *off, const int64_t *ec, double *Vi,
                          int n_threads)
{
    set_threads(n_threads);
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_nodes; i++) {
        double s = 0.0;
        for (int64_t k = off[i]; k < off[i + 1]; k++) s += vol[ec[k] / 4] / 4.0;
        Vi[i] = s;
    }
}

/*
 * One explicit step (Algorithm 1, time-stepping block).
 * T_in [N] -> T_out [N].  Optional outputs: F [N] assembled conduction loads
 * (Eq 11) and C [N] lumped thermal mass C_i(T_in).  Fe is scratch [4E].
 */
void oracle_step(const oracle_problem *p, const double *T_in, double *T_out,
                 double *F, double *C, double *Fe)
{
    const double *m = p->mat;
    set_threads(p->n_threads);
    /* element loop: Eq 13 then Eq 17 */
#pragma omp parallel for schedule(static)
    for (int64_t e = 0; e < p->n_tets; e++) {
        const int32_t *n = p->tets + 4 * e;
        double Te[4];
        double ke = 0.0;
        for (int a = 0; a < 4; a++) {
            Te[a] = T_in[n[a]];
            ke += prop_k(Te[a], m, p->tabs);
        }
        ke /= 4.0;
        const double *Ae = p->A + 16 * e;
        for (int a = 0; a < 4; a++) {
            double s = 0.0;
            for (int b = 0; b < 4; b++) s += Ae[4 * a + b] * Te[b];
            Fe[4 * e + a] = ke * s;
        }
    }
    /* node loop: Eq 11 (ascending element order) then Eq 19 */
    const double wbcb = m[M_WB] * m[M_CB];
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < p->n_nodes; i++) {
        double Fi = 0.0;
        for (int64_t k = p->csr_off[i]; k < p->csr_off[i + 1]; k++)
            Fi += Fe[p->csr_ec[k]];
        double Ti = T_in[i];
        double Ci = prop_rho_c(Ti, m, p->tabs) * p->Vi[i];
        if (F) F[i] = Fi;
        if (C) C[i] = Ci;
        if (p->is_dir[i]) {
            T_out[i] = p->T_dir[i];
            continue;
        }
        double Kb = wbcb * p->Vi[i];
        double Qb = wbcb * m[M_TA] * p->Vi[i];
        double Qm = m[M_QM] * p->Vi[i];
        double Qr = p->q ? p->q[i] : 0.0;
        T_out[i] = Ti + p->dt / Ci * (Qr + Qm + Qb - Kb * Ti - Fi);
    }
}

/*
 * n explicit steps.  T [N] holds T(t) on entry and T(t + n dt) on return.
 * Dirichlet nodes are set to T_Gamma before the first step (Eq 3 holds at
 * every step, including the initial state).
 */
int oracle_run(const oracle_problem *p, int64_t n_steps, double *T)
{
    int64_t N = p->n_nodes;
    double *Tb = (double *)malloc(sizeof(double) * (size_t)N);
    double *Fe = (double *)malloc(sizeof(double) * (size_t)(4 * p->n_tets));
    if (!Tb || !Fe) {
        free(Tb);
        free(Fe);
        return -1;
    }
    for (int64_t i = 0; i < N; i++)
        if (p->is_dir[i]) T[i] = p->T_dir[i];
    double *cur = T, *nxt = Tb;
    for (int64_t s = 0; s < n_steps; s++) {
        oracle_step(p, cur, nxt, NULL, NULL, Fe);
        double *t = cur;
        cur = nxt;
        nxt = t;
    }
    if (cur != T) memcpy(T, cur, sizeof(double) * (size_t)N);
    free(Tb);
    free(Fe);
    return 0;
}

/* ---------------------------------------------------------------------- */
/* Gaussian regional heat sources -> nodal heat flows Q_r,i [W].           */
/* Q_r(x) = Q0 exp(-|x - c|^2 / (2 sigma^2)) [W/m^3]; params per source:    */
/* (cx, cy, cz, sigma, Q0).                                                 */
/* ---------------------------------------------------------------------- */

static double gauss_density(const double *x, const double *src, int n_src)
{
    double s = 0.0;
    for (int k = 0; k < n_src; k++) {
        const double *g = src + 5 * k;
        double dx = x[0] - g[0], dy = x[1] - g[1], dz = x[2] - g[2];
        s += g[4] * exp(-(dx * dx + dy * dy + dz * dz) / (2.0 * g[3] * g[3]));
    }
    return s;
}

/* Nodal sampling: Q_r,i = Q_r(x_i) V_i. */
void oracle_source_nodal(int64_t n_nodes, const double *xyz, const double *Vi,
                         int n_src, const double *src, double *q)
{
    for (int64_t i = 0; i < n_nodes; i++)
        q[i] = gauss_density(xyz + 3 * i, src, n_src) * Vi[i];
}

/*
 * Composite quadrature for Q_r,i = integral of Q_r N_i over the mesh.
 * Every tetrahedron is refined twice by regular (Bey) subdivision into 64
 * children of volume V/64; each child carries the symmetric 4-point degree-2
 * rule (barycentric (a,b,b,b) and permutations, a = (5+3 sqrt5)/20,
 * b = (5-sqrt5)/20, weight 1/4).  The 256 points are kept in parent
 * barycentric coordinates, so N_i at a point is its i-th coordinate.
 * The refinement depends on which corner is which, so before refining, the
 * element's corners are put in lexicographic (x, then y, then z) order of
 * their coordinates; the integral is then independent of the numbering.
 * An element whose bounding sphere (centroid, largest centroid-vertex
 * distance) lies wholly beyond 8 sigma of a source gets nothing from it.
 */
#define QN 256
static double g_qbar[QN][4];
static int g_q_ready = 0;

static void subdivide(const double v[4][4], int level, int *n)
{
    if (level == 0) {
        const double a = (5.0 + 3.0 * sqrt(5.0)) / 20.0;
        const double b = (5.0 - sqrt(5.0)) / 20.0;
        for (int q = 0; q < 4; q++) {
            for (int i = 0; i < 4; i++) {
                double s = 0.0;
                for (int k = 0; k < 4; k++) s += (k == q ? a : b) * v[k][i];
                g_qbar[*n][i] = s;
            }
            (*n)++;
        }
        return;
    }
    double m[4][4][4]; /* m[i][j] = midpoint of v_i, v_j */
    for (int i = 0; i < 4; i++)
        for (int j = 0; j < 4; j++)
            for (int c = 0; c < 4; c++) m[i][j][c] = 0.5 * (v[i][c] + v[j][c]);
    const double *child[8][4] = {
        {v[0], m[0][1], m[0][2], m[0][3]},
        {m[0][1], v[1], m[1][2], m[1][3]},
        {m[0][2], m[1][2], v[2], m[2][3]},
        {m[0][3], m[1][3], m[2][3], v[3]},
        /* inner octahedron split along the m02 - m13 diagonal */
        {m[0][1], m[0][2], m[0][3], m[1][3]},
        {m[0][1], m[0][2], m[1][2], m[1][3]},
        {m[0][2], m[0][3], m[1][3], m[2][3]},
        {m[0][2], m[1][2], m[1][3], m[2][3]},
    };
    for (int c = 0; c < 8; c++) {
        double w[4][4];
        for (int k = 0; k < 4; k++) memcpy(w[k], child[c][k], sizeof(w[k]));
        subdivide(w, level - 1, n);
    }
}

static void quad_init(void)
{
    if (g_q_ready) return;
    double v[4][4] = {{1, 0, 0, 0}, {0, 1, 0, 0}, {0, 0, 1, 0}, {0, 0, 0, 1}};
    int n = 0;
    subdivide(v, 2, &n);
    g_q_ready = 1;
}

/* Quadrature points in parent barycentric coordinates, for inspection. */
void oracle_quadrature_points(double *out /* [256][4] */)
{
    quad_init();
    memcpy(out, g_qbar, sizeof(g_qbar));
}

void oracle_source_consistent(int64_t n_nodes, const double *xyz,
                              int64_t n_tets, const int32_t *tets,
                              const double *vol, const int64_t *off,
                              const int64_t *ec, int n_src, const double *src,
                              double *q, int n_threads)
{
    quad_init();
    double *qe = (double *)calloc((size_t)(4 * n_tets), sizeof(double));
    set_threads(n_threads);
#pragma omp parallel for schedule(dynamic, 1024)
    for (int64_t e = 0; e < n_tets; e++) {
        const double *p[4];
        int corner[4]; /* corner[r] = element corner placed at rank r */
        for (int a = 0; a < 4; a++) corner[a] = a;
        for (int a = 1; a < 4; a++) /* insertion sort by coordinates */
            for (int b = a; b > 0; b--) {
                const double *u = xyz + 3 * (int64_t)tets[4 * e + corner[b - 1]];
                const double *v = xyz + 3 * (int64_t)tets[4 * e + corner[b]];
                int greater = u[0] != v[0] ? u[0] > v[0]
                            : (u[1] != v[1] ? u[1] > v[1] : u[2] > v[2]);
                if (!greater) break;
                int t = corner[b - 1];
                corner[b - 1] = corner[b];
                corner[b] = t;
            }
        for (int r = 0; r < 4; r++)
            p[r] = xyz + 3 * (int64_t)tets[4 * e + corner[r]];
        double cen[3] = {0, 0, 0};
        for (int a = 0; a < 4; a++)
            for (int i = 0; i < 3; i++) cen[i] += p[a][i] / 4.0;
        double rad = 0.0;
        for (int a = 0; a < 4; a++) {
            double d0 = p[a][0] - cen[0], d1 = p[a][1] - cen[1],
                   d2 = p[a][2] - cen[2];
            double r = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            if (r > rad) rad = r;
        }
        double acc[4] = {0, 0, 0, 0};
        for (int k = 0; k < n_src; k++) {
            const double *g = src + 5 * k;
            double d0 = cen[0] - g[0], d1 = cen[1] - g[1], d2 = cen[2] - g[2];
            double dist = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            if (dist - rad > 8.0 * g[3]) continue;
            for (int qi = 0; qi < QN; qi++) {
                double x[3] = {0, 0, 0};
                for (int a = 0; a < 4; a++)
                    for (int i = 0; i < 3; i++) x[i] += g_qbar[qi][a] * p[a][i];
                double f = gauss_density(x, g, 1);
                for (int a = 0; a < 4; a++) acc[a] += f * g_qbar[qi][a];
            }
        }
        for (int r = 0; r < 4; r++) qe[4 * e + corner[r]] = acc[r] * vol[e] / QN;
    }
#pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < n_nodes; i++) {
        double s = 0.0;
        for (int64_t k = off[i]; k < off[i + 1]; k++) s += qe[ec[k]];
        q[i] = s;
    }
    free(qe);
}
