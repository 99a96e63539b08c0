/*
 * The FP64 oracle's OpenMP loops under ThreadSanitizer (test infrastructure
 * checking test infrastructure).  The oracle parallelises element geometry,
 * lumping, the consistent source and each time step (Algorithm 1's element
 * and node loops); this driver runs all of them on a jittered Kuhn box with
 * 4 threads and with 1 thread and requires bit-identical temperatures, as
 * the oracle sums every node in a fixed order whatever the thread count.
 * Built by the test with clang -fopenmp -fsanitize=thread and run with the
 * Archer OpenMP tool, which tells ThreadSanitizer about OpenMP's barriers.
 */
#include <stdio.h>

#include "../../oracle/fedfem_oracle.c"

#define NX 14
#define NY 12
#define NZ 10

static int nid(int i, int j, int k) { return (k * (NY + 1) + j) * (NX + 1) + i; }

int main(void)
{
    const int64_t N = (int64_t)(NX + 1) * (NY + 1) * (NZ + 1);
    const int64_t E = 6LL * NX * NY * NZ;
    const double h = 1e-3;
    double *xyz = malloc(sizeof(double) * 3 * N);
    int32_t *tets = malloc(sizeof(int32_t) * 4 * E);
    uint8_t *is_dir = calloc(N, 1);
    double *T_dir = calloc(N, sizeof(double));
    uint64_t s = 12345;
    for (int k = 0; k <= NZ; k++)
        for (int j = 0; j <= NY; j++)
            for (int i = 0; i <= NX; i++) {
                int inner = i > 0 && j > 0 && k > 0 && i < NX && j < NY && k < NZ;
                double *p = xyz + 3 * nid(i, j, k);
                double c[3] = {i * h, j * h, k * h};
                for (int a = 0; a < 3; a++) {
                    s = s * 6364136223846793005ULL + 1442695040888963407ULL;
                    double u = (double)(s >> 11) / 9007199254740992.0 * 2.0 - 1.0;
                    p[a] = c[a] + (inner ? 0.2 * h * u : 0.0);
                }
                if (!inner) {
                    is_dir[nid(i, j, k)] = 1;
                    T_dir[nid(i, j, k)] = 37.0;
                }
            }
    static const int perm[6][3] = {{0, 1, 2}, {0, 2, 1}, {1, 0, 2}, {1, 2, 0}, {2, 0, 1}, {2, 1, 0}};
    int64_t e = 0;
    for (int k = 0; k < NZ; k++)
        for (int j = 0; j < NY; j++)
            for (int i = 0; i < NX; i++)
                for (int t = 0; t < 6; t++) {
                    int c[3] = {0, 0, 0};
                    tets[4 * e] = nid(i, j, k);
                    for (int a = 0; a < 3; a++) {
                        c[perm[t][a]] = 1;
                        tets[4 * e + 1 + a] = nid(i + c[0], j + c[1], k + c[2]);
                    }
                    e++;
                }
    /* temperature-dependent laws with perfusion and metabolic heat */
    double mat[M_COUNT] = {1060.0, 3600.0, 0.512, 0.0, -1.8, 0.0006656, 37.0, 0.0, 100.0,
                           6.4, 4180.0, 37.0, 500.0};
    double *A = malloc(sizeof(double) * 16 * E), *vol = malloc(sizeof(double) * E);
    double *detJ = malloc(sizeof(double) * E), *gradN = malloc(sizeof(double) * 12 * E);
    int64_t *off = malloc(sizeof(int64_t) * (N + 1)), *ec = malloc(sizeof(int64_t) * 4 * E);
    double *Vi = malloc(sizeof(double) * N), *q = malloc(sizeof(double) * N);
    double *T[2] = {malloc(sizeof(double) * N), malloc(sizeof(double) * N)};
    const double src[5] = {7e-3, 6e-3, 5e-3, 1.5e-3, 4e8};
    const int threads[2] = {4, 1};
    for (int r = 0; r < 2; r++) {
        if (oracle_geometry(E, xyz, tets, A, vol, detJ, gradN, threads[r]) >= 0) {
            printf("degenerate element\n");
            return 1;
        }
        oracle_build_csr(N, E, tets, off, ec);
        oracle_lumped_volume(N, vol, off, ec, Vi, threads[r]);
        oracle_source_consistent(N, xyz, E, tets, vol, off, ec, 1, src, q, threads[r]);
        oracle_problem p = {N, E, tets, A, Vi, mat, is_dir, T_dir, q, off, ec, 0.05,
                            threads[r], NULL};
        for (int64_t i = 0; i < N; i++) T[r][i] = is_dir[i] ? T_dir[i] : 37.0;
        if (oracle_run(&p, 40, T[r]) != 0) {
            printf("oracle_run failed\n");
            return 1;
        }
    }
    double peak = 0.0;
    for (int64_t i = 0; i < N; i++) {
        if (T[0][i] != T[1][i]) {
            printf("node %lld: %.17g with 4 threads, %.17g with 1\n", (long long)i, T[0][i],
                   T[1][i]);
            return 1;
        }
        if (T[0][i] > peak) peak = T[0][i];
    }
    printf("oracle_threads: %lld nodes bit-identical with 4 and 1 threads (peak %.4f C)\n",
           (long long)N, peak);
    return 0;
}
