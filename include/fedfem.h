/*
 * fedfem.h -- C ABI of the MI355X (gfx950) FED-FEM bio-heat library.
 *
 * The library advances the Pennes bio-heat equation (Zhang & Chauhan,
 * arXiv 1909.05098, Eq 1-2) on a mesh of four-node linear tetrahedra with
 * the fast explicit dynamics finite element algorithm (Algorithm 1):
 * pre-computed element matrices A = V_tet B^T B (Eq 15-16), element-level
 * thermal loads F_e = k(T) A T_e with k averaged over the element's nodes
 * (Eq 13, 17), assembly at the nodes (Eq 11) and the explicit nodal update
 * with lumped capacity and perfusion (Eq 19).
 *
 * Conventions shared by every entry point:
 *   - All host values are double precision, SI units, temperatures in degC.
 *   - Node and element ids are 0-based and refer to the caller's numbering;
 *     the library may renumber internally but never exposes that order.
 *   - Every function returns FEDFEM_OK (0) or a negative FEDFEM_E_* code.
 *     No C++ exception crosses the ABI.  A handle is not thread-safe.
 *   - Host pointers passed in are only read during the call (the library
 *     deep-copies what it keeps); the caller keeps ownership.
 *   - After FEDFEM_E_HIP a handle is unusable except for fedfem_destroy.
 */
#ifndef FEDFEM_H
#define FEDFEM_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ---- return codes ------------------------------------------------------ */
#define FEDFEM_OK 0
#define FEDFEM_E_INVALID (-1)         /* bad argument; see fedfem_last_error */
#define FEDFEM_E_DEGENERATE (-2)      /* |det J| <= 1e-12 (longest edge)^3   */
#define FEDFEM_E_NOT_PRECOMPUTED (-3) /* call fedfem_precompute first        */
#define FEDFEM_E_UNSTABLE (-4)        /* dt >= critical dt (Eq 9)            */
#define FEDFEM_E_DIVERGED (-5)        /* non-finite or |T| > 1e4 degC seen   */
#define FEDFEM_E_HIP (-6)             /* HIP runtime failure (sticky)        */
#define FEDFEM_E_NOMEM (-7)           /* host or device allocation failed    */
#define FEDFEM_E_STATE (-8)           /* call not valid in the current state */
#define FEDFEM_E_TOO_LARGE (-9)       /* beyond fedfem_step_static's scratch */

/* ---- precision of the time-stepping kernels ----------------------------- */
#define FEDFEM_FP64 0  /* element loop and nodal state in double             */
#define FEDFEM_FP32C 1 /* element loop in float; nodal T carried as a        */
                       /* compensated float pair hi + lo                      */

/* ---- how a Gaussian source density becomes nodal heat flows ------------ */
#define FEDFEM_SOURCE_NODAL 0      /* Q_i = Q_r(x_i) V_i (lumped volume)     */
#define FEDFEM_SOURCE_CONSISTENT 1 /* Q_i = integral of Q_r N_i dV           */

/* Mesh (Sec 2.3.3): xyz is [n_nodes][3] metres, tets is [n_tets][4]. */
typedef struct {
    int64_t n_nodes;
    const double *xyz;
    int64_t n_tets;
    const int32_t *tets;
} fedfem_mesh;

/*
 * Tissue and blood properties (Eq 1-2).  Each tissue property follows
 *   p(T) = p0 + dp_dT * (clamp(T, T_lo, T_hi) - T_ref),
 * i.e. linear interpolation of tabulated data with constant extension
 * outside [T_lo, T_hi] (Sec 3.1.6).  w_b is the perfusion mass rate
 * [kg/(m^3 s)], c_b the blood heat capacity, T_a the arterial temperature,
 * Q_m the metabolic heat density [W/m^3].  rho(T) c(T) and k(T) must stay
 * positive on the window.
 */
typedef struct {
    double rho0, c0, k0;
    double drho_dT, dc_dT, dk_dT;
    double T_ref, T_lo, T_hi;
    double w_b, c_b, T_a, Q_m;
    int32_t precision; /* FEDFEM_FP64 or FEDFEM_FP32C */
} fedfem_materials;

/*
 * Initial and essential boundary conditions (Eq 3; Algorithm 1,
 * initialisation).  Dirichlet nodes are held at dir_T from the initial state
 * on.  dt > 0 fixes the step; -1 < dt < 0 asks for |dt| times the critical
 * step found by fedfem_precompute (Eq 9).
 */
typedef struct {
    double T0;
    int64_t n_dir;
    const int32_t *dir_nodes;
    const double *dir_T;
    double dt;
} fedfem_bc;

/*
 * Layout options, read by fedfem_precompute.  reorder = 1 renumbers nodes
 * and elements along a Morton (Z-order) curve of their coordinates, 0 keeps
 * the caller's order.  Elements are processed in tiles of consecutive
 * elements whose loads are gathered in on-chip memory before assembly:
 * tile_elems (64..8192, multiple of 64; 0 = 2048) bounds the elements of a
 * tile and max_tile_nodes (4..4*tile_elems; 0 = tile_elems/2 with reorder,
 * 4*tile_elems without) the distinct nodes it may touch.  threads is the
 * element kernel's workgroup size (64..1024, multiple of 64, dividing
 * tile_elems into 1, 2 or 4 elements per thread; 0 = tile_elems/4 within
 * [64, 1024]).  xcd = 1 maps workgroups so that each of the 8 XCDs walks one
 * contiguous stretch of the element order.
 */
typedef struct {
    int32_t reorder;
    int32_t tile_elems;
    int32_t threads;
    int32_t max_tile_nodes;
    int32_t xcd;
    int32_t reserved[3];
} fedfem_options;

/* Sizes of the pre-computed layout, for reporting. */
typedef struct {
    int64_t n_nodes, n_tets, n_dirichlet;
    int64_t n_tiles, n_partials, max_tile_nodes;
    int32_t precision, tile_elems, threads, reorder;
    int64_t device_bytes;     /* device memory owned by the handle */
    double lambda_geometry;   /* top eigenvalue of (sum A_e, diag V) */
    int32_t lanczos_iterations;
    /* exact tile sums (Eq 11): corner loads are added as 64-bit integers
     * in units of 2^-fixed_point_shift; the shift leaves room for the most
     * corners one tile places on a node (max_tile_valence) */
    int32_t max_tile_valence;
    int32_t fixed_point_shift;
    /* nodes that a single tile touches (reordered tetrahedral layouts; 0
     * otherwise): the nodal update reads their one tile sum at the node's
     * own index */
    int32_t n_single_tile_nodes;
    int32_t reserved[4];
} fedfem_info;

/*
 * A mesh of eight-node hexahedra (Sec 2.3.3, Eq 14).  Each element lists its
 * nodes in the order of its corners at natural coordinates (xi, eta, zeta) =
 * (-1,-1,-1), (1,-1,-1), (1,1,-1), (-1,1,-1), (-1,-1,1), (1,-1,1), (1,1,1),
 * (-1,1,1): one face counter-clockwise, then the opposite face in the same
 * order.  hexes is [8 * n_hexes] node ids; the caller keeps ownership.
 */
typedef struct {
    int64_t n_nodes;
    const double *xyz;
    int64_t n_hexes;
    const int32_t *hexes;
} fedfem_mesh_hex;

typedef struct fedfem_handle fedfem_handle;

/*
 * Create a handle: validates the mesh (counts, node ids, finite
 * coordinates), materials (positive properties on the window) and boundary
 * conditions (ids in range, no duplicates, finite values), deep-copies all
 * inputs, and creates the handle's HIP stream on the current device.  No
 * device memory is allocated until fedfem_precompute.
 */
int fedfem_create(const fedfem_mesh *mesh, const fedfem_materials *mat,
                  const fedfem_bc *bc, fedfem_handle **out);

/*
 * Create a handle on a mesh of eight-node hexahedra with one integration
 * point (Sec 2.3.3): the element matrix is A_e = 8 |det J| B^T B with J and
 * B at the element centre (Eq 14, 16), k_e the mean of k over the eight
 * nodes (Eq 13), and each node receives an eighth of every element volume
 * 8 |det J| (Sec 2.3.4).  The paper adds no hourglass control, and neither
 * does the library: fields with zero gradient at every element centre carry
 * no conduction load.  Validation, ownership and the rest of the API are as
 * for fedfem_create, with these differences: reordered tiles may hold up
 * to twice as many nodes as elements (default 4096 for 2048-element
 * tiles); surface flux takes quadrilateral faces (fedfem_flux_loads_quad;
 * fedfem_flux_loads and fedfem_resample give FEDFEM_E_INVALID, being
 * defined on triangles and tetrahedra); batches accept tetrahedral handles
 * only (FEDFEM_E_STATE).  fedfem_get_info reports elements in
 * n_tets.
 */
int fedfem_create_hex(const fedfem_mesh_hex *mesh, const fedfem_materials *mat,
                      const fedfem_bc *bc, fedfem_handle **out);

/* Set layout options (before fedfem_precompute; FEDFEM_E_STATE after). */
int fedfem_set_options(fedfem_handle *h, const fedfem_options *opt);

/*
 * Autotuner: choose layout options for this handle's mesh by timing
 * candidate layouts (Morton order with 1024, 2048 and 4096-element tiles,
 * the caller's order with 1024-element tiles; for hexahedra 512, 1024 and
 * 2048, and the caller's order with 512; each with 4, 2 and 1 elements per
 * thread and both XCD mappings) on the GPU with HIP events, and set the fastest
 * (element pass + node pass per step) as the handle's options.  With
 * FEDFEM_TUNE_BATCH in flags only layouts that share one workgroup size in a
 * batch are tried (Morton order, 1024 or 2048-element tiles, 4 elements per
 * thread).  Must run before fedfem_precompute.  cache_path (NULL = no cache)
 * is a text file of earlier choices keyed by flags, precision and mesh size
 * (quarter-octave buckets of the element count); a hit skips the timing, a
 * miss appends a line.  chosen (NULL allowed) receives the options.
 * Temporary device memory of one extra layout at a time is used.
 */
#define FEDFEM_TUNE_BATCH 1
int fedfem_autotune(fedfem_handle *h, const char *cache_path, int32_t flags,
                    fedfem_options *chosen);

/*
 * Pre-computation (Algorithm 1, pre-computation block; Sec 2.3.5), on the
 * GPU in double precision: Jacobians, volumes, gradients and element
 * matrices (Eq 15-16), lumped nodal volumes (Sec 2.3.4), the critical step
 * (Eq 9) by Lanczos iteration on (sum_e A_e, diag V) over the free nodes
 * bounded over the property window, and the initial state.  Returns
 * FEDFEM_E_DEGENERATE naming the first bad element in fedfem_last_error,
 * FEDFEM_E_UNSTABLE if a fixed dt is not below the critical step.
 */
int fedfem_precompute(fedfem_handle *h);

/*
 * Temperature-dependent properties from tables (Eq 2; Sec 3.1.6 gives the
 * tissue's density, conductivity and specific heat at two temperatures and
 * interpolates linearly): n points (T [degC] strictly increasing, value > 0)
 * per property, interpolated linearly and held constant outside the table
 * (the constant extension used for the clamped linear laws).  n = 0 keeps
 * the material's linear law for that property (k0 + dk_dT (T - T_ref) on
 * [T_lo, T_hi], and likewise rho, c).  k(T) enters the element loads
 * (Eq 13: nodal k averaged over the element), rho(T) c(T) the lumped
 * capacity (Eq 19), and the critical step (Eq 9) uses the largest k and the
 * smallest rho c over all temperatures.  Must precede fedfem_precompute
 * (FEDFEM_E_STATE after); at most FEDFEM_MAX_TABLE points per table.
 */
#define FEDFEM_MAX_TABLE 16
int fedfem_set_property_tables(fedfem_handle *h, int32_t n_k, const double *T_k,
                               const double *k, int32_t n_rho,
                               const double *T_rho, const double *rho,
                               int32_t n_c, const double *T_c,
                               const double *c);

/*
 * fedfem_precompute on n distinct handles at once, by `threads` host
 * threads (0: the environment variable FEDFEM_PRECOMPUTE_THREADS if set,
 * else up to 16, one per core) that each take the next handle:
 * one scenario's host-side layout overlaps another's device work, each on
 * its handle's own stream.  rcs (may be NULL) receives each handle's return
 * code; the function returns the first nonzero one in handle order, else
 * FEDFEM_OK.  A NULL or repeated handle gives FEDFEM_E_INVALID before any
 * work starts.  The handles must not be used by other threads meanwhile.
 */
int fedfem_precompute_many(fedfem_handle *const *handles, int32_t n,
                           int32_t threads, int32_t *rcs);

/*
 * Advance n_steps explicit steps (Algorithm 1, time-stepping block;
 * Eq 13, 17, 11, 19).  source is a nodal heat flow Q_r [W] per node
 * (length n_nodes, caller's numbering); when non-NULL it replaces the active
 * source before stepping, when NULL the active source (zero initially) is
 * kept.  The n steps run as captured HIP graphs on the handle's stream; the
 * call returns after they finish.  Returns FEDFEM_E_DIVERGED if any node
 * went non-finite or beyond 1e4 degC (the state is then the post-step
 * state).
 */
int fedfem_step(fedfem_handle *h, int64_t n_steps, const double *source);

/*
 * fedfem_step without allocation, for callers that cannot allocate device
 * memory or instantiate graphs: tight serving loops and harnesses that
 * forbid allocation.  Same arguments, results (bit for bit) and return
 * codes as fedfem_step, but the steps are launched one by one on the
 * handle's stream, and the tile partials live in a device array of the
 * library's own, of fixed size (32 MiB), instead of the handle's buffer.
 * Each GPU the library runs on holds one copy of that array until the
 * process ends; every call on that GPU shares it, so calls on one GPU that
 * overlap in time (other host threads, other streams) race and must not be
 * made.  Refused: a handle whose partials exceed the array (n_partials *
 * 4 bytes in FEDFEM_FP32C, * 8 in FEDFEM_FP64; FEDFEM_E_TOO_LARGE, nothing
 * advances) and a handle with source schedules (FEDFEM_E_STATE).  Like
 * fedfem_step it waits for its steps before returning.
 */
int fedfem_step_static(fedfem_handle *h, int64_t n_steps, const double *source);

/*
 * Instantiate the HIP graphs that an n_steps call of fedfem_step uses (for
 * either ping-pong parity), so that the call itself launches without
 * capture cost, e.g. in a real-time loop.  Does not advance the state.
 */
int fedfem_prepare(fedfem_handle *h, int64_t n_steps);

/* Replace the active nodal source [W] (NULL = zero). */
int fedfem_set_source(fedfem_handle *h, const double *source);

/*
 * Set the active source from n_src Gaussian densities
 * Q_r(x) = Q0 exp(-|x - c|^2 / (2 sigma^2)) [W/m^3], params = n_src rows
 * of (cx, cy, cz, sigma, Q0).  mode FEDFEM_SOURCE_NODAL samples the density
 * at the nodes times the lumped nodal volume; FEDFEM_SOURCE_CONSISTENT
 * integrates Q_r N_i over each element with a 256-point composite rule (two
 * regular refinements, 4-point degree-2 rule per child, corners in
 * lexicographic coordinate order; on hexahedra the 4 x 4 x 4 Gauss-Legendre
 * rule on the trilinear map; elements whose bounding sphere lies beyond
 * 8 sigma get nothing).  Computed on the GPU in double precision.
 */
int fedfem_set_gaussian_sources(fedfem_handle *h, int32_t n_src,
                                const double *params, int32_t mode);

/* Copy the active nodal source [W] to host memory (length n_nodes). */
int fedfem_read_source(fedfem_handle *h, double *out);

/*
 * Time-varying sources on the device (Algorithm 1 applies the external heat
 * at every step; Sec 3.1.5 heats, then lets the tissue relax).  Pattern p is
 * a nodal heat-flow vector Q_p [W] in caller order (patterns: [n][N]); its
 * amplitude a_p(t) is piecewise linear through the points (times, amps) of
 * that pattern (n_points[p] points each, concatenated over the patterns,
 * times non-decreasing), constant before the first and after the last
 * point; where a time repeats, the last point given at it holds from that
 * time on, so a jump is two points at the same time.  Step n, from t_n to
 * t_n + dt, uses the source  q + sum_p a_p(t_n) Q_p,  where q is the source
 * of fedfem_set_source / fedfem_step and t_n the handle's time at the start
 * of the step (fedfem_get_time).  Amplitudes are evaluated in FP64 on the
 * host per graph chunk and applied in the working precision by the nodal
 * update.  n_patterns = 0 removes the schedule.  Requires a precomputed
 * handle; a batch refuses handles with a schedule (FEDFEM_E_STATE).
 */
#define FEDFEM_MAX_PATTERNS 4
int fedfem_set_schedule(fedfem_handle *h, int32_t n_patterns,
                        const double *patterns, const int32_t *n_points,
                        const double *times, const double *amps);

/*
 * Nodal loads of a prescribed surface heat flux on Gamma_H (Eq 4): each
 * triangle f = faces[3f..3f+2] (caller node ids, three distinct) with flux
 * flux[f] [W/m^2] into the body gives each of its three nodes
 * flux[f] |f| / 3, the integral of the flux against the linear shape
 * functions over the face.  out [N] (host, caller order) receives the
 * nodal sums [W], ready for fedfem_set_source or a schedule pattern.  Face
 * areas are computed on the device in FP64 and summed per node in ascending
 * face order.
 */
int fedfem_flux_loads(fedfem_handle *h, int64_t n_faces, const int32_t *faces,
                      const double *flux, double *out);

/*
 * The same on a hexahedral mesh, for bilinear quadrilaterals: faces is
 * [4 n_faces] caller node ids, each face's corners in order around it (four
 * distinct); corner a receives the integral of flux[f] N_a over the face,
 * by the 2 x 2 Gauss-Legendre rule on the bilinear map (exact on planar
 * parallelograms, where each corner gets flux[f] |f| / 4).  Sums per node
 * in ascending face order; FEDFEM_E_INVALID on a tetrahedral handle.
 */
int fedfem_flux_loads_quad(fedfem_handle *h, int64_t n_faces, const int32_t *faces,
                           const double *flux, double *out);

/*
 * Thermal dose accumulated at every node during the following steps.  The
 * paper names thermal dose computation for hyperthermia treatment planning
 * as the use of fast solutions (Sec 1) and as future work (Sec 5) without a
 * dose model; the library offers two published ones:
 *   FEDFEM_DOSE_CEM43      cumulative equivalent minutes at 43 C (Sapareto
 *                          and Dewey 1984): each second at T adds
 *                          R^(43 - T) / 60, R = 1/2 at or above 43 C and
 *                          1/4 below (a, b ignored);
 *   FEDFEM_DOSE_ARRHENIUS  damage integral (Henriques and Moritz 1947):
 *                          each second adds a exp(-b / (R_gas (T + 273.15)))
 *                          with frequency factor a > 0 [1/s], activation
 *                          energy b >= 0 [J/mol], R_gas = 8.314462618.
 * Step n (from t_n to t_n + dt) adds dt times the rate at the node's
 * temperature at t_n (the explicit update, Eq 19, takes every term there);
 * Dirichlet nodes accumulate at their held temperature.  The accumulators
 * are FP64, fused into the nodal update, and start at zero on every call
 * of fedfem_set_dose; FEDFEM_DOSE_OFF frees them.  The raw state
 * (fedfem_read_state / fedfem_write_state) does not include them.  A
 * batch refuses a handle with a dose model (FEDFEM_E_STATE).  Requires a
 * precomputed handle; FEDFEM_E_INVALID for an unknown model or bad a, b.
 */
#define FEDFEM_DOSE_OFF 0
#define FEDFEM_DOSE_CEM43 1
#define FEDFEM_DOSE_ARRHENIUS 2
int fedfem_set_dose(fedfem_handle *h, int32_t model, double a, double b);

/* Blocking copy of the accumulated dose [n_nodes] (CEM43 minutes or the
 * dimensionless Arrhenius integral) to host, caller node order;
 * FEDFEM_E_STATE when no dose model is set. */
int fedfem_read_dose(fedfem_handle *h, double *dose_out);

/* Blocking copy of the nodal temperatures (hi + lo in double) to host. */
int fedfem_read_T(fedfem_handle *h, double *T_out);

/* Same into device memory d_out (n_nodes doubles); synchronises. */
int fedfem_read_T_device(fedfem_handle *h, double *d_out);

/* Current step, critical step (Eq 9) and simulated time. */
int fedfem_get_dt(const fedfem_handle *h, double *dt, double *dt_cr);
int fedfem_get_time(const fedfem_handle *h, double *t, int64_t *steps);

/* Change the step; FEDFEM_E_UNSTABLE unless 0 < dt < dt_cr. */
int fedfem_set_dt(fedfem_handle *h, double dt);

/*
 * Use a caller-owned HIP stream (e.g. a torch stream, passed as its
 * hipStream_t); NULL returns to the handle's own stream.  The stream must
 * outlive its use by the handle.
 */
int fedfem_set_stream(fedfem_handle *h, void *stream);

/*
 * Raw state for checkpoints.  fedfem_state_bytes gives the size of the
 * state buffer: FP32C stores hi[n] then lo[n] (float), FP64 stores T[n]
 * (double), in the caller's node order.  Reading then writing the same
 * buffer restores the state bit for bit.
 */
int fedfem_state_bytes(const fedfem_handle *h, size_t *bytes);
int fedfem_read_state(fedfem_handle *h, void *buf, double *t, int64_t *steps);
int fedfem_write_state(fedfem_handle *h, const void *buf, double t,
                       int64_t steps);

/* Layout sizes and estimator results (after fedfem_precompute). */
int fedfem_get_info(const fedfem_handle *h, fedfem_info *info);

/*
 * Profiling aid: the mean duration [ms] of the element-load kernel and of
 * the node-update kernel of one step, each launched n_steps times back to
 * back between two HIP events on the handle's stream, every launch from the
 * current state (the element pass rewrites the tile partials, the node pass
 * the other ping-pong buffer, and a thermal dose goes to a staging buffer).
 * The state, the clock, the step count and the dose do not change.
 * FEDFEM_E_STATE while a source schedule is set (the amplitudes are applied
 * per graph chunk by fedfem_step only).
 */
int fedfem_time_kernels(fedfem_handle *h, int64_t n_steps, double *elem_ms,
                        double *node_ms);

/* Release all host and device resources of h (NULL is accepted). */
int fedfem_destroy(fedfem_handle *h);

/* Text for a return code, and the handle's last error message. */
const char *fedfem_strerror(int code);

/*
 * Device blocks freed by destroyed handles and batches are kept by the
 * library for reuse (per device and size class, up to FEDFEM_DEVICE_CACHE_MB
 * megabytes, default 16384; 0 disables the cache).  This returns every
 * cached block to the device and gives the number of bytes released.
 * Thread-safe.
 */
size_t fedfem_release_cached_memory(void);
int fedfem_last_error(const fedfem_handle *h, char *buf, size_t len);

/* ---- batched execution ------------------------------------------------- */
/*
 * Many independent scenarios (Algorithm 1 applied to each) advanced by one
 * graph-captured launch sequence.  The handles must be precomputed, share
 * one precision, and stay alive while the batch exists.  A batch copies
 * their pre-computed layouts once; each run takes every handle's current
 * state and active source, advances scenario j by n_steps[j] steps, and
 * writes the states back to the handles (read them with fedfem_read_T).
 * sources may be NULL; else sources[j], when non-NULL, is a nodal heat flow
 * [W] for scenario j (its caller's numbering) that replaces that handle's
 * active source before the run, as the source argument of fedfem_step does
 * (FEDFEM_E_INVALID if any is not finite; no source is replaced and no
 * scenario advances then).  fedfem_batch_create refuses hexahedral handles
 * and handles with a source schedule or a dose model (FEDFEM_E_STATE);
 * fedfem_batch_run gives FEDFEM_E_STATE, advancing nothing, when a
 * schedule or dose model was set on a member handle after creation.
 */
typedef struct fedfem_batch fedfem_batch;

int fedfem_batch_create(fedfem_handle *const *handles, int32_t n,
                        fedfem_batch **out);
int fedfem_batch_run(fedfem_batch *b, const int64_t *n_steps,
                     const double *const *sources);
/* Mean device time [ms] of the last fedfem_batch_run's launch sequence. */
int fedfem_batch_last_ms(const fedfem_batch *b, double *ms);
int fedfem_batch_destroy(fedfem_batch *b);

#ifdef __cplusplus
}
#endif

#endif /* FEDFEM_H */
