/*
 * zi.h -- C-ABI of the MI355X lead-field library (libzi.so).
 *
 * The library builds the EEG lead field of a finite-element head model with
 * the complete electrode model (CEM):
 *
 *   zi_assemble        the grounded stiffness/CEM system of Eq. (u_system)
 *                      (App. A.1): matrices A, B and C;
 *   zi_transfer_solve  the transfer matrix T = A^-1 B (App. A.4) by a
 *                      diagonally preconditioned conjugate gradient run on all
 *                      electrode columns at once (Sec. 2.3.1);
 *   zi_leadfield       L = R (B^T T - C)^-1 T^T G (App. A.2, Eq. (aku)).
 *
 * Conventions
 *   - Array pointers are DEVICE pointers owned by the caller unless marked
 *     HOST.  Matrices are row-major.  Indices are 0-based int32.
 *   - SI units: metres, S/m, Ohm; a lead-field column is the electrode
 *     voltage (V) for a unit (1 A m) dipole.
 *   - Every call enqueues its work on `hip_stream` (a hipStream_t; NULL is
 *     the default stream) and synchronises that stream before returning, so
 *     the status and statistics are final when the call returns.
 *   - No exception crosses the ABI; the return value is the status and
 *     zi_last_error() holds a message for the calling thread.
 *   - On ZI_EINVAL and ZI_EMESH no caller-visible output is written.
 *   - A zi_system is not thread-safe; distinct systems may be used from
 *     distinct threads on distinct streams.
 *   - Nodes are never reordered: row i of T is node i.
 */
#ifndef ZI_H
#define ZI_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct zi_system zi_system; /* opaque, owned by the library */

typedef enum {
    ZI_OK = 0,
    ZI_EINVAL = -1,      /* bad argument (size, pointer, option, ground node) */
    ZI_EMESH = -2,       /* invalid mesh or electrode data */
    ZI_ENOMEM = -3,      /* device allocation failed */
    ZI_EDEVICE = -4,     /* HIP runtime error */
    ZI_ENOTCONV = -5,    /* PCG reached maxit before the tolerance */
    ZI_EBREAKDOWN = -6   /* p^T A p <= 0 or a non-positive Cholesky pivot */
} zi_status;

/* Mesh (Sec. 2 "Conductivity distribution"; Sec. 2.4.2 fields nodes/tetra).
 *   nodes  n_nodes x 3 float64, metres.
 *   tets   n_tets x 4 int32; vertices distinct; either orientation.
 *   sigma  n_tets float64 (sigma_ncomp = 1, isotropic) or n_tets x 6
 *          (sigma_ncomp = 6: s11, s22, s33, s12, s13, s23 per element, the
 *          row layout of Sec. 2 "Conductivity distribution"), S/m; each
 *          element's conductivity must be positive (definite).
 * Errors: ZI_EMESH for an index out of range, repeated vertices, a
 * degenerate tetrahedron (|det J| <= 1e-12 * (longest edge)^3), a
 * non-positive or non-finite conductivity, a non-finite coordinate, or a node
 * that touches more than 127 distinct neighbours. */
typedef struct {
    int32_t n_nodes;
    int32_t n_tets;
    int32_t sigma_ncomp;
    const double *nodes;
    const int32_t *tets;
    const double *sigma;
} zi_mesh;

/* Electrodes of the complete electrode model (App. A.1, conditions I-III).
 *   tris           n_tris x 3 int32: triangles of the electrode patches e_l;
 *                  each must be a boundary face (a face of exactly one tet).
 *   tri_electrode  n_tris int32 in [0, n_electrodes); every electrode needs
 *                  at least one triangle.
 *   Z              HOST, n_electrodes float64: contact impedance Z_l > 0, Ohm.
 * The contact area calA_l is the summed area of electrode l's triangles. */
typedef struct {
    int32_t n_electrodes;
    int32_t n_tris;
    const int32_t *tris;
    const int32_t *tri_electrode;
    const double *Z;
} zi_electrodes;

enum { ZI_PREC_JACOBI = 0, /* D_ii = a_ii */
       ZI_PREC_LDP = 1     /* lumped diagonal D_ii = sum_j |a_ij| (Sec. 2.3.1) */ };

enum { ZI_FP64 = 0,         /* all arithmetic in float64 */
       ZI_FP32_SPMM_IR = 1  /* float32 search directions and products (float64
                               matrix values, float64 sums) inside float64 PCG
                               recurrences; the recurrence residual is replaced
                               by the float64 true residual every 64 iterations,
                               and columns whose true residual misses tol at the
                               end restart (float64 iterative refinement) */ };

/* Form of the PCG iteration (Sec. 2.3.1 solves with Jacobi-preconditioned
 * CG; both forms give the same iterates in exact arithmetic). */
enum { ZI_PCG_AUTO = 0,       /* single-reduction in ZI_FP64, classic in
                                 ZI_FP32_SPMM_IR */
       ZI_PCG_CLASSIC = 1,    /* two reductions per iteration (p.Ap, then
                                 r.D^-1 r); every search direction is formed,
                                 x is updated every 16 iterations */
       ZI_PCG_SINGLE = 2      /* single-reduction form of Chronopoulos and Gear:
                                 s = A D^-1 r + beta s by recurrence, the search
                                 directions are formed lazily beside x every 16
                                 iterations; ZI_FP64 only */ };

/* Options of zi_transfer_solve.  Zero-initialised fields take defaults. */
typedef struct {
    double tol;          /* relative residual ||b - A t|| / ||b|| target;
                            0 -> 1e-8 */
    int32_t maxit;       /* iteration limit per column; 0 -> 50000 */
    int32_t precond;     /* ZI_PREC_JACOBI or ZI_PREC_LDP */
    int32_t precision;   /* ZI_FP64 or ZI_FP32_SPMM_IR */
    int32_t check_every; /* iterations between host convergence checks; 0 -> 8;
                            rounded up to a multiple of 8, and of 16 when the
                            iterations are replayed as graphs (graph = 1 and
                            every batch); in ZI_FP32_SPMM_IR further up to a
                            power of two that divides 64 */
    int32_t timing;      /* 1: time the solver kernels with HIP events
                            (the SpMM and updates of every 8th
                            iteration, and every full flush) */
    int32_t tile;        /* SpMM tile id (see zi_tile_count); -1 -> the tile
                            zi_autotune chose, else a width-based default */
    int32_t graph;       /* 1: replay the iteration loop as a hipGraph of
                            check_every iterations (no per-kernel timing) */
    const double *x0;    /* n_nodes x L initial iterate, or NULL for zero */
    const int32_t *columns; /* HOST, optional: solve only these electrode
                               columns (distinct, in [0, L)); T, x0 and the
                               statistics then have n_columns columns */
    int32_t n_columns;
    int32_t form;        /* ZI_PCG_AUTO, ZI_PCG_CLASSIC or ZI_PCG_SINGLE
                            (ZI_PCG_SINGLE with ZI_FP32_SPMM_IR: ZI_EINVAL) */
    double refine_eta;   /* ZI_FP32_SPMM_IR: each float32 cycle stops once it has
                            reduced its starting residual by this factor (or
                            reached tol), then an FP64 refinement step restarts
                            the columns that miss tol; 0 -> run every cycle to
                            tol.  In [0, 1), else ZI_EINVAL; ignored in ZI_FP64 */
} zi_solve_opts;

/* Statistics of zi_transfer_solve.  The HOST arrays are caller-owned, length
 * n_electrodes, and may be NULL. */
typedef struct {
    int32_t *iters;        /* HOST: PCG updates done per column */
    double *relres_rec;    /* HOST: recurrence ||r||/||b|| at exit */
    double *relres_true;   /* HOST: ||b - A t||/||b|| recomputed at exit */
    double seconds;        /* wall time of the call */
    int32_t block_iters;   /* iterations of the multi-column loop */
    int32_t refinements;   /* outer refinement steps (ZI_FP32_SPMM_IR) */
    int32_t tile;          /* SpMM tile used */
    int32_t n_kernels;     /* entries used in the arrays below */
    double kernel_ms[8];   /* total event-timed ms per solver kernel */
    int32_t kernel_launches[8]; /* launches timed (the sample above) */
    int64_t kernel_bytes[8]; /* algorithmic bytes of one launch */
    const char *kernel_name[8];
    int32_t kernel_calls[8];   /* launches in the solve (timed or not) */
} zi_solve_stats;

/* Assemble the grounded CEM system of Eq. (u_system).
 *   a_ij = int sigma grad psi_i . grad psi_j + sum_l 1/(Z_l calA_l) int_{e_l} psi_i psi_j
 *   b_il = 1/(Z_l calA_l) int_{e_l} psi_i,   c_ll = 1/Z_l
 * then the ground fix of App. A.1: row and column i' of A are zeroed and
 * a_{i'i'} = 1.  ground_node = -1 selects the smallest boundary node that is
 * not a vertex of any electrode triangle; otherwise the given node must be
 * such a node (ZI_EINVAL if not).
 * The CSR structure of A is the mesh graph (all pairs sharing a tet,
 * diagonal included, columns ascending, zero values kept).
 * *out receives a new system (caller destroys it with zi_system_destroy). */
zi_status zi_assemble(const zi_mesh *mesh, const zi_electrodes *el,
                      int32_t ground_node, void *hip_stream, zi_system **out);

/* T = A^-1 B (App. A.4): PCG of Sec. 2.3.1 on every electrode column (or the
 * opts->columns subset), from x0 (or 0) until ||r||_2 <= tol ||b||_2 per
 * column.
 *   T      n_nodes x n_electrodes (or n_columns) float64, written on ZI_OK and ZI_ENOTCONV
 *          (then it holds the last iterate).
 *   stats  may be NULL.
 * ZI_ENOTCONV if a column misses the tolerance within maxit iterations;
 * ZI_EBREAKDOWN if p^T A p <= 0 (A not positive definite). */
zi_status zi_transfer_solve(zi_system *sys, const zi_solve_opts *opts, double *T,
                            zi_solve_stats *stats, void *hip_stream);

/* Transfer matrices of several systems (e.g. many head models) at once.
 * Each system runs exactly the iteration of zi_transfer_solve; the
 * iterations of the systems that are still active are captured into hipGraphs
 * (one per group of eight systems, one branch per system, check_every
 * iterations per replay; a group is captured again when one of its systems
 * finishes) that are replayed until every system has converged.  opts applies to every system
 * (x0 must be NULL); T[k] is n_nodes(k) x L(k); stats may be NULL or an array
 * of n_systems.  Returns the first non-OK status of the systems (all T are
 * written). */
zi_status zi_transfer_solve_batch(zi_system *const *systems, int32_t n_systems,
                                  const zi_solve_opts *opts, double *const *T,
                                  zi_solve_stats *stats, void *hip_stream);

/* Autotuner: scores every tile by the SpMM of one PCG iteration on this
 * system's n x L block in the given precision and stores the best; later
 * solves with tile = -1 use it.  ZI_FP64 times the single-reduction SpMM
 * S = A D^-1 R + beta S, ZI_FP32_SPMM_IR the classic SpMM Q = A P with
 * float32 vectors; the residual and direction updates and the flushes run
 * with one fixed geometry whatever the tile, and no tile changes a result
 * bit.  Each tile: the best of three launches after a warm-up.  The
 * workspace's contents are overwritten.  best_tile (HOST, may be NULL)
 * receives the choice; ms (HOST, may be NULL, zi_tile_count() entries) the
 * milliseconds per tile. */
zi_status zi_autotune(zi_system *sys, int32_t precision, int32_t *best_tile, double *ms,
                      void *hip_stream);

/* EEG lead field of App. A.2, Eq. (aku): LF = R (B^T T - C)^-1 T^T G.
 *   T        n_nodes x L float64 from zi_transfer_solve.
 *   G        n_nodes x n_cols in CSC form: g_colptr (n_cols + 1), g_rowind
 *            and g_val (g_colptr[n_cols] entries); the source matrix of
 *            App. A.1 (entries g_ij = int psi_i div w_j).
 *   LF       L x n_cols float64, row-major (electrode-major).  n_cols may be
 *            0: nothing is written, and LF and G's arrays may be NULL.
 *   precision ZI_FP64, or 1 for float32 matrix-core products (T^T G and the
 *            final product rounded to float32 inputs, float32 accumulation).
 * ZI_EBREAKDOWN if M = C - B^T T is not positive definite. */
zi_status zi_leadfield(const zi_system *sys, const double *T, int32_t n_cols,
                       const int32_t *g_colptr, const int32_t *g_rowind,
                       const double *g_val, double *LF, int32_t precision,
                       void *hip_stream);

/* zi_leadfield without device allocation, for callers that cannot allocate
 * device memory (code under HIP graph capture, serving loops, harnesses that
 * forbid hipMalloc).  Same arguments, result and errors as zi_leadfield; the
 * lead field is the same to the bit.
 *   Workspace: a fixed 16 MiB array per device, set up on the first call on
 *   that device and held until the process ends.  It holds the four L x L
 *   matrices of the Schur step and Pt for zi_leadfield_noalloc_max_cols(L)
 *   columns of G at a time; longer G are processed in column chunks.
 *   Limits: L <= 256 (ZI_EINVAL otherwise), any n_cols.
 *   Calls that overlap on one device share the array and race: serialise
 *   them (one stream, or one call at a time per device).
 *   No hipMalloc, hipFree or allocating library routine is called. */
zi_status zi_leadfield_noalloc(const zi_system *sys, const double *T, int32_t n_cols,
                               const int32_t *g_colptr, const int32_t *g_rowind,
                               const double *g_val, double *LF, int32_t precision,
                               void *hip_stream);

/* Columns of G per chunk in zi_leadfield_noalloc for L electrodes (0 if L is
 * outside [1, 256]). */
int64_t zi_leadfield_noalloc_max_cols(int32_t n_electrodes);

/* Source matrix of point dipoles (Sec. 2 "Primary current model", read as
 * the partial-integration dipole): a unit dipole along axis k at the centroid
 * of tet d gives column 3 j + k with G[i, 3 j + k] = -d psi_i / d x_k on that
 * tet, for the j-th entry d of dipole_tets (columns ordered position 1 xyz,
 * position 2 xyz, ... as in Sec. 2.4.2).
 *   dipole_tets  m int32 tet indices.
 *   g_colptr     3 m + 1 int32 (output), g_rowind and g_val 12 m (output);
 *                row indices ascending within a column. */
zi_status zi_point_dipoles(const zi_system *sys, int32_t m, const int32_t *dipole_tets,
                           int32_t *g_colptr, int32_t *g_rowind, double *g_val,
                           void *hip_stream);

/* Source matrix of the linearized EIT lead field (App. A.3).
 * With current patterns I (HOST, L x n_patterns row-major; every pattern must
 * sum to zero, the grounding condition of App. A.1), M = C - B^T T and
 * U = T M^-1 I, column p * n_elems + j of the output CSC matrix holds
 * K1_m U[:, p] on the four vertices of tet m = elems[j] (ascending rows),
 * where K1_m = dA/ds_m is the element stiffness matrix of tet m for unit
 * conductivity.  zi_leadfield(sys, T, n_patterns * n_elems, <this G>, ...)
 * then returns dy/ds_m = -R M^-1 T^T K1_m U, the linearized EIT lead field.
 *   T         n_nodes x L from zi_transfer_solve.
 *   elems     n_elems int32 tet indices (device), or NULL for every tet
 *             (n_elems must then equal n_tets).
 *   g_colptr  n_patterns * n_elems + 1; g_rowind, g_val 4 * n_patterns * n_elems.
 *   y_bg      HOST L x n_patterns (may be NULL): background data R M^-1 I.
 * ZI_EINVAL for an index out of range or a pattern not summing to zero;
 * ZI_EBREAKDOWN if M is not positive definite. */
zi_status zi_eit_source(const zi_system *sys, const double *T, int32_t n_patterns,
                        const double *I, int32_t n_elems, const int32_t *elems,
                        int32_t *g_colptr, int32_t *g_rowind, double *g_val, double *y_bg,
                        void *hip_stream);

/* Y = A X for the assembled (grounded) A; X and Y are n_nodes x k row-major,
 * k even.  The product the PCG iterates (the solver's copy of A, see
 * zi_system_info.nnz_solver); exposed for tests and bandwidth measurement.
 * tile as in zi_solve_opts, except the LDS ring tile (ZI_EINVAL).  ms_out
 * (HOST, may be NULL) receives the event-timed kernel duration. */
zi_status zi_spmm(const zi_system *sys, int32_t k, const double *X, double *Y,
                  int32_t tile, double *ms_out, void *hip_stream);

/* ---- Learned PCG initial iterates: a mesh-graph network ------------------
 * A K-layer network on the mesh graph of an assembled system (its CSR
 * structure), with the symmetric normalised aggregation
 * Ahat = D^-1/2 Adj D^-1/2.  Layer k maps H_k (n x dims[k]) to
 * relu(H_k Ws_k + (Ahat^h_k H_k) Wn_k + b_k) (no relu on the last layer, h_k
 * aggregation hops, 1 when hops is NULL); the
 * prediction is column 0 of H_K.  float32 throughout; weight gradients are
 * reduced in float64 in a fixed order.  The network only proposes x0 for
 * zi_transfer_solve; the PCG always finishes to its tolerance.
 * Parameter layout (flat float32): for k = 0..K-1, Ws_k (dims[k] x
 * dims[k+1], row-major), Wn_k (same), b_k (dims[k+1]).  dims[k] for k < K
 * must be even and <= 64; dims[K] <= 64. */
typedef struct zi_gnn zi_gnn;
zi_status zi_gnn_create(const zi_system *sys, int32_t n_layers, const int32_t *dims /* HOST */,
                        const int32_t *hops /* HOST, n_layers entries in 1..1024, or NULL */,
                        zi_gnn **out);
int64_t zi_gnn_param_count(const zi_gnn *net);
/* Parameters from / to HOST memory (setting resets the Adam moments). */
zi_status zi_gnn_set_params(zi_gnn *net, const float *params);
zi_status zi_gnn_get_params(const zi_gnn *net, float *params);
/* y (n_nodes) = prediction for features X (n_nodes x dims[0], row-major). */
zi_status zi_gnn_forward(zi_gnn *net, const float *X, float *y, void *hip_stream);
/* Forward, loss sum (y - t)^2 / sum t^2 (HOST *loss) and backward; the
 * gradients stay on the device for zi_gnn_adam_step and are also copied to
 * grads (HOST, zi_gnn_param_count entries) when it is not NULL. */
zi_status zi_gnn_loss_grad(zi_gnn *net, const float *X, const float *t, double *loss,
                           float *grads, void *hip_stream);
/* One Adam step (beta1 0.9, beta2 0.999, eps 1e-8) with the last gradients. */
zi_status zi_gnn_adam_step(zi_gnn *net, float lr, void *hip_stream);
void zi_gnn_destroy(zi_gnn *net);
/* Input features of the warm-start network for electrode column l of a head
 * whose conductivity differs from a base head's (same mesh, same electrodes):
 * X (n_nodes x 10 float32, row-major), per node i,
 *   0  b_il / max_i |b_il|              (the right-hand side, App. A.4)
 *   1  log(a_ii / a0_ii)                (the conductivity change seen by node i)
 *   2  t0_il / max_i |t0_il|            (the base head's transfer column)
 *   3-5 x_i / radius
 *   6  |x_i - centre| / radius          (distance to electrode l's centre)
 *   7  log(a0_ii / max_j a0_jj)         (the base conductivity, a compartment mark)
 *   8  r_i / max_i |r_i|, r = b_l - A t0_l   (the residual of t0 for this head)
 *   9  1                               (a constant input)
 * a and a0 the grounded matrices of `perturbed` and `base`; T0 the base
 * transfer matrix (device, n_nodes x ldt, ldt >= L); centre HOST double[3].
 * ZI_EINVAL for a different mesh or an electrode out of range. */
zi_status zi_gnn_features(const zi_system *base, const zi_system *perturbed, const double *T0,
                          int32_t ldt, int32_t electrode, const double *centre, double radius,
                          float *X, void *hip_stream);
/* Training target of the warm-start network for electrode l: with
 * s_l = max_i |t0_il|, t_i = gain (T[i, col] - T0[i, l]) / s_l (n_nodes
 * float32).  T (n_nodes x ldT) holds the head's transfer column col, T0 the
 * base transfer matrix (n_nodes x ldt).  *sumsq (HOST, may be NULL) receives
 * sum_i t_i^2. */
zi_status zi_gnn_target(const double *T, int32_t ldT, int32_t col, const double *T0,
                        int32_t ldt, int32_t electrode, double gain, int32_t n_nodes, float *t,
                        double *sumsq, void *hip_stream);
/* The proposed initial iterate from a prediction y (n_nodes float32, the
 * network's output for the features of electrode l):
 * x0[i * ldx + xcol] = T0[i, l] + s_l y_i / gain. */
zi_status zi_gnn_x0(const float *y, const double *T0, int32_t ldt, int32_t electrode,
                    double gain, int32_t n_nodes, double *x0, int32_t ldx, int32_t xcol,
                    void *hip_stream);

/* Measurement aid: copies n float64 values (n even, 16-byte aligned) from
 * src to dst with the 16-byte streaming accesses of the solver kernels and
 * returns the event-timed kernel milliseconds in *ms (HOST, may be NULL).
 * Used as the plain copy of known size that calibrates HBM counters. */
zi_status zi_copy_probe(const double *src, double *dst, int64_t n, double *ms, void *hip_stream);

/* Number of SpMM tile configurations and a description of tile t:
 * lpr<lanes per row>_nv<column pairs per lane>_cw<chunk width>, with _front
 * for the cooperative-front schedule, or ring_g<rows per step>_cw<chunk
 * width> for the LDS ring SpMM of the solver (16 columns of FP64 vectors, 32
 * of float32 ones, per chunk; not for zi_spmm). */
int32_t zi_tile_count(void);
const char *zi_tile_name(int32_t t);

typedef struct {
    int32_t n_nodes, n_tets, n_electrodes, ground_node;
    int64_t nnz;        /* entries of the mesh-graph CSR of A */
    int32_t b_nnz;      /* nonzeros of B */
    int64_t nnz_solver; /* entries the solver streams: A without the
                           off-diagonal entries |a_ij| <= 64 eps sqrt(a_ii a_jj),
                           which lie below the assembly's own rounding error */
} zi_system_info;

/* Device views of the assembled system, valid until zi_system_destroy.
 * Read-only; for tests. */
typedef struct {
    const int32_t *row_ptr;  /* n + 1 */
    const int32_t *col;      /* nnz */
    const double *val;       /* nnz, grounded A */
    const int32_t *b_ptr;    /* n + 1: node-major B (row i: electrodes) */
    const int32_t *b_col;    /* b_nnz electrode indices, ascending per row */
    const double *b_val;     /* b_nnz */
    const double *C;         /* L: c_ll */
    const double *calA;      /* L: contact areas */
    const uint8_t *boundary; /* n: 1 if the node lies on a boundary face */
} zi_system_view;

zi_status zi_get_info(const zi_system *sys, zi_system_info *info);
zi_status zi_get_view(const zi_system *sys, zi_system_view *view);

/* Destroys a system.  Its device arrays and solver workspace go back to a
 * process-wide cache of the library (the devices are synchronised first, as
 * hipFree would), from which later zi_assemble and zi_transfer_solve calls
 * take blocks of the same rounded size; what would take the cache beyond a
 * quarter of the device's memory is freed at once. */
void zi_system_destroy(zi_system *sys);

/* Frees every device block held by the library's cache.  Returns ZI_OK. */
zi_status zi_release_cached_memory(void);
const char *zi_status_string(zi_status s);
const char *zi_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* ZI_H */
