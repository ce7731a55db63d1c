// Internal declarations shared by the HIP sources of libzi.
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <vector>

#include "../../include/zi.h"

namespace zi {

void set_error(const char *fmt, ...);
bool g_err_empty();

#define ZI_HIP(call)                                                              \
    do {                                                                          \
        hipError_t zi_e_ = (call);                                                \
        if (zi_e_ != hipSuccess) {                                                \
            ::zi::set_error("%s failed: %s (%s:%d)", #call,                       \
                            hipGetErrorString(zi_e_), __FILE__, __LINE__);        \
            return zi_e_ == hipErrorOutOfMemory ? ZI_ENOMEM : ZI_EDEVICE;         \
        }                                                                         \
    } while (0)

#define ZI_TRY(expr)                                                              \
    do {                                                                          \
        zi_status zi_s_ = (expr);                                                 \
        if (zi_s_ != ZI_OK) return zi_s_;                                         \
    } while (0)

// Validation flags raised by kernels (bitwise OR into a device word).
enum : int {
    F_TET_INDEX = 1 << 0,     // vertex index out of range or repeated
    F_SIGMA = 1 << 1,         // conductivity not positive (definite) / finite
    F_COORD = 1 << 2,         // non-finite node coordinate
    F_DEGENERATE = 1 << 3,    // |det J| too small
    F_TRI_INDEX = 1 << 4,     // electrode triangle index out of range / repeated
    F_TRI_ELECTRODE = 1 << 5, // tri_electrode out of range
    F_TRI_NOT_FACE = 1 << 6,  // electrode triangle is not a boundary face
    F_DEGREE = 1 << 7,        // node with more than MAX_NEIGHBOURS neighbours
    F_EMPTY_ELECTRODE = 1 << 8,
    F_DIPOLE_INDEX = 1 << 9,
};

constexpr int MAX_NEIGHBOURS = 128;   // distinct CSR columns per row (incl. diagonal)

// Process-wide cache of device blocks (k_util.hip).  Long-lived pools (a
// system's arrays and its solver workspace) return their blocks here when they
// are released instead of freeing them, and take blocks of the same rounded
// size from here first, so that building one system after another does not
// pay for hipMalloc / hipFree (which unmaps and synchronises) every time.
size_t cache_round(size_t bytes);
void *cache_take(size_t bytes, int dev);
bool cache_put(void *p, size_t bytes, int dev);   // false: over the cap, caller frees
zi_status cache_clear();

// Owned device allocation list: everything allocated through a Pool is freed
// by release() (or, for a cached pool, returned to the cache).  A cached pool
// synchronises its devices before handing its blocks back, as hipFree would.
struct Pool {
    struct Blk {
        void *p;
        size_t bytes;
        int dev;
    };
    std::vector<Blk> blks;
    bool cached = false;
    template <class T>
    zi_status alloc(T **p, size_t count) {
        *p = nullptr;
        if (count == 0) count = 1;
        size_t bytes = count * sizeof(T);
        int dev = 0;
        (void)hipGetDevice(&dev);
        void *q = nullptr;
        if (cached) {
            bytes = cache_round(bytes);
            q = cache_take(bytes, dev);
        }
        if (!q) {
            hipError_t e = hipMalloc(&q, bytes);
            if (e == hipErrorOutOfMemory) {   // idle cached blocks may be in the way
                (void)hipGetLastError();
                (void)cache_clear();
                e = hipMalloc(&q, bytes);
            }
            if (e != hipSuccess) {
                (void)hipGetLastError();
                set_error("hipMalloc of %zu bytes failed: %s", bytes, hipGetErrorString(e));
                return e == hipErrorOutOfMemory ? ZI_ENOMEM : ZI_EDEVICE;
            }
        }
        blks.push_back({q, bytes, dev});
        *p = static_cast<T *>(q);
        return ZI_OK;
    }
    void release() {
        if (cached && !blks.empty()) {
            int cur = 0;
            (void)hipGetDevice(&cur);
            std::vector<int> devs;
            for (const Blk &b : blks) {
                bool seen = false;
                for (int d : devs) seen = seen || d == b.dev;
                if (!seen) devs.push_back(b.dev);
            }
            for (int d : devs) {
                (void)hipSetDevice(d);
                (void)hipDeviceSynchronize();
            }
            (void)hipSetDevice(cur);
        }
        for (const Blk &b : blks)
            if (!(cached && cache_put(b.p, b.bytes, b.dev))) (void)hipFree(b.p);
        blks.clear();
    }
    ~Pool() { release(); }
};

// ---------------------------------------------------------------------------
// Generic device utilities (k_util.hip)
// ---------------------------------------------------------------------------

// Exclusive scan of `count` int32 values: out[0..count], out[count] = total.
// `out` may not alias `in`.  Temporaries come from `pool`.
zi_status scan_exclusive(const int32_t *in, int32_t *out, int32_t count, Pool &pool,
                         hipStream_t s);

// Bucket the items k = 0..n_items-1 by keys[k] in [0, n_buckets): ptr gets
// n_buckets + 1 offsets and items the item ids grouped by bucket, ascending
// inside each bucket when `sort` is true.  Keys must be in range.
zi_status bucketize(const int32_t *keys, int32_t n_items, int32_t n_buckets,
                    int32_t *ptr, int32_t *items, bool sort, Pool &pool, hipStream_t s);

zi_status fill_i32(int32_t *p, int32_t value, size_t count, hipStream_t s);
zi_status spmm_f32(const int32_t *rp, const int32_t *ci, const float *va, const float *X, float *Y,
                   int32_t n, int32_t ld, hipStream_t s);
zi_status fill_f64(double *p, double value, size_t count, hipStream_t s);
zi_status copy_probe(const double *src, double *dst, size_t n, double *ms, hipStream_t s);
zi_status copy_cols(const double *src, int32_t lds, double *dst, int32_t ldd,
                    int32_t rows, int32_t cols, hipStream_t s);
// dst[r * ldd + c] = src[rows[r] * lds + c] for r < n, c < cols.
zi_status gather_rows(const double *src, int32_t lds, const int32_t *rows, double *dst,
                      int32_t ldd, int32_t n, int32_t cols, hipStream_t s);

}  // namespace zi

// ---------------------------------------------------------------------------
// The assembled system
// ---------------------------------------------------------------------------

struct zi_solver_ws;   // PCG workspace (k_pcg.hip)

struct zi_system {
    int32_t n = 0, e = 0, L = 0, ntris = 0, ncomp = 1;
    int32_t ground = -1;
    int64_t nnz = 0;
    int32_t b_nnz = 0;
    int device = 0;

    // copies of the inputs the later stages need
    double *nodes = nullptr;     // n x 3
    int32_t *tets = nullptr;     // e x 4
    double *sigma = nullptr;     // e x ncomp

    // A: mesh-graph CSR, grounded values
    int32_t *row_ptr = nullptr, *col = nullptr;
    double *val = nullptr;
    // the solver's copy of A: off-diagonal entries below 64 eps sqrt(a_ii a_jj)
    // (rounding residue of couplings that vanish in exact arithmetic) left out,
    // rows and columns in the solver's locality order: solver row r is node
    // perm[r], node i is solver row iperm[i]
    int32_t *perm = nullptr, *iperm = nullptr;
    int32_t *sp_ptr = nullptr, *sp_col = nullptr;
    double *sp_val = nullptr;
    int64_t sp_nnz = 0;
    double *diag = nullptr;      // a_ii
    double *absrow = nullptr;    // sum_j |a_ij|

    // B node-major (row i -> electrodes) and electrode-major (l -> entries)
    int32_t *b_ptr = nullptr, *b_col = nullptr, *b_row = nullptr;
    double *b_val = nullptr;
    int32_t *e_ptr = nullptr, *e_item = nullptr;
    double *C = nullptr, *calA = nullptr;
    uint8_t *boundary = nullptr;

    // lead-field scratch
    double *W = nullptr;         // L x L
    double *Pt = nullptr;        // n_cols x L (grows)
    size_t Pt_cap = 0;

    int32_t *colmap = nullptr;   // electrode -> solved column for column subsets

    // halo lists of the ring SpMM tile (built on first use)
    int32_t *ring_halo = nullptr;

    // SpMM tile chosen by zi_autotune per precision (for that ldp)
    int32_t tuned_tile[2] = {-1, -1};
    int32_t tuned_ldp[2] = {0, 0};

    zi::Pool pool;               // owns every array above
    zi_solver_ws *ws = nullptr;  // lazily created
};

// Stage entry points (defined in the .hip files).
zi_status zi_assemble_impl(const zi_mesh *mesh, const zi_electrodes *el, int32_t ground,
                           hipStream_t s, zi_system **out);
zi_status zi_solve_impl(zi_system *sys, const zi_solve_opts *opts, double *T,
                        zi_solve_stats *stats, hipStream_t s);
zi_status zi_solve_batch_impl(zi_system *const *systems, int32_t nsys, const zi_solve_opts *o,
                              double *const *T, zi_solve_stats *st, hipStream_t s);
zi_status zi_autotune_impl(zi_system *sys, int32_t precision, int32_t *best, double *ms_out,
                           hipStream_t s);
zi_status zi_spmm_impl(const zi_system *sys, int32_t k, const double *X, double *Y,
                       int32_t tile, double *ms, hipStream_t s);
zi_status zi_leadfield_impl(const zi_system *sys, const double *T, int32_t n_cols,
                            const int32_t *cp, const int32_t *ri, const double *gv,
                            double *LF, int32_t precision, hipStream_t s);
zi_status zi_leadfield_noalloc_impl(const zi_system *sys, const double *T, int32_t n_cols,
                                    const int32_t *cp, const int32_t *ri, const double *gv,
                                    double *LF, int32_t precision, hipStream_t s);
int64_t zi_leadfield_noalloc_max_cols_impl(int32_t L);
zi_status zi_point_dipoles_impl(const zi_system *sys, int32_t m, const int32_t *dt,
                                int32_t *cp, int32_t *ri, double *gv, hipStream_t s);
zi_status zi_eit_columns_impl(const zi_system *sys, const double *U, int32_t P, int32_t ne,
                              const int32_t *elems, int32_t *cp, int32_t *ri, double *gv,
                              hipStream_t s);
zi_status zi_eit_source_impl(const zi_system *sys, const double *T, int32_t P, const double *I,
                             int32_t ne, const int32_t *elems, int32_t *cp, int32_t *ri,
                             double *gv, double *y_bg, hipStream_t s);
void zi_solver_ws_destroy(zi_solver_ws *ws);
zi_status zi_gnn_create_impl(const zi_system *sys, int32_t K, const int32_t *dims,
                             const int32_t *hops, zi_gnn **out);
zi_status zi_gnn_features_impl(const zi_system *base, const zi_system *pert, const double *T0,
                               int32_t ldt, int32_t l, const double *centre, double radius,
                               float *X, hipStream_t s);
zi_status zi_gnn_target_impl(const double *T, int32_t ldT, int32_t col, const double *T0,
                             int32_t ldt, int32_t l, double gain, int32_t n, float *t,
                             double *sumsq, hipStream_t s);
zi_status zi_gnn_x0_impl(const float *y, const double *T0, int32_t ldt, int32_t l, double gain,
                         int32_t n, double *x0, int32_t ldx, int32_t xcol, hipStream_t s);
void zi_gnn_destroy_impl(zi_gnn *g);
int64_t zi_gnn_param_count_impl(const zi_gnn *g);
zi_status zi_gnn_set_params_impl(zi_gnn *g, const float *p);
zi_status zi_gnn_get_params_impl(const zi_gnn *g, float *p);
zi_status zi_gnn_forward_impl(zi_gnn *g, const float *X, float *y, hipStream_t s);
zi_status zi_gnn_loss_grad_impl(zi_gnn *g, const float *X, const float *t, double *loss,
                                float *grads_host, hipStream_t s);
zi_status zi_gnn_adam_step_impl(zi_gnn *g, float lr, hipStream_t s);
int32_t zi_tile_count_impl();
const char *zi_tile_name_impl(int32_t t);
