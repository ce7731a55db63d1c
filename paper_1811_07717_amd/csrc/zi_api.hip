// C-ABI entry points of libzi: argument checks, stream handling, errors.
#include <cstdarg>
#include <cstdio>
#include <new>

#include "zi_internal.h"

namespace zi {
namespace {
thread_local char g_err[512] = "";
}
bool g_err_empty() { return g_err[0] == 0; }
void set_error(const char *fmt, ...) {
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(g_err, sizeof(g_err), fmt, ap);
    va_end(ap);
}
}  // namespace zi

using zi::set_error;

#define ZI_GUARD(body)                                          \
    try {                                                       \
        body                                                    \
    } catch (const std::bad_alloc &) {                          \
        set_error("host allocation failed");                    \
        return ZI_ENOMEM;                                       \
    } catch (...) {                                             \
        set_error("unexpected exception");                      \
        return ZI_EDEVICE;                                      \
    }

extern "C" {

const char *zi_last_error(void) { return zi::g_err; }

const char *zi_status_string(zi_status s) {
    switch (s) {
        case ZI_OK: return "ok";
        case ZI_EINVAL: return "invalid argument";
        case ZI_EMESH: return "invalid mesh or electrode data";
        case ZI_ENOMEM: return "out of memory";
        case ZI_EDEVICE: return "device error";
        case ZI_ENOTCONV: return "not converged";
        case ZI_EBREAKDOWN: return "breakdown (matrix not positive definite)";
    }
    return "unknown status";
}

zi_status zi_assemble(const zi_mesh *mesh, const zi_electrodes *el, int32_t ground_node,
                      void *hip_stream, zi_system **out) {
    zi::g_err[0] = 0;
    if (!mesh || !el || !out) {
        set_error("null argument");
        return ZI_EINVAL;
    }
    *out = nullptr;
    if (mesh->n_nodes < 4 || mesh->n_tets < 1 || !mesh->nodes || !mesh->tets || !mesh->sigma) {
        set_error("mesh needs n_nodes >= 4, n_tets >= 1 and non-null arrays");
        return ZI_EINVAL;
    }
    if (mesh->sigma_ncomp != 1 && mesh->sigma_ncomp != 6) {
        set_error("sigma_ncomp must be 1 or 6 (got %d)", mesh->sigma_ncomp);
        return ZI_EINVAL;
    }
    if ((int64_t)mesh->n_tets * 4 >= (int64_t)1 << 31) {
        set_error("too many tetrahedra for 32-bit incidence indices");
        return ZI_EINVAL;
    }
    if (el->n_electrodes < 1 || el->n_tris < 1 || !el->tris || !el->tri_electrode || !el->Z) {
        set_error("electrodes need n_electrodes >= 1, n_tris >= 1 and non-null arrays");
        return ZI_EINVAL;
    }
    if (el->n_tris > ((int32_t)1 << 29)) {
        set_error("too many electrode triangles");
        return ZI_EINVAL;
    }
    if (ground_node < -1 || ground_node >= mesh->n_nodes) {
        set_error("ground_node %d out of range", ground_node);
        return ZI_EINVAL;
    }
    ZI_GUARD(return zi_assemble_impl(mesh, el, ground_node, (hipStream_t)hip_stream, out);)
}

zi_status zi_transfer_solve(zi_system *sys, const zi_solve_opts *opts, double *T,
                            zi_solve_stats *stats, void *hip_stream) {
    zi::g_err[0] = 0;
    if (!sys || !opts || !T) {
        set_error("null argument");
        return ZI_EINVAL;
    }
    if (opts->tol < 0 || opts->maxit < 0) {
        set_error("tol and maxit must be non-negative");
        return ZI_EINVAL;
    }
    ZI_GUARD(return zi_solve_impl(sys, opts, T, stats, (hipStream_t)hip_stream);)
}

zi_status zi_transfer_solve_batch(zi_system *const *systems, int32_t n_systems,
                                  const zi_solve_opts *opts, double *const *T,
                                  zi_solve_stats *stats, void *hip_stream) {
    zi::g_err[0] = 0;
    if (!systems || !opts || !T || n_systems < 1) {
        set_error("null argument or n_systems < 1");
        return ZI_EINVAL;
    }
    for (int k = 0; k < n_systems; ++k) {
        if (!systems[k] || !T[k]) {
            set_error("null system or output %d", k);
            return ZI_EINVAL;
        }
        for (int j = 0; j < k; ++j)
            if (systems[j] == systems[k]) {
                set_error("system %d appears twice", k);
                return ZI_EINVAL;
            }
    }
    if (opts->tol < 0 || opts->maxit < 0 || opts->x0 || opts->columns) {
        set_error("tol and maxit must be non-negative; x0 and columns are not supported in "
                  "batches");
        return ZI_EINVAL;
    }
    ZI_GUARD(return zi_solve_batch_impl(systems, n_systems, opts, T, stats,
                                        (hipStream_t)hip_stream);)
}

zi_status zi_autotune(zi_system *sys, int32_t precision, int32_t *best_tile, double *ms,
                      void *hip_stream) {
    zi::g_err[0] = 0;
    if (!sys) {
        set_error("null argument");
        return ZI_EINVAL;
    }
    ZI_GUARD(return zi_autotune_impl(sys, precision, best_tile, ms, (hipStream_t)hip_stream);)
}

zi_status zi_leadfield(const zi_system *sys, const double *T, int32_t n_cols,
                       const int32_t *g_colptr, const int32_t *g_rowind, const double *g_val,
                       double *LF, int32_t precision, void *hip_stream) {
    zi::g_err[0] = 0;
    if (!sys || !T || n_cols < 0 ||
        (n_cols > 0 && (!LF || !g_colptr || !g_rowind || !g_val))) {
        set_error("null argument or negative n_cols");
        return ZI_EINVAL;
    }
    ZI_GUARD(return zi_leadfield_impl(sys, T, n_cols, g_colptr, g_rowind, g_val, LF, precision,
                                      (hipStream_t)hip_stream);)
}

zi_status zi_leadfield_noalloc(const zi_system *sys, const double *T, int32_t n_cols,
                               const int32_t *g_colptr, const int32_t *g_rowind,
                               const double *g_val, double *LF, int32_t precision,
                               void *hip_stream) {
    zi::g_err[0] = 0;
    if (!sys || !T || n_cols < 0 ||
        (n_cols > 0 && (!LF || !g_colptr || !g_rowind || !g_val))) {
        set_error("null argument or negative n_cols");
        return ZI_EINVAL;
    }
    ZI_GUARD(return zi_leadfield_noalloc_impl(sys, T, n_cols, g_colptr, g_rowind, g_val, LF,
                                              precision, (hipStream_t)hip_stream);)
}

int64_t zi_leadfield_noalloc_max_cols(int32_t n_electrodes) {
    return zi_leadfield_noalloc_max_cols_impl(n_electrodes);
}

zi_status zi_point_dipoles(const zi_system *sys, int32_t m, const int32_t *dipole_tets,
                           int32_t *g_colptr, int32_t *g_rowind, double *g_val,
                           void *hip_stream) {
    zi::g_err[0] = 0;
    if (!sys || m < 0 || !g_colptr || (m > 0 && (!dipole_tets || !g_rowind || !g_val))) {
        set_error("null argument or negative m");
        return ZI_EINVAL;
    }
    if ((int64_t)m * 12 >= (int64_t)1 << 31) {
        set_error("too many dipoles");
        return ZI_EINVAL;
    }
    ZI_GUARD({
        const zi_status st = zi_point_dipoles_impl(sys, m, dipole_tets, g_colptr, g_rowind,
                                                   g_val, (hipStream_t)hip_stream);
        if (st != ZI_OK) return st;
        if (hipStreamSynchronize((hipStream_t)hip_stream) != hipSuccess) {
            set_error("hipStreamSynchronize failed");
            return ZI_EDEVICE;
        }
        return ZI_OK;
    })
}

zi_status zi_spmm(const zi_system *sys, int32_t k, const double *X, double *Y, int32_t tile,
                  double *ms_out, void *hip_stream) {
    zi::g_err[0] = 0;
    if (!sys || !X || !Y || k <= 0) {
        set_error("null argument or k <= 0");
        return ZI_EINVAL;
    }
    ZI_GUARD(return zi_spmm_impl(sys, k, X, Y, tile, ms_out, (hipStream_t)hip_stream);)
}

zi_status zi_eit_source(const zi_system *sys, const double *T, int32_t n_patterns,
                        const double *I, int32_t n_elems, const int32_t *elems,
                        int32_t *g_colptr, int32_t *g_rowind, double *g_val, double *y_bg,
                        void *hip_stream) {
    zi::g_err[0] = 0;
    if (!sys || !T || !I || !g_colptr || !g_rowind || !g_val || n_patterns < 1 || n_elems < 1) {
        set_error("null argument, n_patterns < 1 or n_elems < 1");
        return ZI_EINVAL;
    }
    if (!elems && n_elems != sys->e) {
        set_error("elems == NULL needs n_elems == n_tets");
        return ZI_EINVAL;
    }
    if ((int64_t)n_patterns * n_elems * 4 >= (int64_t)1 << 31) {
        set_error("too many EIT source columns");
        return ZI_EINVAL;
    }
    ZI_GUARD(return zi_eit_source_impl(sys, T, n_patterns, I, n_elems, elems, g_colptr, g_rowind,
                                       g_val, y_bg, (hipStream_t)hip_stream);)
}

zi_status zi_gnn_create(const zi_system *sys, int32_t n_layers, const int32_t *dims,
                        const int32_t *hops, zi_gnn **out) {
    zi::g_err[0] = 0;
    if (!sys || !dims || !out || n_layers < 1 || n_layers > 32) {
        set_error("null argument or n_layers outside [1, 32]");
        return ZI_EINVAL;
    }
    *out = nullptr;
    for (int k = 0; k <= n_layers; ++k) {
        if (dims[k] < 1 || dims[k] > 64 || (k < n_layers && dims[k] % 2 != 0)) {
            set_error("dims[%d] = %d: need 1..64, even below the output layer", k, dims[k]);
            return ZI_EINVAL;
        }
    }
    for (int k = 0; hops && k < n_layers; ++k) {
        if (hops[k] < 1 || hops[k] > 1024) {
            set_error("hops[%d] = %d: need 1..1024", k, hops[k]);
            return ZI_EINVAL;
        }
    }
    ZI_GUARD(return zi_gnn_create_impl(sys, n_layers, dims, hops, out);)
}

zi_status zi_gnn_target(const double *T, int32_t ldT, int32_t col, const double *T0,
                        int32_t ldt, int32_t electrode, double gain, int32_t n_nodes, float *t,
                        double *sumsq, void *hip_stream) {
    zi::g_err[0] = 0;
    if (!T || !T0 || !t || n_nodes < 1 || col < 0 || col >= ldT || electrode < 0 ||
        electrode >= ldt || !(gain > 0.0)) {
        set_error("null argument, column out of range or gain <= 0");
        return ZI_EINVAL;
    }
    ZI_GUARD(return zi_gnn_target_impl(T, ldT, col, T0, ldt, electrode, gain, n_nodes, t, sumsq,
                                       (hipStream_t)hip_stream);)
}

zi_status zi_gnn_x0(const float *y, const double *T0, int32_t ldt, int32_t electrode,
                    double gain, int32_t n_nodes, double *x0, int32_t ldx, int32_t xcol,
                    void *hip_stream) {
    zi::g_err[0] = 0;
    if (!y || !T0 || !x0 || n_nodes < 1 || electrode < 0 || electrode >= ldt || xcol < 0 ||
        xcol >= ldx || !(gain > 0.0)) {
        set_error("null argument, column out of range or gain <= 0");
        return ZI_EINVAL;
    }
    ZI_GUARD(return zi_gnn_x0_impl(y, T0, ldt, electrode, gain, n_nodes, x0, ldx, xcol,
                                   (hipStream_t)hip_stream);)
}

zi_status zi_gnn_features(const zi_system *base, const zi_system *perturbed, const double *T0,
                          int32_t ldt, int32_t electrode, const double *centre, double radius,
                          float *X, void *hip_stream) {
    zi::g_err[0] = 0;
    if (!base || !perturbed || !T0 || !centre || !X) {
        set_error("null argument");
        return ZI_EINVAL;
    }
    if (perturbed->n != base->n || perturbed->nnz != base->nnz) {
        set_error("the perturbed system must share the base system's mesh");
        return ZI_EINVAL;
    }
    if (electrode < 0 || electrode >= base->L || ldt < base->L || !(radius > 0.0)) {
        set_error("electrode %d outside [0, %d), ldt %d < L, or radius <= 0", electrode, base->L,
                  ldt);
        return ZI_EINVAL;
    }
    ZI_GUARD(return zi_gnn_features_impl(base, perturbed, T0, ldt, electrode, centre, radius, X,
                                         (hipStream_t)hip_stream);)
}

int64_t zi_gnn_param_count(const zi_gnn *net) { return net ? zi_gnn_param_count_impl(net) : 0; }

zi_status zi_gnn_set_params(zi_gnn *net, const float *params) {
    zi::g_err[0] = 0;
    if (!net || !params) {
        set_error("null argument");
        return ZI_EINVAL;
    }
    ZI_GUARD(return zi_gnn_set_params_impl(net, params);)
}

zi_status zi_gnn_get_params(const zi_gnn *net, float *params) {
    zi::g_err[0] = 0;
    if (!net || !params) {
        set_error("null argument");
        return ZI_EINVAL;
    }
    ZI_GUARD(return zi_gnn_get_params_impl(net, params);)
}

zi_status zi_gnn_forward(zi_gnn *net, const float *X, float *y, void *hip_stream) {
    zi::g_err[0] = 0;
    if (!net || !X || !y) {
        set_error("null argument");
        return ZI_EINVAL;
    }
    ZI_GUARD(return zi_gnn_forward_impl(net, X, y, (hipStream_t)hip_stream);)
}

zi_status zi_gnn_loss_grad(zi_gnn *net, const float *X, const float *t, double *loss,
                           float *grads, void *hip_stream) {
    zi::g_err[0] = 0;
    if (!net || !X || !t) {
        set_error("null argument");
        return ZI_EINVAL;
    }
    ZI_GUARD(return zi_gnn_loss_grad_impl(net, X, t, loss, grads, (hipStream_t)hip_stream);)
}

zi_status zi_gnn_adam_step(zi_gnn *net, float lr, void *hip_stream) {
    zi::g_err[0] = 0;
    if (!net || !(lr > 0.f)) {
        set_error("null argument or lr <= 0");
        return ZI_EINVAL;
    }
    ZI_GUARD(return zi_gnn_adam_step_impl(net, lr, (hipStream_t)hip_stream);)
}

void zi_gnn_destroy(zi_gnn *net) {
    if (net) zi_gnn_destroy_impl(net);
}

zi_status zi_copy_probe(const double *src, double *dst, int64_t n, double *ms, void *hip_stream) {
    zi::g_err[0] = 0;
    if (!src || !dst || n < 2 || (n & 1)) {
        set_error("null argument or n not a positive even count");
        return ZI_EINVAL;
    }
    ZI_GUARD(return zi::copy_probe(src, dst, (size_t)n, ms, (hipStream_t)hip_stream);)
}

int32_t zi_tile_count(void) { return zi_tile_count_impl(); }
const char *zi_tile_name(int32_t t) { return zi_tile_name_impl(t); }

zi_status zi_get_info(const zi_system *sys, zi_system_info *info) {
    if (!sys || !info) {
        set_error("null argument");
        return ZI_EINVAL;
    }
    info->n_nodes = sys->n;
    info->n_tets = sys->e;
    info->n_electrodes = sys->L;
    info->ground_node = sys->ground;
    info->nnz = sys->nnz;
    info->b_nnz = sys->b_nnz;
    info->nnz_solver = sys->sp_nnz;
    return ZI_OK;
}

zi_status zi_get_view(const zi_system *sys, zi_system_view *v) {
    if (!sys || !v) {
        set_error("null argument");
        return ZI_EINVAL;
    }
    v->row_ptr = sys->row_ptr;
    v->col = sys->col;
    v->val = sys->val;
    v->b_ptr = sys->b_ptr;
    v->b_col = sys->b_col;
    v->b_val = sys->b_val;
    v->C = sys->C;
    v->calA = sys->calA;
    v->boundary = sys->boundary;
    return ZI_OK;
}

zi_status zi_release_cached_memory(void) { return zi::cache_clear(); }

void zi_system_destroy(zi_system *sys) {
    if (!sys) return;
    if (sys->ws) zi_solver_ws_destroy(sys->ws);
    if (sys->Pt) (void)hipFree(sys->Pt);
    delete sys;
}

}  // extern "C"
