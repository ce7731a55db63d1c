// Mesh-graph network for learned PCG initial iterates (float32).
//
// The network runs on the mesh graph of the assembled system (the CSR
// structure of A), aggregated with Ahat = D^-1/2 Adj D^-1/2 (diagonal entries
// stored as zeros), which is symmetric, so the backward aggregation is the
// same SpMM.  Layer k with h_k hops:  M = Ahat^h_k H,  Z = H Ws + M Wn + b,
// H' = relu(Z) (identity on the last layer); prediction y = H_K[:, 0]; loss
// sum (y - t)^2 / sum t^2.  Weight gradients are reduced per block in float64
// and across blocks in a fixed order, so training is bitwise reproducible.
#include <cmath>
#include <vector>

#include "zi_internal.h"

struct zi_gnn {
    const zi_system *sys = nullptr;
    int K = 0;
    std::vector<int> dims;
    std::vector<int> hops;                 // aggregation hops per layer (>= 1)
    std::vector<int64_t> off_ws, off_wn, off_b;   // offsets into the flat parameter array
    int64_t nparam = 0;
    float *params = nullptr, *grads = nullptr, *adam_m = nullptr, *adam_v = nullptr;
    float *ahat = nullptr;                 // nnz values on the system's CSR structure
    std::vector<float *> H, M;             // H[0..K], M[0..K-1]; H[0] is the input copy
    float *dH = nullptr, *dZ = nullptr, *dM = nullptr, *tmp = nullptr, *tmp2 = nullptr;
    double *part = nullptr;                // weight-gradient partials
    int nblk = 0;
    double *lpart = nullptr;               // loss partials
    double *scal = nullptr;                // [loss, 2 / sum t^2]
    int adam_t = 0;
    zi::Pool pool;
};

namespace {

using namespace zi;

constexpr int GBLK = 256;
constexpr int WG_BLOCKS = 512;     // blocks of the weight-gradient reduction
constexpr int WG_ROWS = 16;        // rows staged per step in LDS

inline unsigned grid_for(size_t n, int threads) {
    return (unsigned)((n + threads - 1) / threads);
}

__global__ void k_ahat(const int32_t *rp, const int32_t *ci, int32_t n, float *ahat) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int di = rp[i + 1] - rp[i] - 1;
    for (int32_t q = rp[i]; q < rp[i + 1]; ++q) {
        const int j = ci[q];
        const int dj = rp[j + 1] - rp[j] - 1;
        ahat[q] = (j == i || di <= 0 || dj <= 0) ? 0.f : (float)(1.0 / sqrt((double)di * dj));
    }
}

// out[r, j] = b[j] + sum_i A[r, i] W1[i, j] + B[r, i] W2[i, j]  (W2, B, b optional)
// then relu when requested, plus an optional additive input add[r, j].
// Weights are staged in LDS; each thread owns one output feature of one row.
__global__ __launch_bounds__(GBLK) void k_dense(const float *A, const float *W1, const float *B,
                                                const float *W2, const float *bias,
                                                const float *add, int fin, int fout,
                                                bool transpose_w, bool relu, int32_t n,
                                                float *out) {
    extern __shared__ float sw[];                 // W1 then W2, fin x fout each
    float *w1 = sw, *w2 = sw + fin * fout;
    for (int k = threadIdx.x; k < fin * fout; k += GBLK) {
        // transpose_w: W given as fout x fin (use W^T)
        const int i = k / fout, j = k % fout;
        w1[k] = transpose_w ? W1[j * fin + i] : W1[k];
        if (W2) w2[k] = transpose_w ? W2[j * fin + i] : W2[k];
    }
    __syncthreads();
    const int rows_per = GBLK / fout;
    const int j = threadIdx.x % fout;
    const int rl = threadIdx.x / fout;
    if (rl >= rows_per) return;
    for (int64_t r = (int64_t)blockIdx.x * rows_per + rl; r < n; r += (int64_t)gridDim.x * rows_per) {
        float z = bias ? bias[j] : 0.f;
        const float *a = A + r * fin;
        for (int i = 0; i < fin; ++i) z = fmaf(a[i], w1[i * fout + j], z);
        if (B) {
            const float *bb = B + r * fin;
            for (int i = 0; i < fin; ++i) z = fmaf(bb[i], w2[i * fout + j], z);
        }
        if (add) z += add[r * fout + j];
        if (relu) z = fmaxf(z, 0.f);
        out[r * fout + j] = z;
    }
}

// dZ = dH * (H' > 0)  (the ReLU mask, from the stored activation)
__global__ void k_relu_mask(const float *Hn, float *dZ, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count && !(Hn[i] > 0.f)) dZ[i] = 0.f;
}

// Block partials of A^T D (fin x fout) over a contiguous row chunk, and of the
// column sums of D when A == nullptr; accumulated in float64.
__global__ __launch_bounds__(GBLK) void k_wgrad(const float *A, const float *D, int fin, int fout,
                                                int32_t n, double *part) {
    __shared__ float sa[WG_ROWS * 64];
    __shared__ float sd[WG_ROWS * 64];
    const int ent = (A ? fin : 1) * fout;
    const int per = (ent + GBLK - 1) / GBLK;        // entries per thread (<= 16)
    double acc[16];
    for (int q = 0; q < 16; ++q) acc[q] = 0.0;
    const int64_t chunk = ((int64_t)n + gridDim.x - 1) / gridDim.x;
    const int64_t r0 = blockIdx.x * chunk;
    const int64_t r1 = min((int64_t)n, r0 + chunk);
    for (int64_t rb = r0; rb < r1; rb += WG_ROWS) {
        const int nr = (int)min((int64_t)WG_ROWS, r1 - rb);
        __syncthreads();
        for (int k = threadIdx.x; k < nr * fout; k += GBLK) sd[k] = D[rb * fout + k];
        if (A)
            for (int k = threadIdx.x; k < nr * fin; k += GBLK) sa[k] = A[rb * fin + k];
        __syncthreads();
        for (int q = 0; q < per; ++q) {
            const int e = threadIdx.x + q * GBLK;
            if (e >= ent) break;
            const int i = e / fout, j = e % fout;
            float s = 0.f;
            for (int r = 0; r < nr; ++r) s = fmaf(A ? sa[r * fin + i] : 1.f, sd[r * fout + j], s);
            acc[q] += (double)s;
        }
    }
    for (int q = 0; q < per; ++q) {
        const int e = threadIdx.x + q * GBLK;
        if (e < ent) part[(size_t)blockIdx.x * ent + e] = acc[q];
    }
}

__global__ void k_wgrad_reduce(const double *part, int nblk, int ent, float *g) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= ent) return;
    double s = 0.0;
    for (int b = 0; b < nblk; ++b) s += part[(size_t)b * ent + e];
    g[e] = (float)s;
}

// loss partials: sum (y - t)^2 and sum t^2 (float64), y = Y[r * ldy]
__global__ __launch_bounds__(GBLK) void k_loss_part(const float *Y, int ldy, const float *t,
                                                    int32_t n, double *part) {
    __shared__ double s1[GBLK], s2[GBLK];
    double a = 0.0, b = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * GBLK + threadIdx.x; r < n; r += (int64_t)gridDim.x * GBLK) {
        const double d = (double)Y[r * ldy] - (double)t[r];
        a += d * d;
        b += (double)t[r] * (double)t[r];
    }
    s1[threadIdx.x] = a;
    s2[threadIdx.x] = b;
    __syncthreads();
    for (int off = GBLK / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            s1[threadIdx.x] += s1[threadIdx.x + off];
            s2[threadIdx.x] += s2[threadIdx.x + off];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        part[2 * blockIdx.x] = s1[0];
        part[2 * blockIdx.x + 1] = s2[0];
    }
}

__global__ void k_loss_final(const double *part, int nblk, double *scal) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double a = 0.0, b = 0.0;
    for (int k = 0; k < nblk; ++k) {
        a += part[2 * k];
        b += part[2 * k + 1];
    }
    scal[0] = b > 0 ? a / b : 0.0;
    scal[1] = b > 0 ? 2.0 / b : 0.0;
}

// dY[r, 0] = (2 / sum t^2) (y - t); other output columns (if any) zero
__global__ void k_dloss(const float *Y, int ldy, const float *t, const double *scal, int32_t n,
                        float *dY) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    dY[r * ldy] = (float)(scal[1] * ((double)Y[r * ldy] - (double)t[r]));
    for (int j = 1; j < ldy; ++j) dY[r * ldy + j] = 0.f;
}

__global__ void k_adam(float *p, const float *g, float *m, float *v, int64_t count, float lr,
                       float b1, float b2, float eps, float c1, float c2) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= count) return;
    const float gi = g[i];
    const float mi = b1 * m[i] + (1.f - b1) * gi;
    const float vi = b2 * v[i] + (1.f - b2) * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= lr * (mi / c1) / (sqrtf(vi / c2) + eps);
}

zi_status dense(const float *A, const float *W1, const float *B, const float *W2, const float *b,
                const float *add, int fin, int fout, bool tw, bool relu, int32_t n, float *out,
                hipStream_t s) {
    const size_t lds = (size_t)2 * fin * fout * sizeof(float);
    const int rows_per = GBLK / fout;
    unsigned grid = grid_for(n, rows_per);
    if (grid > 8192) grid = 8192;
    hipLaunchKernelGGL(k_dense, dim3(grid), dim3(GBLK), lds, s, A, W1, B, W2, b, add, fin, fout, tw,
                       relu, n, out);
    ZI_HIP(hipGetLastError());
    return ZI_OK;
}

zi_status wgrad(zi_gnn *g, const float *A, const float *D, int fin, int fout, float *out,
                hipStream_t s) {
    const int32_t n = g->sys->n;
    const int ent = (A ? fin : 1) * fout;
    hipLaunchKernelGGL(k_wgrad, dim3(g->nblk), dim3(GBLK), 0, s, A, D, fin, fout, n, g->part);
    hipLaunchKernelGGL(k_wgrad_reduce, dim3(grid_for(ent, 256)), dim3(256), 0, s, g->part,
                       g->nblk, ent, out);
    ZI_HIP(hipGetLastError());
    return ZI_OK;
}

// out = Ahat^hops in (hops >= 1): one product at a time through the two
// scratch blocks a and b, the last product written to out.
zi_status aggregate(zi_gnn *g, const float *in, int hops, int fi, float *out, float *a, float *b,
                    hipStream_t s) {
    const int32_t n = g->sys->n;
    const float *src = in;
    for (int h = 0; h < hops; ++h) {
        float *dst = h == hops - 1 ? out : ((hops - 1 - h) % 2 ? a : b);
        ZI_TRY(spmm_f32(g->sys->row_ptr, g->sys->col, g->ahat, src, dst, n, fi, s));
        src = dst;
    }
    return ZI_OK;
}

zi_status forward(zi_gnn *g, const float *X, hipStream_t s) {
    const int32_t n = g->sys->n;
    ZI_HIP(hipMemcpyAsync(g->H[0], X, sizeof(float) * (size_t)n * g->dims[0],
                          hipMemcpyDeviceToDevice, s));
    for (int k = 0; k < g->K; ++k) {
        const int fi = g->dims[k], fo = g->dims[k + 1];
        ZI_TRY(aggregate(g, g->H[k], g->hops[k], fi, g->M[k], g->tmp, g->tmp2, s));
        ZI_TRY(dense(g->H[k], g->params + g->off_ws[k], g->M[k], g->params + g->off_wn[k],
                     g->params + g->off_b[k], nullptr, fi, fo, false, k < g->K - 1, n,
                     g->H[k + 1], s));
    }
    return ZI_OK;
}

}  // namespace

zi_status zi_gnn_create_impl(const zi_system *sys, int32_t K, const int32_t *dims,
                             const int32_t *hops, zi_gnn **out) {
    zi_gnn *g = new zi_gnn();
    struct Guard {
        zi_gnn *p;
        ~Guard() {
            if (p) delete p;
        }
    } guard{g};
    g->sys = sys;
    g->K = K;
    g->dims.assign(dims, dims + K + 1);
    g->hops.assign(K, 1);
    if (hops) g->hops.assign(hops, hops + K);
    int64_t off = 0;
    for (int k = 0; k < K; ++k) {
        const int64_t w = (int64_t)dims[k] * dims[k + 1];
        g->off_ws.push_back(off);
        off += w;
        g->off_wn.push_back(off);
        off += w;
        g->off_b.push_back(off);
        off += dims[k + 1];
    }
    g->nparam = off;
    const int32_t n = sys->n;
    int fmax = 0;
    for (int d : g->dims) fmax = d > fmax ? d : fmax;
    ZI_TRY(g->pool.alloc(&g->params, (size_t)off));
    ZI_TRY(g->pool.alloc(&g->grads, (size_t)off));
    ZI_TRY(g->pool.alloc(&g->adam_m, (size_t)off));
    ZI_TRY(g->pool.alloc(&g->adam_v, (size_t)off));
    ZI_TRY(g->pool.alloc(&g->ahat, (size_t)sys->nnz));
    g->H.resize(K + 1);
    g->M.resize(K);
    for (int k = 0; k <= K; ++k) ZI_TRY(g->pool.alloc(&g->H[k], (size_t)n * dims[k]));
    for (int k = 0; k < K; ++k) ZI_TRY(g->pool.alloc(&g->M[k], (size_t)n * dims[k]));
    ZI_TRY(g->pool.alloc(&g->dH, (size_t)n * fmax));
    ZI_TRY(g->pool.alloc(&g->dZ, (size_t)n * fmax));
    ZI_TRY(g->pool.alloc(&g->dM, (size_t)n * fmax));
    ZI_TRY(g->pool.alloc(&g->tmp, (size_t)n * fmax));
    ZI_TRY(g->pool.alloc(&g->tmp2, (size_t)n * fmax));
    g->nblk = WG_BLOCKS;
    ZI_TRY(g->pool.alloc(&g->part, (size_t)g->nblk * fmax * fmax));
    ZI_TRY(g->pool.alloc(&g->lpart, (size_t)2 * 1024));
    ZI_TRY(g->pool.alloc(&g->scal, 2));
    hipLaunchKernelGGL(k_ahat, dim3(grid_for(n, 256)), dim3(256), 0, 0, sys->row_ptr, sys->col, n,
                       g->ahat);
    ZI_HIP(hipGetLastError());
    ZI_HIP(hipMemset(g->grads, 0, sizeof(float) * off));
    ZI_HIP(hipMemset(g->adam_m, 0, sizeof(float) * off));
    ZI_HIP(hipMemset(g->adam_v, 0, sizeof(float) * off));
    ZI_HIP(hipMemset(g->params, 0, sizeof(float) * off));
    ZI_HIP(hipDeviceSynchronize());
    guard.p = nullptr;
    *out = g;
    return ZI_OK;
}

void zi_gnn_destroy_impl(zi_gnn *g) { delete g; }
int64_t zi_gnn_param_count_impl(const zi_gnn *g) { return g->nparam; }

zi_status zi_gnn_set_params_impl(zi_gnn *g, const float *p) {
    ZI_HIP(hipMemcpy(g->params, p, sizeof(float) * g->nparam, hipMemcpyHostToDevice));
    ZI_HIP(hipMemset(g->adam_m, 0, sizeof(float) * g->nparam));
    ZI_HIP(hipMemset(g->adam_v, 0, sizeof(float) * g->nparam));
    g->adam_t = 0;
    return ZI_OK;
}

zi_status zi_gnn_get_params_impl(const zi_gnn *g, float *p) {
    ZI_HIP(hipMemcpy(p, g->params, sizeof(float) * g->nparam, hipMemcpyDeviceToHost));
    return ZI_OK;
}

zi_status zi_gnn_forward_impl(zi_gnn *g, const float *X, float *y, hipStream_t s) {
    ZI_TRY(forward(g, X, s));
    const int32_t n = g->sys->n;
    const int fo = g->dims[g->K];
    if (fo == 1) {
        ZI_HIP(hipMemcpyAsync(y, g->H[g->K], sizeof(float) * n, hipMemcpyDeviceToDevice, s));
    } else {
        ZI_HIP(hipMemcpy2DAsync(y, sizeof(float), g->H[g->K], sizeof(float) * fo, sizeof(float), n,
                                hipMemcpyDeviceToDevice, s));
    }
    ZI_HIP(hipStreamSynchronize(s));
    return ZI_OK;
}

zi_status zi_gnn_loss_grad_impl(zi_gnn *g, const float *X, const float *t, double *loss,
                                float *grads_host, hipStream_t s) {
    const int32_t n = g->sys->n;
    const int K = g->K;
    ZI_TRY(forward(g, X, s));
    const int fo = g->dims[K];
    const int lb = 256;
    hipLaunchKernelGGL(k_loss_part, dim3(lb), dim3(GBLK), 0, s, g->H[K], fo, t, n, g->lpart);
    hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(64), 0, s, g->lpart, lb, g->scal);
    hipLaunchKernelGGL(k_dloss, dim3(grid_for(n, 256)), dim3(256), 0, s, g->H[K], fo, t, g->scal,
                       n, g->dH);
    ZI_HIP(hipGetLastError());
    for (int k = K - 1; k >= 0; --k) {
        const int fi = g->dims[k], fok = g->dims[k + 1];
        const int64_t cnt = (int64_t)n * fok;
        ZI_HIP(hipMemcpyAsync(g->dZ, g->dH, sizeof(float) * cnt, hipMemcpyDeviceToDevice, s));
        if (k < K - 1)
            hipLaunchKernelGGL(k_relu_mask, dim3(grid_for(cnt, 256)), dim3(256), 0, s, g->H[k + 1],
                               g->dZ, cnt);
        ZI_TRY(wgrad(g, g->H[k], g->dZ, fi, fok, g->grads + g->off_ws[k], s));
        ZI_TRY(wgrad(g, g->M[k], g->dZ, fi, fok, g->grads + g->off_wn[k], s));
        ZI_TRY(wgrad(g, nullptr, g->dZ, fi, fok, g->grads + g->off_b[k], s));
        if (k == 0) break;
        // dM = dZ Wn^T;  dH = dZ Ws^T + Ahat dM
        ZI_TRY(dense(g->dZ, g->params + g->off_wn[k], nullptr, nullptr, nullptr, nullptr, fok, fi,
                     true, false, n, g->dM, s));
        ZI_TRY(aggregate(g, g->dM, g->hops[k], fi, g->tmp, g->dH, g->tmp2, s));
        ZI_TRY(dense(g->dZ, g->params + g->off_ws[k], nullptr, nullptr, nullptr, g->tmp, fok, fi,
                     true, false, n, g->dH, s));
    }
    double h[2] = {0, 0};
    ZI_HIP(hipMemcpyAsync(h, g->scal, sizeof(double) * 2, hipMemcpyDeviceToHost, s));
    if (grads_host)
        ZI_HIP(hipMemcpyAsync(grads_host, g->grads, sizeof(float) * g->nparam,
                              hipMemcpyDeviceToHost, s));
    ZI_HIP(hipStreamSynchronize(s));
    if (loss) *loss = h[0];
    return ZI_OK;
}

zi_status zi_gnn_adam_step_impl(zi_gnn *g, float lr, hipStream_t s) {
    g->adam_t += 1;
    const float b1 = 0.9f, b2 = 0.999f;
    const float c1 = 1.f - powf(b1, (float)g->adam_t), c2 = 1.f - powf(b2, (float)g->adam_t);
    hipLaunchKernelGGL(k_adam, dim3(grid_for(g->nparam, 256)), dim3(256), 0, s, g->params, g->grads,
                       g->adam_m, g->adam_v, g->nparam, lr, b1, b2, 1e-8f, c1, c2);
    ZI_HIP(hipGetLastError());
    ZI_HIP(hipStreamSynchronize(s));
    return ZI_OK;
}

// ---------------------------------------------------------------------------
// Input features of the warm-start network (see zi_gnn_features in zi.h).

namespace {

constexpr int FEAT = 10;
constexpr int FBLK = 256;
constexpr int FBLOCKS = 512;

// raw[3 i + (0, 1, 2)] = (b_il, t0_il, (b_l - A t0_l)_i) and block maxima of
// |b|, |t0|, |r| and a0_ii (maxima: the same in any order).
__global__ __launch_bounds__(FBLK) void k_feat_raw(
    int32_t n, int32_t l, const int32_t *bp, const int32_t *bc, const double *bv,
    const double *T0, int32_t ldt, const int32_t *rp, const int32_t *ci, const double *va,
    const double *d0, double *raw, double *part) {
    __shared__ double sm[4][FBLK];
    double m[4] = {0.0, 0.0, 0.0, 0.0};
    for (int64_t i = (int64_t)blockIdx.x * FBLK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * FBLK) {
        double b = 0.0;
        for (int32_t k = bp[i]; k < bp[i + 1]; ++k)
            if (bc[k] == l) b += bv[k];
        const double t0 = T0[i * ldt + l];
        double at = 0.0;
        for (int32_t q = rp[i]; q < rp[i + 1]; ++q) at = fma(va[q], T0[(int64_t)ci[q] * ldt + l], at);
        const double r = b - at;
        raw[3 * i] = b;
        raw[3 * i + 1] = t0;
        raw[3 * i + 2] = r;
        m[0] = fmax(m[0], fabs(b));
        m[1] = fmax(m[1], fabs(t0));
        m[2] = fmax(m[2], fabs(r));
        m[3] = fmax(m[3], d0[i]);
    }
    for (int q = 0; q < 4; ++q) sm[q][threadIdx.x] = m[q];
    __syncthreads();
    for (int off = FBLK / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off)
            for (int q = 0; q < 4; ++q)
                sm[q][threadIdx.x] = fmax(sm[q][threadIdx.x], sm[q][threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x < 4) part[4 * blockIdx.x + threadIdx.x] = sm[threadIdx.x][0];
}

__global__ void k_feat_max(const double *part, int nblk, double *mx) {
    const int q = threadIdx.x;
    if (q >= 4) return;
    double m = 0.0;
    for (int b = 0; b < nblk; ++b) m = fmax(m, part[4 * b + q]);
    mx[q] = m > 0.0 ? m : 1.0;
}

__global__ void k_feat_write(int32_t n, const double *raw, const double *mx, const double *d,
                             const double *d0, const double *nodes, double cx, double cy,
                             double cz, double inv_r, float *X) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const double x = nodes[3 * i], y = nodes[3 * i + 1], z = nodes[3 * i + 2];
    const double dx = x - cx, dy = y - cy, dz = z - cz;
    float *o = X + i * FEAT;
    o[0] = (float)(raw[3 * i] / mx[0]);
    o[1] = (float)log(d[i] / d0[i]);
    o[2] = (float)(raw[3 * i + 1] / mx[1]);
    o[3] = (float)(x * inv_r);
    o[4] = (float)(y * inv_r);
    o[5] = (float)(z * inv_r);
    o[6] = (float)(sqrt(dx * dx + dy * dy + dz * dz) * inv_r);
    o[7] = (float)log(d0[i] / mx[3]);
    o[8] = (float)(raw[3 * i + 2] / mx[2]);
    o[9] = 1.f;   // a constant input (the aggregation sees the node degree)
}

}  // namespace

zi_status zi_gnn_features_impl(const zi_system *base, const zi_system *pert, const double *T0,
                               int32_t ldt, int32_t l, const double *centre, double radius,
                               float *X, hipStream_t s) {
    const int32_t n = base->n;
    Pool tmp;
    double *raw = nullptr, *part = nullptr, *mx = nullptr;
    ZI_TRY(tmp.alloc(&raw, (size_t)3 * n));
    ZI_TRY(tmp.alloc(&part, (size_t)4 * FBLOCKS));
    ZI_TRY(tmp.alloc(&mx, 4));
    hipLaunchKernelGGL(k_feat_raw, dim3(FBLOCKS), dim3(FBLK), 0, s, n, l, base->b_ptr,
                       base->b_col, base->b_val, T0, ldt, pert->row_ptr, pert->col, pert->val,
                       base->diag, raw, part);
    hipLaunchKernelGGL(k_feat_max, dim3(1), dim3(64), 0, s, part, FBLOCKS, mx);
    hipLaunchKernelGGL(k_feat_write, dim3(grid_for(n, 256)), dim3(256), 0, s, n, raw, mx,
                       pert->diag, base->diag, base->nodes, centre[0], centre[1], centre[2],
                       1.0 / radius, X);
    ZI_HIP(hipGetLastError());
    ZI_HIP(hipStreamSynchronize(s));
    return ZI_OK;
}

// ---------------------------------------------------------------------------
// Training targets and proposed initial iterates: with s_l = max_i |t0_il|,
// target t_i = gain (T_i,col - t0_il) / s_l and x0_i = t0_il + s_l y_i / gain.

namespace {

__global__ __launch_bounds__(FBLK) void k_colmax_part(const double *T0, int32_t ldt, int32_t l,
                                                      int32_t n, double *part) {
    __shared__ double sm[FBLK];
    double m = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * FBLK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * FBLK)
        m = fmax(m, fabs(T0[i * ldt + l]));
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int off = FBLK / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sm[threadIdx.x] = fmax(sm[threadIdx.x], sm[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ void k_colmax_final(const double *part, int nblk, double *mx) {
    if (threadIdx.x != 0) return;
    double m = 0.0;
    for (int b = 0; b < nblk; ++b) m = fmax(m, part[b]);
    mx[0] = m > 0.0 ? m : 1.0;
}

// target and its sum of squares per block (float64, fixed order)
__global__ __launch_bounds__(FBLK) void k_target(const double *T, int32_t ldT, int32_t col,
                                                 const double *T0, int32_t ldt, int32_t l,
                                                 double gain, const double *mx, int32_t n,
                                                 float *t, double *part) {
    __shared__ double sm[FBLK];
    double a = 0.0;
    const double f = gain / mx[0];
    for (int64_t i = (int64_t)blockIdx.x * FBLK + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * FBLK) {
        const float v = (float)(f * (T[i * ldT + col] - T0[i * ldt + l]));
        t[i] = v;
        a += (double)v * (double)v;
    }
    sm[threadIdx.x] = a;
    __syncthreads();
    for (int off = FBLK / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sm[threadIdx.x] += sm[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = sm[0];
}

__global__ void k_x0(const float *y, const double *T0, int32_t ldt, int32_t l, double gain,
                     const double *mx, int32_t n, double *x0, int32_t ldx, int32_t xcol) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    x0[i * ldx + xcol] = T0[i * ldt + l] + mx[0] * (double)y[i] / gain;
}

zi_status colmax(const double *T0, int32_t ldt, int32_t l, int32_t n, double *part, double *mx,
                 hipStream_t s) {
    hipLaunchKernelGGL(k_colmax_part, dim3(FBLOCKS), dim3(FBLK), 0, s, T0, ldt, l, n, part);
    hipLaunchKernelGGL(k_colmax_final, dim3(1), dim3(64), 0, s, part, FBLOCKS, mx);
    ZI_HIP(hipGetLastError());
    return ZI_OK;
}

}  // namespace

zi_status zi_gnn_target_impl(const double *T, int32_t ldT, int32_t col, const double *T0,
                             int32_t ldt, int32_t l, double gain, int32_t n, float *t,
                             double *sumsq, hipStream_t s) {
    Pool tmp;
    double *part = nullptr, *mx = nullptr;
    ZI_TRY(tmp.alloc(&part, (size_t)FBLOCKS));
    ZI_TRY(tmp.alloc(&mx, 1));
    ZI_TRY(colmax(T0, ldt, l, n, part, mx, s));
    hipLaunchKernelGGL(k_target, dim3(FBLOCKS), dim3(FBLK), 0, s, T, ldT, col, T0, ldt, l, gain,
                       mx, n, t, part);
    ZI_HIP(hipGetLastError());
    std::vector<double> h(FBLOCKS);
    ZI_HIP(hipMemcpyAsync(h.data(), part, sizeof(double) * FBLOCKS, hipMemcpyDeviceToHost, s));
    ZI_HIP(hipStreamSynchronize(s));
    double a = 0.0;
    for (double v : h) a += v;
    if (sumsq) *sumsq = a;
    return ZI_OK;
}

zi_status zi_gnn_x0_impl(const float *y, const double *T0, int32_t ldt, int32_t l, double gain,
                         int32_t n, double *x0, int32_t ldx, int32_t xcol, hipStream_t s) {
    Pool tmp;
    double *part = nullptr, *mx = nullptr;
    ZI_TRY(tmp.alloc(&part, (size_t)FBLOCKS));
    ZI_TRY(tmp.alloc(&mx, 1));
    ZI_TRY(colmax(T0, ldt, l, n, part, mx, s));
    hipLaunchKernelGGL(k_x0, dim3(grid_for(n, 256)), dim3(256), 0, s, y, T0, ldt, l, gain, mx, n,
                       x0, ldx, xcol);
    ZI_HIP(hipGetLastError());
    ZI_HIP(hipStreamSynchronize(s));
    return ZI_OK;
}
