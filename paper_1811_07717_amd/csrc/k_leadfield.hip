// EEG lead field, App. A.2 Eq. (aku):  LF = R (B^T T - C)^-1 T^T G.
//
//   schur   S = B^T T - C            (L x L; gathers T rows of each electrode)
//   chol_w  M = -(S + S^T)/2 = LL^T, W = R S^-1 = -R M^-1   (one workgroup)
//   gather  Pt[c, :] = sum_k G[k, c] T[k, :]   (T^T G stored n_cols x L)
//   gemm    LF = W Pt^T on the matrix cores (v_mfma_f64_16x16x4f64, or the
//           float32 variant), each wave owning 16 output columns and every
//           electrode row so that a Pt row is read once per wave.
#include <algorithm>
#include <cmath>
#include <mutex>

#include "zi_internal.h"

namespace {

using namespace zi;

inline unsigned grid_for(size_t n, int threads) {
    return (unsigned)((n + threads - 1) / threads);
}

// Caller's G in CSC form: colptr non-decreasing from 0, row indices in range.
__global__ void k_check_colptr(const int32_t *cp, int n_cols, int *flag) {
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c > n_cols) return;
    if (c == 0 && cp[0] != 0) atomicOr(flag, 2);
    if (c < n_cols && cp[c + 1] < cp[c]) atomicOr(flag, 2);
}

__global__ void k_check_rowind(const int32_t *ri, int32_t nnz, int32_t n, int *flag) {
    const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz && (ri[p] < 0 || ri[p] >= n)) atomicOr(flag, 2);
}

// S[l, m] = sum_{i in e_l} b_il T[i, m] - c_ll delta_lm; one block per l.
__global__ void k_schur(const int32_t *e_ptr, const int32_t *e_item, const int32_t *b_row,
                        const double *b_val, const double *C, const double *T, int L,
                        double *S) {
    const int l = blockIdx.x;
    for (int m = threadIdx.x; m < L; m += blockDim.x) {
        double s = 0.0;
        for (int32_t p = e_ptr[l]; p < e_ptr[l + 1]; ++p) {
            const int32_t k = e_item[p];
            s = fma(b_val[k], T[(size_t)b_row[k] * L + m], s);
        }
        if (m == l) s -= C[l];
        S[(size_t)l * L + m] = s;
    }
}

// In-place Cholesky of M = -(S + S^T)/2 (lower factor in Lf), then
// Minv = M^-1 by forward/backward substitution per column, then
// W = -R Minv with R = I - 11^T / L:  W_ij = -(Minv_ij - mean_k Minv_kj).
// Single workgroup; flag = 1 on a non-positive pivot.
constexpr int CHOL_THREADS = 256;

__global__ __launch_bounds__(CHOL_THREADS) void k_chol_w(const double *S, int L, double *Lf,
                                                         double *Minv, double *W, int *flag) {
    __shared__ double red[CHOL_THREADS];
    __shared__ double piv;
    const int tid = threadIdx.x;
    for (int idx = tid; idx < L * L; idx += CHOL_THREADS) {
        const int i = idx / L, j = idx % L;
        Lf[idx] = -0.5 * (S[(size_t)i * L + j] + S[(size_t)j * L + i]);
    }
    __syncthreads();
    for (int j = 0; j < L; ++j) {
        double part = 0.0;
        for (int k = tid; k < j; k += CHOL_THREADS) part = fma(Lf[j * L + k], Lf[j * L + k], part);
        red[tid] = part;
        __syncthreads();
        for (int off = CHOL_THREADS / 2; off > 0; off >>= 1) {
            if (tid < off) red[tid] += red[tid + off];
            __syncthreads();
        }
        if (tid == 0) {
            const double d = Lf[j * L + j] - red[0];
            if (!(d > 0.0)) *flag = 1;
            piv = d > 0.0 ? sqrt(d) : 1.0;
            Lf[j * L + j] = piv;
        }
        __syncthreads();
        for (int i = j + 1 + tid; i < L; i += CHOL_THREADS) {
            double s = Lf[i * L + j];
            for (int k = 0; k < j; ++k) s = fma(-Lf[i * L + k], Lf[j * L + k], s);
            Lf[i * L + j] = s / piv;
        }
        __syncthreads();
    }
    // Minv column c: solve L y = e_c, L^T x = y  (stored in Minv[:, c])
    for (int c = tid; c < L; c += CHOL_THREADS) {
        for (int i = 0; i < L; ++i) {
            double s = (i == c) ? 1.0 : 0.0;
            for (int k = c; k < i; ++k) s = fma(-Lf[i * L + k], Minv[(size_t)k * L + c], s);
            Minv[(size_t)i * L + c] = (i < c) ? 0.0 : s / Lf[i * L + i];
        }
        for (int i = L - 1; i >= 0; --i) {
            double s = Minv[(size_t)i * L + c];
            for (int k = i + 1; k < L; ++k) s = fma(-Lf[k * L + i], Minv[(size_t)k * L + c], s);
            Minv[(size_t)i * L + c] = s / Lf[i * L + i];
        }
    }
    __syncthreads();
    for (int c = tid; c < L; c += CHOL_THREADS) {
        double mean = 0.0;
        for (int k = 0; k < L; ++k) mean += Minv[(size_t)k * L + c];
        mean /= L;
        for (int i = 0; i < L; ++i) W[(size_t)i * L + c] = -(Minv[(size_t)i * L + c] - mean);
    }
}

// The same for L <= CHOL_LDS_MAX, in LDS: M is factored in place by a
// right-looking Cholesky (lower triangle, rows padded to L + 1 doubles so that
// column-parallel reads fall in different banks), L^-1 goes to the free upper
// triangle (transposed) and its diagonal to idiag, then M^-1 = L^-T L^-1 and W.
constexpr int CHOL_LDS_MAX = 128;
constexpr int CHOL_LDS_THREADS = 1024;

__global__ __launch_bounds__(CHOL_LDS_THREADS) void k_chol_lds(const double *S, int L,
                                                               double *Minv, double *W,
                                                               int *flag) {
    __shared__ double A[CHOL_LDS_MAX * (CHOL_LDS_MAX + 1)];
    __shared__ double idiag[CHOL_LDS_MAX];
    __shared__ double mean[CHOL_LDS_MAX];
    __shared__ int bad;
    const int tid = threadIdx.x, ld = L + 1;
    for (int idx = tid; idx < L * L; idx += CHOL_LDS_THREADS) {
        const int i = idx / L, j = idx % L;
        A[i * ld + j] = -0.5 * (S[(size_t)i * L + j] + S[(size_t)j * L + i]);
    }
    if (tid == 0) bad = 0;
    __syncthreads();
    for (int j = 0; j < L; ++j) {
        if (tid == 0) {
            const double d = A[j * ld + j];
            if (!(d > 0.0)) bad = 1;
            A[j * ld + j] = d > 0.0 ? sqrt(d) : 1.0;
        }
        __syncthreads();
        const double piv = A[j * ld + j];
        for (int i = j + 1 + tid; i < L; i += CHOL_LDS_THREADS) A[i * ld + j] /= piv;
        __syncthreads();
        const int m = L - j - 1;
        for (int idx = tid; idx < m * m; idx += CHOL_LDS_THREADS) {
            const int i = j + 1 + idx / m, k = j + 1 + idx % m;
            if (k <= i) A[i * ld + k] = fma(-A[i * ld + j], A[k * ld + j], A[i * ld + k]);
        }
        __syncthreads();
    }
    if (tid == 0 && bad) *flag = 1;
    // column c of L^-1: Linv[c][c] = 1 / L_cc, Linv[i][c] (i > c) stored at A[c][i]
    for (int c = tid; c < L; c += CHOL_LDS_THREADS) {
        const double dc = 1.0 / A[c * ld + c];
        idiag[c] = dc;
        for (int i = c + 1; i < L; ++i) {
            double sum = A[i * ld + c] * dc;
            for (int k = c + 1; k < i; ++k) sum = fma(A[i * ld + k], A[c * ld + k], sum);
            A[c * ld + i] = -sum / A[i * ld + i];
        }
    }
    __syncthreads();
    // M^-1[i][j] = sum_{k >= max(i, j)} Linv[k][i] Linv[k][j]
    for (int idx = tid; idx < L * L; idx += CHOL_LDS_THREADS) {
        const int i = idx / L, j = idx % L;
        const int k0 = i > j ? i : j;
        double sum = 0.0;
        for (int k = k0; k < L; ++k) {
            const double a = k == i ? idiag[i] : A[i * ld + k];
            const double b = k == j ? idiag[j] : A[j * ld + k];
            sum = fma(a, b, sum);
        }
        Minv[idx] = sum;
    }
    __syncthreads();
    for (int c = tid; c < L; c += CHOL_LDS_THREADS) {
        double sum = 0.0;
        for (int k = 0; k < L; ++k) sum += Minv[(size_t)k * L + c];
        mean[c] = sum / L;
    }
    __syncthreads();
    for (int idx = tid; idx < L * L; idx += CHOL_LDS_THREADS)
        W[idx] = -(Minv[idx] - mean[idx % L]);
}

void launch_chol(const double *S, int L, double *Lf, double *Minv, double *W, int *flag,
                 hipStream_t s) {
    if (L <= CHOL_LDS_MAX)
        hipLaunchKernelGGL(k_chol_lds, dim3(1), dim3(CHOL_LDS_THREADS), 0, s, S, L, Minv, W,
                           flag);
    else
        hipLaunchKernelGGL(k_chol_w, dim3(1), dim3(CHOL_THREADS), 0, s, S, L, Lf, Minv, W, flag);
}

// Pt[c, :] = sum_k G[k, c] T[k, :]; one wave per column, lanes over electrodes.
__global__ void k_gather(const int32_t *cp, const int32_t *ri, const double *gv, int n_cols,
                         const double *T, int L, double *Pt) {
    const int64_t c = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) >> 6;
    const int lane = threadIdx.x & 63;
    if (c >= n_cols) return;
    const int32_t s = cp[c], e = cp[c + 1];
    for (int l = lane; l < L; l += 64) {
        double acc = 0.0;
        for (int32_t p = s; p < e; ++p) acc = fma(gv[p], T[(size_t)ri[p] * L + l], acc);
        Pt[(size_t)c * L + l] = acc;
    }
}

// LF[l, c] = sum_k W[l, k] Pt[c, k].  One wave per 16 output columns, all L
// rows (L <= 256 -> at most 16 row tiles of 16).  MFMA 16x16x4 operand layout:
// lane t supplies A[t%16][t/16] and B[t/16][t%16]; it receives, for
// i = 0..3, D[t/16 + 4 i][t%16] (float64 variant) or D[4 (t/16) + i][t%16]
// (float32 variant) -- both measured with an in-bounds probe on gfx950.
typedef double dbl4 __attribute__((ext_vector_type(4)));
typedef float flt4 __attribute__((ext_vector_type(4)));

// Four waves per block, 16 output columns each (64 per block).  W is staged
// in LDS gk(MT) columns at a time (rows padded to gk + 1 so that the 16 rows a
// wave reads per MFMA fall in different banks) in two alternating buffers:
// the next chunk of W and of the B operand (Pt) is requested before the MFMAs
// of the current one and stored after them, so one barrier per chunk orders
// the buffers and no MFMA waits for a global load.  Every wave forms all MT
// row tiles of its columns from the staged chunk, so W is read once per 64
// output columns and the B operand once per k step.
constexpr int GEMM_THREADS = 256;
template <int MT>
constexpr int gk() { return MT <= 8 ? 16 : 8; }   // two buffers stay within 64 KB

template <int MT, class F>
__device__ __forceinline__ void gemm_tile(const double *W, const double *Pt, int L, int n_cols,
                                          double (*Ws)[MT * 16][gk<MT>() + 1], F mfma_step) {
    constexpr int GK = gk<MT>();
    constexpr int NW = MT * 16 * GK;                              // W entries per chunk
    constexpr int PER = (NW + GEMM_THREADS - 1) / GEMM_THREADS;   // per thread
    const int t = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + wv * 16 + (t & 15);
    const int kq = t >> 4;
    const int nchunk = (L + GK - 1) / GK;
    double wreg[PER], breg[GK / 4];
    auto request = [&](int k0) {
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = threadIdx.x + i * GEMM_THREADS;
            const int r = idx / GK, kk = idx % GK;
            wreg[i] = (idx < NW && r < L && k0 + kk < L) ? W[(size_t)r * L + k0 + kk] : 0.0;
        }
#pragma unroll
        for (int j = 0; j < GK / 4; ++j) {
            const int k = k0 + 4 * j + kq;
            breg[j] = (col < n_cols && k < L) ? Pt[(size_t)col * L + k] : 0.0;
        }
    };
    request(0);
    for (int c = 0; c < nchunk; ++c) {
        const int buf = c & 1;
        // buffer buf was last read in chunk c - 2, before the previous barrier
#pragma unroll
        for (int i = 0; i < PER; ++i) {
            const int idx = threadIdx.x + i * GEMM_THREADS;
            if (idx < NW) Ws[buf][idx / GK][idx % GK] = wreg[i];
        }
        double bcur[GK / 4];
#pragma unroll
        for (int j = 0; j < GK / 4; ++j) bcur[j] = breg[j];
        __syncthreads();
        if (c + 1 < nchunk) request((c + 1) * GK);
#pragma unroll
        for (int j = 0; j < GK / 4; ++j) mfma_step(Ws[buf], 4 * j + kq, bcur[j]);
    }
}

template <int MT>
__global__ __launch_bounds__(GEMM_THREADS) void k_gemm_f64(const double *W, const double *Pt,
                                                           int L, int n_cols, int64_t ldlf,
                                                           double *LF) {
    __shared__ double Ws[2][MT * 16][gk<MT>() + 1];
    const int t = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + wv * 16 + (t & 15);
    const int kq = t >> 4;
    dbl4 acc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m] = dbl4{0.0, 0.0, 0.0, 0.0};
    gemm_tile<MT>(W, Pt, L, n_cols, Ws, [&](const double (*Wb)[gk<MT>() + 1], int kk, double b) {
#pragma unroll
        for (int m = 0; m < MT; ++m)
            acc[m] = __builtin_amdgcn_mfma_f64_16x16x4f64(Wb[m * 16 + (t & 15)][kk], b, acc[m],
                                                          0, 0, 0);
    });
    if (col >= n_cols) return;
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = m * 16 + kq + 4 * i;   // f64 result layout
            if (row < L) LF[(size_t)row * ldlf + col] = acc[m][i];
        }
}

template <int MT>
__global__ __launch_bounds__(GEMM_THREADS) void k_gemm_f32(const double *W, const double *Pt,
                                                           int L, int n_cols, int64_t ldlf,
                                                           double *LF) {
    __shared__ double Ws[2][MT * 16][gk<MT>() + 1];
    const int t = threadIdx.x & 63, wv = threadIdx.x >> 6;
    const int col = blockIdx.x * 64 + wv * 16 + (t & 15);
    const int kq = t >> 4;
    flt4 acc[MT];
#pragma unroll
    for (int m = 0; m < MT; ++m) acc[m] = flt4{0.f, 0.f, 0.f, 0.f};
    gemm_tile<MT>(W, Pt, L, n_cols, Ws, [&](const double (*Wb)[gk<MT>() + 1], int kk, double b) {
#pragma unroll
        for (int m = 0; m < MT; ++m)
            acc[m] = __builtin_amdgcn_mfma_f32_16x16x4f32((float)Wb[m * 16 + (t & 15)][kk],
                                                          (float)b, acc[m], 0, 0, 0);
    });
    if (col >= n_cols) return;
#pragma unroll
    for (int m = 0; m < MT; ++m)
#pragma unroll
        for (int i = 0; i < 4; ++i) {
            const int row = m * 16 + 4 * kq + i;   // f32 result layout
            if (row < L) LF[(size_t)row * ldlf + col] = (double)acc[m][i];
        }
}

#define ZI_GEMM_SWITCH(KER, mt, ...)                                   \
    switch (mt) {                                                      \
        case 1: hipLaunchKernelGGL(KER<1>, __VA_ARGS__); break;        \
        case 2: hipLaunchKernelGGL(KER<2>, __VA_ARGS__); break;        \
        case 3: hipLaunchKernelGGL(KER<3>, __VA_ARGS__); break;        \
        case 4: hipLaunchKernelGGL(KER<4>, __VA_ARGS__); break;        \
        case 5: hipLaunchKernelGGL(KER<5>, __VA_ARGS__); break;        \
        case 6: hipLaunchKernelGGL(KER<6>, __VA_ARGS__); break;        \
        case 7: hipLaunchKernelGGL(KER<7>, __VA_ARGS__); break;        \
        case 8: hipLaunchKernelGGL(KER<8>, __VA_ARGS__); break;        \
        case 9: hipLaunchKernelGGL(KER<9>, __VA_ARGS__); break;        \
        case 10: hipLaunchKernelGGL(KER<10>, __VA_ARGS__); break;      \
        case 11: hipLaunchKernelGGL(KER<11>, __VA_ARGS__); break;      \
        case 12: hipLaunchKernelGGL(KER<12>, __VA_ARGS__); break;      \
        case 13: hipLaunchKernelGGL(KER<13>, __VA_ARGS__); break;      \
        case 14: hipLaunchKernelGGL(KER<14>, __VA_ARGS__); break;      \
        case 15: hipLaunchKernelGGL(KER<15>, __VA_ARGS__); break;      \
        default: hipLaunchKernelGGL(KER<16>, __VA_ARGS__); break;      \
    }

// Mi = Minv I (L x P) and y_bg = R Mi; one thread per (l, p).
__global__ void k_minv_apply(const double *Minv, const double *I, int L, int P, double *Mi) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= L * P) return;
    const int l = idx / P, p = idx % P;
    double s = 0.0;
    for (int k = 0; k < L; ++k) s = fma(Minv[(size_t)l * L + k], I[(size_t)k * P + p], s);
    Mi[idx] = s;
}

__global__ void k_avg_ref(const double *Mi, int L, int P, double *y) {
    const int idx = blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= L * P) return;
    const int p = idx % P;
    double mean = 0.0;
    for (int k = 0; k < L; ++k) mean += Mi[(size_t)k * P + p];
    y[idx] = Mi[idx] - mean / L;
}

// U = T Mi (n x P), one thread per (i, p).
__global__ void k_apply_T(const double *T, const double *Mi, int32_t n, int L, int P, double *U) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)n * P) return;
    const int64_t i = idx / P;
    const int p = (int)(idx % P);
    double s = 0.0;
    for (int l = 0; l < L; ++l) s = fma(T[i * L + l], Mi[(size_t)l * P + p], s);
    U[idx] = s;
}

}  // namespace

zi_status zi_eit_source_impl(const zi_system *sys, const double *T, int32_t P, const double *I,
                             int32_t ne, const int32_t *elems, int32_t *cp, int32_t *ri,
                             double *gv, double *y_bg, hipStream_t s) {
    const int L = sys->L;
    if (L > 1024) {
        set_error("zi_eit_source supports at most 1024 electrodes");
        return ZI_EINVAL;
    }
    for (int p = 0; p < P; ++p) {
        double sum = 0.0, mx = 0.0;
        for (int l = 0; l < L; ++l) {
            sum += I[(size_t)l * P + p];
            mx = fmax(mx, fabs(I[(size_t)l * P + p]));
        }
        if (!(fabs(sum) <= 1e-12 * mx)) {
            set_error("current pattern %d does not sum to zero", p);
            return ZI_EINVAL;
        }
    }
    Pool tmp;
    double *S = nullptr, *Lf = nullptr, *Minv = nullptr, *W = nullptr, *Id = nullptr,
           *Mi = nullptr, *Y = nullptr, *U = nullptr;
    int *flag = nullptr;
    ZI_TRY(tmp.alloc(&S, (size_t)L * L));
    ZI_TRY(tmp.alloc(&Lf, (size_t)L * L));
    ZI_TRY(tmp.alloc(&Minv, (size_t)L * L));
    ZI_TRY(tmp.alloc(&W, (size_t)L * L));
    ZI_TRY(tmp.alloc(&Id, (size_t)L * P));
    ZI_TRY(tmp.alloc(&Mi, (size_t)L * P));
    ZI_TRY(tmp.alloc(&Y, (size_t)L * P));
    ZI_TRY(tmp.alloc(&U, (size_t)sys->n * P));
    ZI_TRY(tmp.alloc(&flag, 1));
    ZI_TRY(fill_i32(flag, 0, 1, s));
    ZI_HIP(hipMemcpyAsync(Id, I, sizeof(double) * L * P, hipMemcpyHostToDevice, s));
    hipLaunchKernelGGL(k_schur, dim3(L), dim3(64), 0, s, sys->e_ptr, sys->e_item, sys->b_row,
                       sys->b_val, sys->C, T, L, S);
    launch_chol(S, L, Lf, Minv, W, flag, s);
    hipLaunchKernelGGL(k_minv_apply, dim3(grid_for((size_t)L * P, 128)), dim3(128), 0, s, Minv, Id,
                       L, P, Mi);
    hipLaunchKernelGGL(k_avg_ref, dim3(grid_for((size_t)L * P, 128)), dim3(128), 0, s, Mi, L, P, Y);
    hipLaunchKernelGGL(k_apply_T, dim3(grid_for((size_t)sys->n * P, 256)), dim3(256), 0, s, T, Mi,
                       sys->n, L, P, U);
    ZI_HIP(hipGetLastError());
    int hflag = 0;
    ZI_HIP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, s));
    ZI_HIP(hipStreamSynchronize(s));
    if (hflag) {
        set_error("M = C - B^T T is not positive definite");
        return ZI_EBREAKDOWN;
    }
    ZI_TRY(zi_eit_columns_impl(sys, U, P, ne, elems, cp, ri, gv, s));
    if (y_bg) ZI_HIP(hipMemcpyAsync(y_bg, Y, sizeof(double) * L * P, hipMemcpyDeviceToHost, s));
    ZI_HIP(hipStreamSynchronize(s));
    return ZI_OK;
}

namespace {

// Workspace of one lead-field evaluation: the L x L matrices of the Schur
// complement step, the flag word, and Pt for up to pt_cols columns of G.
struct LfWork {
    double *S, *Lf, *Minv, *W, *Pt;
    int *flag;
    int64_t pt_cols;
};

zi_status leadfield_core(const zi_system *sys, const double *T, int32_t n_cols,
                         const int32_t *cp, const int32_t *ri, const double *gv, double *LF,
                         int32_t precision, const LfWork &w, hipStream_t s) {
    const int L = sys->L;
    ZI_TRY(fill_i32(w.flag, 0, 1, s));
    int hflag = 0;
    if (n_cols > 0) {
        hipLaunchKernelGGL(k_check_colptr, dim3(grid_for((size_t)n_cols + 1, 256)), dim3(256), 0,
                           s, cp, n_cols, w.flag);
        ZI_HIP(hipGetLastError());
        int32_t gnnz = 0;
        ZI_HIP(hipMemcpyAsync(&gnnz, cp + n_cols, sizeof(int32_t), hipMemcpyDeviceToHost, s));
        ZI_HIP(hipMemcpyAsync(&hflag, w.flag, sizeof(int), hipMemcpyDeviceToHost, s));
        ZI_HIP(hipStreamSynchronize(s));
        if (!hflag && gnnz > 0) {
            hipLaunchKernelGGL(k_check_rowind, dim3(grid_for(gnnz, 256)), dim3(256), 0, s, ri,
                               gnnz, sys->n, w.flag);
            ZI_HIP(hipGetLastError());
            ZI_HIP(hipMemcpyAsync(&hflag, w.flag, sizeof(int), hipMemcpyDeviceToHost, s));
            ZI_HIP(hipStreamSynchronize(s));
        }
        if (hflag) {
            set_error("G: column pointers not monotone from 0, or a row index out of range");
            return ZI_EINVAL;
        }
    }
    hipLaunchKernelGGL(k_schur, dim3(L), dim3(64), 0, s, sys->e_ptr, sys->e_item, sys->b_row,
                       sys->b_val, sys->C, T, L, w.S);
    launch_chol(w.S, L, w.Lf, w.Minv, w.W, w.flag, s);
    ZI_HIP(hipGetLastError());
    // columns in chunks of at most pt_cols: the gather of a chunk, then its
    // product into columns [c0, c0 + nc) of LF (leading dimension n_cols)
    const int mt = (L + 15) / 16;
    for (int64_t c0 = 0; c0 < n_cols; c0 += w.pt_cols) {
        const int nc = (int)std::min<int64_t>(w.pt_cols, n_cols - c0);
        hipLaunchKernelGGL(k_gather, dim3(grid_for((size_t)nc * 64, 256)), dim3(256), 0, s,
                           cp + c0, ri, gv, nc, T, L, w.Pt);
        const dim3 grid(grid_for(nc, 64)), block(GEMM_THREADS);
        if (precision == 0) {
            ZI_GEMM_SWITCH(k_gemm_f64, mt, grid, block, 0, s, w.W, w.Pt, L, nc,
                           (int64_t)n_cols, LF + c0);
        } else {
            ZI_GEMM_SWITCH(k_gemm_f32, mt, grid, block, 0, s, w.W, w.Pt, L, nc,
                           (int64_t)n_cols, LF + c0);
        }
        ZI_HIP(hipGetLastError());
    }
    ZI_HIP(hipMemcpyAsync(&hflag, w.flag, sizeof(int), hipMemcpyDeviceToHost, s));
    ZI_HIP(hipStreamSynchronize(s));
    if (hflag) {
        set_error("M = C - B^T T is not positive definite");
        return ZI_EBREAKDOWN;
    }
    return ZI_OK;
}

zi_status leadfield_args(const zi_system *sys, int32_t precision) {
    if (sys->L > 256) {
        set_error("zi_leadfield supports at most 256 electrodes (got %d)", sys->L);
        return ZI_EINVAL;
    }
    if (precision != 0 && precision != 1) {
        set_error("unknown lead-field precision %d", precision);
        return ZI_EINVAL;
    }
    return ZI_OK;
}

// ---------------------------------------------------------------------------
// Lead field without device allocation.  The workspace lives in `scratch`, a
// fixed array of every device the library runs on; host code reaches it only
// through the address hipGetSymbolAddress returns for the current device.
constexpr size_t NOALLOC_DOUBLES = (size_t)2 << 20;   // 16 MiB
static __device__ __align__(256) double scratch[NOALLOC_DOUBLES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
double *g_scratch[MAX_DEVICES] = {};

zi_status scratch_for_current_device(double **out) {
    int dev = -1;
    ZI_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= MAX_DEVICES) {
        set_error("device index %d out of range", dev);
        return ZI_EDEVICE;
    }
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch[dev]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p) {
            set_error("hipGetSymbolAddress(scratch) failed: %s", hipGetErrorString(e));
            return ZI_EDEVICE;
        }
        g_scratch[dev] = static_cast<double *>(p);
    }
    *out = g_scratch[dev];
    return ZI_OK;
}

}  // namespace

int64_t zi_leadfield_noalloc_max_cols_impl(int32_t L) {
    if (L < 1 || L > 256) return 0;
    const size_t mat = (size_t)L * L;
    return (int64_t)((NOALLOC_DOUBLES - 4 * mat - 32) / (size_t)L);
}

zi_status zi_leadfield_noalloc_impl(const zi_system *sys, const double *T, int32_t n_cols,
                                    const int32_t *cp, const int32_t *ri, const double *gv,
                                    double *LF, int32_t precision, hipStream_t s) {
    ZI_TRY(leadfield_args(sys, precision));
    double *base = nullptr;
    ZI_TRY(scratch_for_current_device(&base));
    const size_t mat = (size_t)sys->L * sys->L;
    LfWork w;
    w.S = base;
    w.Lf = base + mat;
    w.Minv = base + 2 * mat;
    w.W = base + 3 * mat;
    w.flag = reinterpret_cast<int *>(base + 4 * mat);
    w.Pt = base + 4 * mat + 32;
    w.pt_cols = zi_leadfield_noalloc_max_cols_impl(sys->L);
    return leadfield_core(sys, T, n_cols, cp, ri, gv, LF, precision, w, s);
}

zi_status zi_leadfield_impl(const zi_system *csys, const double *T, int32_t n_cols,
                            const int32_t *cp, const int32_t *ri, const double *gv, double *LF,
                            int32_t precision, hipStream_t s) {
    zi_system *sys = const_cast<zi_system *>(csys);
    ZI_TRY(leadfield_args(sys, precision));
    const int L = sys->L;
    Pool tmp;
    LfWork w;
    ZI_TRY(tmp.alloc(&w.S, (size_t)L * L));
    ZI_TRY(tmp.alloc(&w.Lf, (size_t)L * L));
    ZI_TRY(tmp.alloc(&w.Minv, (size_t)L * L));
    ZI_TRY(tmp.alloc(&w.flag, 1));
    if (!sys->W) ZI_TRY(sys->pool.alloc(&sys->W, (size_t)L * L));
    w.W = sys->W;
    const size_t need = (size_t)n_cols * L;
    if (need > sys->Pt_cap) {
        if (sys->Pt) (void)hipFree(sys->Pt);
        sys->Pt = nullptr;
        sys->Pt_cap = 0;
        ZI_HIP(hipMalloc(&sys->Pt, need * sizeof(double)));
        sys->Pt_cap = need;
    }
    w.Pt = sys->Pt;
    w.pt_cols = std::max<int64_t>(n_cols, 1);
    return leadfield_core(sys, T, n_cols, cp, ri, gv, LF, precision, w, s);
}
