// Transfer matrix T = A^-1 B (App. A.4) by the diagonally preconditioned
// conjugate gradient of Sec. 2.3.1, run on all electrode columns at once.
//
// Every column runs its own textbook PCG (its own alpha, beta, rho and stop
// test); the columns only share the sweeps over A.  Block vectors are n x ldp
// row-major (node-major), ldp = L rounded up to even; padding columns are
// zero and inactive.
//
// Kernels per iteration:
//   spmm_pq   Q = A P            + per-column partial p.q
//   red_alpha alpha = rho / p.q  (one block per column, fixed order)
//   update    X += alpha P, R -= alpha Q + partials r.D^-1 r and r.r
//   red_beta  stop test, beta = rho'/rho, iteration counts
//   pupdate   P = D^-1 R + beta P
//
// Tiling: a wave holds 64/LPR rows; each lane owns NV column pairs (double2).
// A block (4 waves) owns a (row tile, column chunk of CW = 2 LPR NV columns).
// Blocks are numbered so that the 8 XCDs (block b runs on XCD b mod 8) each
// receive a contiguous range of tiles: consecutive rows (and their shared
// neighbours) stay in one XCD's L2.  Dot-product partials are reduced inside
// the block in a fixed order and across blocks by the red_* kernels in a
// fixed order, so results are bitwise reproducible.
#include <chrono>
#include <cmath>
#include <cstring>

#include "zi_internal.h"

namespace {

using namespace zi;

constexpr int BLOCK = 256;           // 4 waves
constexpr int TARGET_BLOCKS = 2048;  // row tiles x column chunks per launch

struct Geom {
    int n, ldp, rb, nrt, ncc, nb, nb_pad;
};

__device__ __forceinline__ bool block_tile(const Geom &g, int &cc, int &rt) {
    const int b = blockIdx.x;
    const int per = g.nb_pad >> 3;
    const int logical = (b & 7) * per + (b >> 3);
    if (logical >= g.nb) return false;
    cc = logical / g.nrt;
    rt = logical - cc * g.nrt;
    return true;
}

template <int LPR, int NV>
struct Lane {
    static constexpr int RPW = 64 / LPR;
    static constexpr int CW = 2 * LPR * NV;
    static constexpr int RSTEP = 4 * RPW;
    int w, r, lr, slot;
    int c[NV];
    bool ok[NV];
    __device__ __forceinline__ Lane(const Geom &g, int cc) {
        const int tid = threadIdx.x;
        w = tid >> 6;
        const int lane = tid & 63;
        r = lane / LPR;
        lr = lane % LPR;
        slot = w * RPW + r;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            c[v] = cc * CW + 2 * (lr + LPR * v);
            ok[v] = c[v] < g.ldp;
        }
    }
};

__device__ __forceinline__ double2 ld2(const double *p) {
    return *reinterpret_cast<const double2 *>(p);
}
__device__ __forceinline__ void st2(double *p, double2 v) {
    *reinterpret_cast<double2 *>(p) = v;
}

// acc = sum_k a_k X[j_k, c..c+1] over row `row`, in column order.
template <int NV>
__device__ __forceinline__ void row_product(const int32_t *__restrict__ rp,
                                            const int32_t *__restrict__ ci,
                                            const double *__restrict__ va,
                                            const double *__restrict__ X, int ldp, int row,
                                            const int c[NV], const bool ok[NV], double2 acc[NV]) {
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = make_double2(0.0, 0.0);
    const int s = rp[row], e = rp[row + 1];
    int k = s;
    for (; k + 4 <= e; k += 4) {
        int j[4];
        double a[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            j[u] = ci[k + u];
            a[u] = va[k + u];
        }
        double2 x[4][NV];
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < NV; ++v)
                x[u][v] = ok[v] ? ld2(X + (size_t)j[u] * ldp + c[v]) : make_double2(0.0, 0.0);
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                acc[v].x = fma(a[u], x[u][v].x, acc[v].x);
                acc[v].y = fma(a[u], x[u][v].y, acc[v].y);
            }
    }
    for (; k < e; ++k) {
        const int j = ci[k];
        const double a = va[k];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const double2 x = ok[v] ? ld2(X + (size_t)j * ldp + c[v]) : make_double2(0.0, 0.0);
            acc[v].x = fma(a, x.x, acc[v].x);
            acc[v].y = fma(a, x.y, acc[v].y);
        }
    }
}

// Sum NQ per-lane partials over the block's rows (fixed order) and store them
// column-major: part[q][col * nrt + rt].
template <int LPR, int NV, int NQ>
__device__ __forceinline__ void block_partials(const Geom &g, const Lane<LPR, NV> &ln, int cc,
                                               int rt, const double2 (&acc)[NQ][NV],
                                               double *const (&part)[NQ]) {
    constexpr int RS = Lane<LPR, NV>::RSTEP;
    constexpr int CW = Lane<LPR, NV>::CW;
    __shared__ double red[NQ][RS][CW];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int cl = 2 * (ln.lr + LPR * v);
            red[q][ln.slot][cl] = acc[q][v].x;
            red[q][ln.slot][cl + 1] = acc[q][v].y;
        }
    __syncthreads();
    for (int idx = threadIdx.x; idx < NQ * CW; idx += BLOCK) {
        const int q = idx / CW, cl = idx - q * CW;
        const int col = cc * CW + cl;
        if (col < g.ldp) {
            double s = 0.0;
            for (int k = 0; k < RS; ++k) s += red[q][k][cl];
            part[q][(size_t)col * g.nrt + rt] = s;
        }
    }
}

// ---------------------------------------------------------------------------

// Y = A X; with WITH_DOT also the partials of sum_i X[i,c] Y[i,c].
template <int LPR, int NV, bool WITH_DOT>
__global__ __launch_bounds__(BLOCK) void k_spmm(Geom g, const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ ci,
                                                const double *__restrict__ va,
                                                const double *__restrict__ X,
                                                double *__restrict__ Y, double *part) {
    int cc, rt;
    if (!block_tile(g, cc, rt)) return;
    Lane<LPR, NV> ln(g, cc);
    double2 dotacc[1][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) dotacc[0][v] = make_double2(0.0, 0.0);
    const int r0 = rt * g.rb;
    const int r1 = min(g.n, r0 + g.rb);
    for (int row = r0 + ln.slot; row < r1; row += Lane<LPR, NV>::RSTEP) {
        double2 acc[NV];
        row_product<NV>(rp, ci, va, X, g.ldp, row, ln.c, ln.ok, acc);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (!ln.ok[v]) continue;
            st2(Y + (size_t)row * g.ldp + ln.c[v], acc[v]);
            if (WITH_DOT) {
                const double2 p = ld2(X + (size_t)row * g.ldp + ln.c[v]);
                dotacc[0][v].x = fma(p.x, acc[v].x, dotacc[0][v].x);
                dotacc[0][v].y = fma(p.y, acc[v].y, dotacc[0][v].y);
            }
        }
    }
    if (WITH_DOT) {
        double *const parts[1] = {part};
        block_partials<LPR, NV, 1>(g, ln, cc, rt, dotacc, parts);
    }
}

// X += alpha P, R -= alpha Q; partials r.D^-1 r and r.r of the new R.
template <int LPR, int NV>
__global__ __launch_bounds__(BLOCK) void k_update(Geom g, const double *__restrict__ alpha,
                                                  const double *__restrict__ dinv,
                                                  double *__restrict__ X,
                                                  double *__restrict__ R,
                                                  const double *__restrict__ P,
                                                  const double *__restrict__ Q, double *prz,
                                                  double *prr) {
    int cc, rt;
    if (!block_tile(g, cc, rt)) return;
    Lane<LPR, NV> ln(g, cc);
    double2 acc[2][NV];
    double2 al[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        acc[0][v] = acc[1][v] = make_double2(0.0, 0.0);
        al[v] = ln.ok[v] ? ld2(alpha + ln.c[v]) : make_double2(0.0, 0.0);
    }
    const int r0 = rt * g.rb;
    const int r1 = min(g.n, r0 + g.rb);
    for (int row = r0 + ln.slot; row < r1; row += Lane<LPR, NV>::RSTEP) {
        const double di = dinv[row];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (!ln.ok[v]) continue;
            const size_t o = (size_t)row * g.ldp + ln.c[v];
            double2 x = ld2(X + o), r = ld2(R + o);
            const double2 p = ld2(P + o), q = ld2(Q + o);
            x.x = fma(al[v].x, p.x, x.x);
            x.y = fma(al[v].y, p.y, x.y);
            r.x = fma(-al[v].x, q.x, r.x);
            r.y = fma(-al[v].y, q.y, r.y);
            st2(X + o, x);
            st2(R + o, r);
            acc[0][v].x = fma(r.x, r.x * di, acc[0][v].x);
            acc[0][v].y = fma(r.y, r.y * di, acc[0][v].y);
            acc[1][v].x = fma(r.x, r.x, acc[1][v].x);
            acc[1][v].y = fma(r.y, r.y, acc[1][v].y);
        }
    }
    double *const parts[2] = {prz, prr};
    block_partials<LPR, NV, 2>(g, ln, cc, rt, acc, parts);
}

// P = D^-1 R + beta P (beta == nullptr: P = D^-1 R).
template <int LPR, int NV>
__global__ __launch_bounds__(BLOCK) void k_pupdate(Geom g, const double *__restrict__ beta,
                                                   const double *__restrict__ dinv,
                                                   const double *__restrict__ R,
                                                   double *__restrict__ P) {
    int cc, rt;
    if (!block_tile(g, cc, rt)) return;
    Lane<LPR, NV> ln(g, cc);
    double2 be[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
        be[v] = (ln.ok[v] && beta) ? ld2(beta + ln.c[v]) : make_double2(0.0, 0.0);
    const int r0 = rt * g.rb;
    const int r1 = min(g.n, r0 + g.rb);
    for (int row = r0 + ln.slot; row < r1; row += Lane<LPR, NV>::RSTEP) {
        const double di = dinv[row];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (!ln.ok[v]) continue;
            const size_t o = (size_t)row * g.ldp + ln.c[v];
            const double2 r = ld2(R + o);
            double2 p;
            if (beta) {
                p = ld2(P + o);
                p.x = fma(be[v].x, p.x, r.x * di);
                p.y = fma(be[v].y, p.y, r.y * di);
            } else {
                p = make_double2(r.x * di, r.y * di);
            }
            st2(P + o, p);
        }
    }
}

// R = B - Q (Q may be null: R = B).  Partials: b.b, r.D^-1 r, r.r.  R may be
// null (only the partials are wanted: true residual).
template <int LPR, int NV>
__global__ __launch_bounds__(BLOCK) void k_residual(Geom g, const int32_t *__restrict__ bp,
                                                    const int32_t *__restrict__ bc,
                                                    const double *__restrict__ bv,
                                                    const double *__restrict__ dinv,
                                                    const double *__restrict__ Q,
                                                    double *__restrict__ R, double *pbb,
                                                    double *prz, double *prr) {
    int cc, rt;
    if (!block_tile(g, cc, rt)) return;
    Lane<LPR, NV> ln(g, cc);
    double2 acc[3][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[0][v] = acc[1][v] = acc[2][v] = make_double2(0.0, 0.0);
    const int r0 = rt * g.rb;
    const int r1 = min(g.n, r0 + g.rb);
    for (int row = r0 + ln.slot; row < r1; row += Lane<LPR, NV>::RSTEP) {
        const double di = dinv[row];
        const int s = bp[row], e = bp[row + 1];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (!ln.ok[v]) continue;
            double2 b = make_double2(0.0, 0.0);
            for (int k = s; k < e; ++k) {
                const int l = bc[k];
                if (l == ln.c[v]) b.x = bv[k];
                if (l == ln.c[v] + 1) b.y = bv[k];
            }
            const size_t o = (size_t)row * g.ldp + ln.c[v];
            double2 r = b;
            if (Q) {
                const double2 q = ld2(Q + o);
                r.x = b.x - q.x;
                r.y = b.y - q.y;
            }
            if (R) st2(R + o, r);
            acc[0][v].x = fma(b.x, b.x, acc[0][v].x);
            acc[0][v].y = fma(b.y, b.y, acc[0][v].y);
            acc[1][v].x = fma(r.x, r.x * di, acc[1][v].x);
            acc[1][v].y = fma(r.y, r.y * di, acc[1][v].y);
            acc[2][v].x = fma(r.x, r.x, acc[2][v].x);
            acc[2][v].y = fma(r.y, r.y, acc[2][v].y);
        }
    }
    double *const parts[3] = {pbb, prz, prr};
    block_partials<LPR, NV, 3>(g, ln, cc, rt, acc, parts);
}

// ---------------------------------------------------------------------------
// Per-column reductions (one block per column, fixed order).

struct Scal {
    double *rho, *alpha, *beta, *bb, *rr;
    int32_t *iters, *active, *flag;   // flag[0]: breakdown
};

constexpr int RED = 256;

__device__ __forceinline__ double col_sum(const double *part, int nrt, int c) {
    __shared__ double s[RED];
    double acc = 0.0;
    for (int k = threadIdx.x; k < nrt; k += RED) acc += part[(size_t)c * nrt + k];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = RED / 2; off > 0; off >>= 1) {
        if (threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    const double r = s[0];
    __syncthreads();
    return r;
}

__global__ __launch_bounds__(RED) void k_red_init(Scal sc, const double *pbb, const double *prz,
                                                  const double *prr, int nrt, int L,
                                                  double tol2) {
    const int c = blockIdx.x;
    const double bb = col_sum(pbb, nrt, c);
    const double rz = col_sum(prz, nrt, c);
    const double rr = col_sum(prr, nrt, c);
    if (threadIdx.x == 0) {
        sc.bb[c] = bb;
        sc.rho[c] = rz;
        sc.rr[c] = rr;
        sc.iters[c] = 0;
        sc.alpha[c] = 0.0;
        sc.beta[c] = 0.0;
        sc.active[c] = (c < L && bb > 0.0 && rr > tol2 * bb) ? 1 : 0;
    }
}

__global__ __launch_bounds__(RED) void k_red_alpha(Scal sc, const double *ppq, int nrt) {
    const int c = blockIdx.x;
    const double pq = col_sum(ppq, nrt, c);
    if (threadIdx.x == 0) {
        double a = 0.0;
        if (sc.active[c]) {
            if (pq > 0.0) {
                a = sc.rho[c] / pq;
            } else {
                sc.active[c] = 0;
                sc.flag[0] = 1;
            }
        }
        sc.alpha[c] = a;
    }
}

__global__ __launch_bounds__(RED) void k_red_beta(Scal sc, const double *prz, const double *prr,
                                                  int nrt, double tol2) {
    const int c = blockIdx.x;
    const double rz = col_sum(prz, nrt, c);
    const double rr = col_sum(prr, nrt, c);
    if (threadIdx.x == 0) {
        double b = 0.0;
        if (sc.active[c]) {
            sc.iters[c] += 1;
            sc.rr[c] = rr;
            if (rr <= tol2 * sc.bb[c]) {
                sc.active[c] = 0;
            } else {
                b = rz / sc.rho[c];
                sc.rho[c] = rz;
            }
        }
        sc.beta[c] = b;
    }
}

__global__ __launch_bounds__(RED) void k_red_sum(const double *part, int nrt, double *out) {
    const int c = blockIdx.x;
    const double s = col_sum(part, nrt, c);
    if (threadIdx.x == 0) out[c] = s;
}

// ---------------------------------------------------------------------------
// Tile table and dispatch

struct TileCfg {
    int lpr, nv;
    const char *name;
};

const TileCfg kTiles[] = {
    {64, 1, "lpr64_nv1_cw128"}, {64, 2, "lpr64_nv2_cw256"}, {32, 1, "lpr32_nv1_cw64"},
    {32, 2, "lpr32_nv2_cw128"}, {16, 1, "lpr16_nv1_cw32"},  {16, 2, "lpr16_nv2_cw64"},
    {8, 1, "lpr8_nv1_cw16"},    {8, 2, "lpr8_nv2_cw32"},    {4, 1, "lpr4_nv1_cw8"},
    {64, 4, "lpr64_nv4_cw512"},
};
constexpr int NTILES = sizeof(kTiles) / sizeof(kTiles[0]);

#define ZI_TILE_SWITCH(tile, FN, ...)                       \
    switch (tile) {                                         \
        case 0: FN<64, 1>(__VA_ARGS__); break;              \
        case 1: FN<64, 2>(__VA_ARGS__); break;              \
        case 2: FN<32, 1>(__VA_ARGS__); break;              \
        case 3: FN<32, 2>(__VA_ARGS__); break;              \
        case 4: FN<16, 1>(__VA_ARGS__); break;              \
        case 5: FN<16, 2>(__VA_ARGS__); break;              \
        case 6: FN<8, 1>(__VA_ARGS__); break;               \
        case 7: FN<8, 2>(__VA_ARGS__); break;               \
        case 8: FN<4, 1>(__VA_ARGS__); break;               \
        default: FN<64, 4>(__VA_ARGS__); break;             \
    }

int auto_tile(int ldp) {
    // narrowest single chunk that holds every column, else the widest tile
    int best = -1, bestcw = 1 << 30;
    for (int t = 0; t < NTILES; ++t) {
        const int cw = 2 * kTiles[t].lpr * kTiles[t].nv;
        if (cw >= ldp && cw < bestcw) {
            best = t;
            bestcw = cw;
        }
    }
    return best >= 0 ? best : 9;
}

Geom make_geom(int n, int ldp, int tile) {
    const TileCfg &t = kTiles[tile];
    const int cw = 2 * t.lpr * t.nv;
    const int rstep = 4 * (64 / t.lpr);
    Geom g;
    g.n = n;
    g.ldp = ldp;
    g.ncc = (ldp + cw - 1) / cw;
    int nrt_target = TARGET_BLOCKS / g.ncc;
    if (nrt_target < 1) nrt_target = 1;
    int rb = (n + nrt_target - 1) / nrt_target;
    rb = ((rb + rstep - 1) / rstep) * rstep;
    if (rb < rstep) rb = rstep;
    g.rb = rb;
    g.nrt = (n + rb - 1) / rb;
    if (g.nrt < 1) g.nrt = 1;
    g.nb = g.ncc * g.nrt;
    g.nb_pad = ((g.nb + 7) / 8) * 8;
    return g;
}

template <int LPR, int NV>
void launch_spmm(const Geom &g, hipStream_t s, const zi_system *sys, const double *X, double *Y,
                 double *part) {
    if (part)
        hipLaunchKernelGGL((k_spmm<LPR, NV, true>), dim3(g.nb_pad), dim3(BLOCK), 0, s, g,
                           sys->row_ptr, sys->col, sys->val, X, Y, part);
    else
        hipLaunchKernelGGL((k_spmm<LPR, NV, false>), dim3(g.nb_pad), dim3(BLOCK), 0, s, g,
                           sys->row_ptr, sys->col, sys->val, X, Y, part);
}

template <int LPR, int NV>
void launch_update(const Geom &g, hipStream_t s, const double *alpha, const double *dinv,
                   double *X, double *R, const double *P, const double *Q, double *prz,
                   double *prr) {
    hipLaunchKernelGGL((k_update<LPR, NV>), dim3(g.nb_pad), dim3(BLOCK), 0, s, g, alpha, dinv, X,
                       R, P, Q, prz, prr);
}

template <int LPR, int NV>
void launch_pupdate(const Geom &g, hipStream_t s, const double *beta, const double *dinv,
                    const double *R, double *P) {
    hipLaunchKernelGGL((k_pupdate<LPR, NV>), dim3(g.nb_pad), dim3(BLOCK), 0, s, g, beta, dinv, R,
                       P);
}

template <int LPR, int NV>
void launch_residual(const Geom &g, hipStream_t s, const zi_system *sys, const double *dinv,
                     const double *Q, double *R, double *pbb, double *prz, double *prr) {
    hipLaunchKernelGGL((k_residual<LPR, NV>), dim3(g.nb_pad), dim3(BLOCK), 0, s, g, sys->b_ptr,
                       sys->b_col, sys->b_val, dinv, Q, R, pbb, prz, prr);
}

__global__ void k_dinv(const double *d, int32_t n, double *dinv) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dinv[i] = 1.0 / d[i];
}

}  // namespace

// ---------------------------------------------------------------------------
// Workspace

struct zi_solver_ws {
    int ldp = 0, nrt_cap = 0;
    double *X = nullptr, *R = nullptr, *P = nullptr, *Q = nullptr, *dinv = nullptr;
    double *part[3] = {nullptr, nullptr, nullptr};
    double *sc_d = nullptr;     // rho alpha beta bb rr (5 ldp)
    int32_t *sc_i = nullptr;    // iters active (2 ldp) + flag
    std::vector<hipEvent_t> ev;
    zi::Pool pool;
    ~zi_solver_ws() {
        for (auto e : ev) (void)hipEventDestroy(e);
    }
};

void zi_solver_ws_destroy(zi_solver_ws *ws) { delete ws; }

int32_t zi_tile_count_impl() { return NTILES; }
const char *zi_tile_name_impl(int32_t t) {
    return (t >= 0 && t < NTILES) ? kTiles[t].name : "invalid";
}

namespace {

zi_status ensure_ws(zi_system *sys, int ldp, int nrt_max) {
    zi_solver_ws *ws = sys->ws;
    if (ws && ws->ldp == ldp && ws->nrt_cap >= nrt_max) return ZI_OK;
    if (ws) {
        delete ws;
        sys->ws = nullptr;
    }
    ws = new zi_solver_ws();
    const size_t blk = (size_t)sys->n * ldp;
    zi_status st = ZI_OK;
    if ((st = ws->pool.alloc(&ws->X, blk)) != ZI_OK || (st = ws->pool.alloc(&ws->R, blk)) != ZI_OK ||
        (st = ws->pool.alloc(&ws->P, blk)) != ZI_OK || (st = ws->pool.alloc(&ws->Q, blk)) != ZI_OK ||
        (st = ws->pool.alloc(&ws->dinv, (size_t)sys->n)) != ZI_OK ||
        (st = ws->pool.alloc(&ws->sc_d, (size_t)5 * ldp)) != ZI_OK ||
        (st = ws->pool.alloc(&ws->sc_i, (size_t)2 * ldp + 1)) != ZI_OK) {
        delete ws;
        return st;
    }
    for (int q = 0; q < 3; ++q) {
        if ((st = ws->pool.alloc(&ws->part[q], (size_t)nrt_max * ldp)) != ZI_OK) {
            delete ws;
            return st;
        }
    }
    ws->ldp = ldp;
    ws->nrt_cap = nrt_max;
    sys->ws = ws;
    return ZI_OK;
}

int max_nrt(int n, int ldp) {
    int m = 1;
    for (int t = 0; t < NTILES; ++t) {
        Geom g = make_geom(n, ldp, t);
        if (g.nrt > m) m = g.nrt;
    }
    return m;
}

struct EventTimer {
    std::vector<hipEvent_t> *pool;
    size_t used = 0;
    zi_status get(hipEvent_t *e) {
        if (used == pool->size()) {
            hipEvent_t x;
            ZI_HIP(hipEventCreate(&x));
            pool->push_back(x);
        }
        *e = (*pool)[used++];
        return ZI_OK;
    }
};

}  // namespace

zi_status zi_solve_impl(zi_system *sys, const zi_solve_opts *o, double *T, zi_solve_stats *st,
                        hipStream_t s) {
    const auto t_start = std::chrono::steady_clock::now();
    const int n = sys->n, L = sys->L;
    const int ldp = L + (L & 1);
    const double tol = o->tol > 0 ? o->tol : 1e-8;
    const double tol2 = tol * tol;
    const int maxit = o->maxit > 0 ? o->maxit : 50000;
    const int check = o->check_every > 0 ? o->check_every : 8;
    int tile = o->tile;
    if (tile < 0) tile = auto_tile(ldp);
    if (tile >= NTILES) {
        set_error("tile %d out of range", tile);
        return ZI_EINVAL;
    }
    if (o->precond != ZI_PREC_JACOBI && o->precond != ZI_PREC_LDP) {
        set_error("unknown preconditioner %d", o->precond);
        return ZI_EINVAL;
    }
    if (o->precision != ZI_FP64) {
        set_error("precision %d not available in this build", o->precision);
        return ZI_EINVAL;
    }
    const Geom g = make_geom(n, ldp, tile);
    ZI_TRY(ensure_ws(sys, ldp, max_nrt(n, ldp)));
    zi_solver_ws *ws = sys->ws;
    Scal sc;
    sc.rho = ws->sc_d;
    sc.alpha = ws->sc_d + ldp;
    sc.beta = ws->sc_d + 2 * ldp;
    sc.bb = ws->sc_d + 3 * ldp;
    sc.rr = ws->sc_d + 4 * ldp;
    sc.iters = ws->sc_i;
    sc.active = ws->sc_i + ldp;
    sc.flag = ws->sc_i + 2 * ldp;

    // preconditioner
    hipLaunchKernelGGL(k_dinv, dim3((n + 255) / 256), dim3(256), 0, s,
                       o->precond == ZI_PREC_LDP ? sys->absrow : sys->diag, n, ws->dinv);
    ZI_TRY(fill_i32(sc.flag, 0, 1, s));

    // X = x0 or 0; R = B - A X
    if (o->x0) {
        ZI_TRY(fill_f64(ws->X, 0.0, (size_t)n * ldp, s));
        ZI_TRY(copy_cols(o->x0, L, ws->X, ldp, n, L, s));
        ZI_TILE_SWITCH(tile, launch_spmm, g, s, sys, ws->X, ws->Q, (double *)nullptr);
    } else {
        ZI_TRY(fill_f64(ws->X, 0.0, (size_t)n * ldp, s));
    }
    ZI_TILE_SWITCH(tile, launch_residual, g, s, sys, ws->dinv, o->x0 ? ws->Q : nullptr, ws->R,
                   ws->part[0], ws->part[1], ws->part[2]);
    hipLaunchKernelGGL(k_red_init, dim3(ldp), dim3(RED), 0, s, sc, ws->part[0], ws->part[1],
                       ws->part[2], g.nrt, L, tol2);
    ZI_TILE_SWITCH(tile, launch_pupdate, g, s, (const double *)nullptr, ws->dinv, ws->R, ws->P);
    ZI_HIP(hipGetLastError());

    EventTimer timer{&ws->ev};
    std::vector<hipEvent_t> ev_spmm, ev_upd;
    const bool timing = o->timing != 0;

    std::vector<int32_t> h_active(ldp), h_iters(ldp);
    int32_t h_flag = 0;
    int it = 0;
    bool any_active = true;
    while (it < maxit) {
        hipEvent_t e0 = nullptr, e1 = nullptr, e2 = nullptr, e3 = nullptr;
        if (timing) {
            ZI_TRY(timer.get(&e0));
            ZI_TRY(timer.get(&e1));
            ZI_HIP(hipEventRecord(e0, s));
        }
        ZI_TILE_SWITCH(tile, launch_spmm, g, s, sys, ws->P, ws->Q, ws->part[0]);
        if (timing) ZI_HIP(hipEventRecord(e1, s));
        hipLaunchKernelGGL(k_red_alpha, dim3(ldp), dim3(RED), 0, s, sc, ws->part[0], g.nrt);
        if (timing) {
            ZI_TRY(timer.get(&e2));
            ZI_TRY(timer.get(&e3));
            ZI_HIP(hipEventRecord(e2, s));
        }
        ZI_TILE_SWITCH(tile, launch_update, g, s, sc.alpha, ws->dinv, ws->X, ws->R, ws->P, ws->Q,
                       ws->part[1], ws->part[2]);
        if (timing) {
            ZI_HIP(hipEventRecord(e3, s));
            ev_spmm.push_back(e0);
            ev_spmm.push_back(e1);
            ev_upd.push_back(e2);
            ev_upd.push_back(e3);
        }
        hipLaunchKernelGGL(k_red_beta, dim3(ldp), dim3(RED), 0, s, sc, ws->part[1], ws->part[2],
                           g.nrt, tol2);
        ZI_TILE_SWITCH(tile, launch_pupdate, g, s, sc.beta, ws->dinv, ws->R, ws->P);
        ZI_HIP(hipGetLastError());
        ++it;
        if (it % check == 0 || it == maxit) {
            ZI_HIP(hipMemcpyAsync(h_active.data(), sc.active, sizeof(int32_t) * ldp,
                                  hipMemcpyDeviceToHost, s));
            ZI_HIP(hipMemcpyAsync(&h_flag, sc.flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
            ZI_HIP(hipStreamSynchronize(s));
            any_active = false;
            for (int c = 0; c < ldp; ++c) any_active = any_active || h_active[c];
            if (h_flag || !any_active) break;
        }
    }
    if (it == 0) {
        ZI_HIP(hipMemcpyAsync(h_active.data(), sc.active, sizeof(int32_t) * ldp,
                              hipMemcpyDeviceToHost, s));
        ZI_HIP(hipStreamSynchronize(s));
        any_active = false;
        for (int c = 0; c < ldp; ++c) any_active = any_active || h_active[c];
    }

    // output and statistics
    ZI_TRY(copy_cols(ws->X, ldp, T, L, n, L, s));
    std::vector<double> h_rr(ldp), h_bb(ldp), h_true(ldp);
    ZI_HIP(hipMemcpyAsync(h_iters.data(), sc.iters, sizeof(int32_t) * ldp, hipMemcpyDeviceToHost, s));
    ZI_HIP(hipMemcpyAsync(h_rr.data(), sc.rr, sizeof(double) * ldp, hipMemcpyDeviceToHost, s));
    ZI_HIP(hipMemcpyAsync(h_bb.data(), sc.bb, sizeof(double) * ldp, hipMemcpyDeviceToHost, s));
    if (st && st->relres_true) {
        ZI_TILE_SWITCH(tile, launch_spmm, g, s, sys, ws->X, ws->Q, (double *)nullptr);
        ZI_TILE_SWITCH(tile, launch_residual, g, s, sys, ws->dinv, ws->Q, (double *)nullptr,
                       ws->part[0], ws->part[1], ws->part[2]);
        hipLaunchKernelGGL(k_red_sum, dim3(ldp), dim3(RED), 0, s, ws->part[2], g.nrt,
                           sc.alpha);   // alpha reused as scratch
        ZI_HIP(hipGetLastError());
        ZI_HIP(hipMemcpyAsync(h_true.data(), sc.alpha, sizeof(double) * ldp,
                              hipMemcpyDeviceToHost, s));
    }
    ZI_HIP(hipMemcpyAsync(&h_flag, sc.flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    ZI_HIP(hipStreamSynchronize(s));

    if (st) {
        for (int c = 0; c < L; ++c) {
            if (st->iters) st->iters[c] = h_iters[c];
            const double bn = h_bb[c] > 0 ? h_bb[c] : 1.0;
            if (st->relres_rec) st->relres_rec[c] = h_bb[c] > 0 ? std::sqrt(h_rr[c] / bn) : 0.0;
            if (st->relres_true) st->relres_true[c] = h_bb[c] > 0 ? std::sqrt(h_true[c] / bn) : 0.0;
        }
        st->block_iters = it;
        st->refinements = 0;
        st->tile = tile;
        st->n_kernels = 0;
        if (timing) {
            double ms_spmm = 0, ms_upd = 0;
            for (size_t k = 0; k + 1 < ev_spmm.size(); k += 2) {
                float a = 0, b = 0;
                ZI_HIP(hipEventElapsedTime(&a, ev_spmm[k], ev_spmm[k + 1]));
                ZI_HIP(hipEventElapsedTime(&b, ev_upd[k], ev_upd[k + 1]));
                ms_spmm += a;
                ms_upd += b;
            }
            const int64_t blk = (int64_t)n * ldp * 8;
            const int64_t abytes = (int64_t)sys->nnz * 12 + (int64_t)(n + 1) * 4;
            st->n_kernels = 2;
            st->kernel_name[0] = "spmm_pq";
            st->kernel_ms[0] = ms_spmm;
            st->kernel_launches[0] = (int32_t)(ev_spmm.size() / 2);
            st->kernel_bytes[0] = abytes + 2 * blk;            // read P, write Q
            st->kernel_name[1] = "update";
            st->kernel_ms[1] = ms_upd;
            st->kernel_launches[1] = (int32_t)(ev_upd.size() / 2);
            st->kernel_bytes[1] = 6 * blk + (int64_t)n * 8;    // r/w X, R; read P, Q; dinv
        }
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - t_start).count();
    }
    if (h_flag) {
        set_error("PCG breakdown: p^T A p <= 0 (matrix not positive definite)");
        return ZI_EBREAKDOWN;
    }
    if (any_active) {
        set_error("PCG did not reach tol %.3g within %d iterations", tol, maxit);
        return ZI_ENOTCONV;
    }
    return ZI_OK;
}

zi_status zi_spmm_impl(const zi_system *sys, int32_t k, const double *X, double *Y, int32_t tile,
                       double *ms, hipStream_t s) {
    if (k % 2 != 0) {
        set_error("zi_spmm needs an even number of columns (got %d)", k);
        return ZI_EINVAL;
    }
    if (tile < 0) tile = auto_tile(k);
    if (tile >= NTILES) {
        set_error("tile %d out of range", tile);
        return ZI_EINVAL;
    }
    const Geom g = make_geom(sys->n, k, tile);
    hipEvent_t e0, e1;
    ZI_HIP(hipEventCreate(&e0));
    ZI_HIP(hipEventCreate(&e1));
    ZI_HIP(hipEventRecord(e0, s));
    ZI_TILE_SWITCH(tile, launch_spmm, g, s, sys, X, Y, (double *)nullptr);
    ZI_HIP(hipGetLastError());
    ZI_HIP(hipEventRecord(e1, s));
    ZI_HIP(hipEventSynchronize(e1));
    float t = 0;
    ZI_HIP(hipEventElapsedTime(&t, e0, e1));
    if (ms) *ms = t;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ZI_OK;
}
