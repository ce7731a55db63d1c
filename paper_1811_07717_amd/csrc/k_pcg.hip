// Transfer matrix T = A^-1 B (App. A.4) by the diagonally preconditioned
// conjugate gradient of Sec. 2.3.1, run on all electrode columns at once.
//
// Every column runs its own PCG (its own alpha, beta, rho and stop test);
// the columns only share the sweeps over A.  Block vectors are n x ldp
// row-major (node-major) in the solver's row order, ldp = L rounded up to
// even; padding columns are zero and inactive.
//
// Two forms of the iteration.  Single-reduction (Chronopoulos-Gear, the FP64
// default), per iteration:
//   spmm_sr      S = A D^-1 R_k + beta S   + partials of delta = z.Az
//   red_alpha_sr alpha from gamma, delta and the previous alpha and beta
//   update       R_{k+1} = R_k - alpha S  + partials of r.D^-1 r, r.r
//   red_beta     stop test, beta
//   pflush       every 16 iterations: the lazy search directions and X
// Classic (and the mixed-precision mode, with float32 P, Q and R):
//   spmm_pq      Q = A P                  + partials of p.q
//   red_alpha, update (R -= alpha Q), red_beta, pupdate (P = D^-1 R + beta P),
//   and every 16 iterations xflush (X += the last 16 alpha P).
//
// Tiling: a wave holds 64/LPR rows; each lane owns NV column pairs (double2;
// the float32 products with two pairs per lane take four adjacent columns
// per lane when the width allows one 16-byte load per gathered row).
// A block (4 waves) owns rows of one column chunk of CW = 2 LPR NV columns.
// Blocks are numbered so that each of the 8 XCDs (block b runs on XCD b
// mod 8) receives contiguous rows: rows that share neighbours stay in one
// XCD's L2.  Schedules: chunk (a block per row range), cooperative front
// (the blocks of an XCD sweep its rows together, in slabs), and the LDS ring
// (a block per row range and 16-column chunk, the gathered rows in LDS).
// Reproducibility: every entry of a product is formed in CSR order whatever
// the tile; the SpMM's dot products are summed on fixed grids (exact in any
// grouping), the other kernels' in a fixed order with one fixed geometry, so
// T is bitwise the same for every tile and every run.
#include <algorithm>
#include <chrono>
#include <climits>
#include <cmath>
#include <cstring>
#include <mutex>
#include <type_traits>

#include "zi_internal.h"

namespace {

using namespace zi;

constexpr int BLOCK = 256;                         // threads per block
constexpr int WAVES = BLOCK / 64;                  // waves per block
constexpr int TARGET_BLOCKS = 2048 * 256 / BLOCK;  // row tiles x column chunks per launch

struct Geom {
    int n, ldp, ncc;      // rows, padded columns, column chunks
    int front;            // 0: each block owns a row chunk; 1: cooperative front
    int rb;               // chunk schedule: rows per block
    int P, B, U;          // front schedule: row parts, blocks per unit, units
    int nrt;              // partial-sum rows per column
    int nb, nb_pad;       // blocks (nb_pad: launched, a multiple of 8)
    int cl2n;             // ceil(log2 n): terms per column of a dot product
    int slabs;            // front schedule: launches per product, each over a slab of every
    int slab;             // row part (slab rows); the unit's blocks start each slab together
    int cur;              // the slab this launch covers
    const int32_t *gate;  // batched heads: 0 = the head has converged, launch does nothing
};

// Rows a block visits: base = rs + first + j * stride (base < re); the block's
// lanes take rows base + slot.  prow indexes the block's partial sums.
struct Sched {
    int cc, rs, re, first, stride, prow;
};

// Hardware block b runs on XCD b mod 8.  Blocks are numbered so that each XCD
// receives contiguous work:
//  * chunk schedule: logical tile (b mod 8) * nb_pad/8 + b/8 covers (column
//    chunk, row chunk) pairs in order, so an XCD gets consecutive rows;
//  * front schedule: each XCD owns units (column chunk, row part); the B
//    blocks of a unit walk its row range together as one front (block k takes
//    row groups k, k + B, ...), so rows that share neighbours are processed
//    close in time on the same XCD and their reuse stays in its L2.
template <int RSTEP>
__device__ __forceinline__ bool block_sched(const Geom &g, Sched &sc) {
    if (g.gate && *g.gate == 0) return false;   // the whole grid of a converged head
    const int b = blockIdx.x;
    if (!g.front) {
        const int per = g.nb_pad >> 3;
        const int logical = (b & 7) * per + (b >> 3);
        if (logical >= g.nb) return false;
        sc.cc = logical / g.nrt;
        const int rt = logical - sc.cc * g.nrt;
        sc.rs = rt * g.rb;
        sc.re = min(g.n, sc.rs + g.rb);
        sc.first = 0;
        sc.stride = RSTEP;
        sc.prow = rt;
        return true;
    }
    const int x = b & 7, j = b >> 3;
    const int m = j / g.B, k = j - m * g.B;
    const int u = x + 8 * m;
    if (u >= g.U) return false;
    sc.cc = u / g.P;
    const int pr = u - sc.cc * g.P;
    const int part = (g.n + g.P - 1) / g.P;
    const int pe = min(g.n, (pr + 1) * part);
    sc.rs = min(pe, pr * part + g.cur * g.slab);
    sc.re = min(pe, sc.rs + g.slab);
    sc.first = k * RSTEP;
    sc.stride = g.B * RSTEP;
    sc.prow = (g.cur * g.P + pr) * g.B + k;
    return true;
}

template <int LPR, int NV>
struct Lane {
    static constexpr int RPW = 64 / LPR;
    static constexpr int CW = 2 * LPR * NV;
    static constexpr int RSTEP = WAVES * RPW;
    int w, r, lr, slot;
    int c[NV];
    int cs[NV];   // c clamped into the padded columns (safe load address)
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
            cs[v] = ok[v] ? c[v] : 0;
        }
    }
};

// Pairs of block-vector entries: double2 (FP64 mode) or float2 (the float32
// search directions of the mixed-precision mode); arithmetic on pairs is
// written out component-wise through d2/f2 conversions.
__device__ __forceinline__ double2 ld2(const double *p) {
    return *reinterpret_cast<const double2 *>(p);
}
__device__ __forceinline__ void st2(double *p, double2 v) {
    *reinterpret_cast<double2 *>(p) = v;
}
__device__ __forceinline__ void st2(float *p, double2 v) {
    *reinterpret_cast<float2 *>(p) = make_float2((float)v.x, (float)v.y);
}
// Streaming (nontemporal) pair accesses for block vectors that a kernel
// touches once: each block vector is far larger than L2 and the Infinity
// Cache, and keeping it out of them leaves room for the SpMM's gathers.  Two
// adjacent scalar accesses become one 16-byte (8-byte) memory instruction.
typedef double dvec2 __attribute__((ext_vector_type(2)));
__device__ __forceinline__ double2 ldn2(const double *p) {
    const dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const dvec2 *>(p));
    return make_double2(v.x, v.y);
}
__device__ __forceinline__ double2 ldn2(const float *p) {
    return make_double2((double)__builtin_nontemporal_load(p),
                        (double)__builtin_nontemporal_load(p + 1));
}
__device__ __forceinline__ void stn2(double *p, double2 v) {
    __builtin_nontemporal_store(v.x, p);
    __builtin_nontemporal_store(v.y, p + 1);
}
__device__ __forceinline__ void stn2(float *p, double2 v) {
    __builtin_nontemporal_store((float)v.x, p);
    __builtin_nontemporal_store((float)v.y, p + 1);
}

// Column pairs of the SpMM.  Sums accumulate in the precision of the matrix
// values (Acc<TV>); the block vectors may be narrower (double values with
// float vectors widen on load and round on store).
template <class TV>
struct Acc;
template <>
struct Acc<double> {
    using type = double2;
    __device__ static double2 zero() { return make_double2(0.0, 0.0); }
};
template <>
struct Acc<float> {
    using type = float2;
    __device__ static float2 zero() { return make_float2(0.f, 0.f); }
};
__device__ __forceinline__ void ldpair(const double *p, double2 &v) {
    v = *reinterpret_cast<const double2 *>(p);
}
__device__ __forceinline__ void ldpair(const float *p, float2 &v) {
    v = *reinterpret_cast<const float2 *>(p);
}
__device__ __forceinline__ void stpair_nt(double *p, double2 v) { stn2(p, v); }
__device__ __forceinline__ void stpair_nt(float *p, double2 v) { stn2(p, v); }
__device__ __forceinline__ void stpair_nt(float *p, float2 v) {
    __builtin_nontemporal_store(v.x, p);
    __builtin_nontemporal_store(v.y, p + 1);
}
__device__ __forceinline__ double2 wide(double2 v) { return v; }
__device__ __forceinline__ double2 wide(float2 v) { return make_double2((double)v.x, (double)v.y); }
// v as a block vector of type TX stores it, in FP64
__device__ __forceinline__ double2 as_stored(double2 v, const double *) { return v; }
__device__ __forceinline__ double2 as_stored(double2 v, const float *) {
    return make_double2((double)(float)v.x, (double)(float)v.y);
}
__device__ __forceinline__ double2 as_stored(float2 v, const float *) { return wide(v); }

// Broadcast lane u of the LPR-lane row group (readlane when one row fills
// the wave, a cross-lane permute otherwise).
template <int LPR>
__device__ __forceinline__ int bcast(int v, int u) {
    if constexpr (LPR == 64)
        return __builtin_amdgcn_readlane(v, u);
    else
        return __shfl(v, u, LPR);
}
template <int LPR>
__device__ __forceinline__ float bcast(float v, int u) {
    if constexpr (LPR == 64)
        return __builtin_bit_cast(float, __builtin_amdgcn_readlane(__builtin_bit_cast(int, v), u));
    else
        return __shfl(v, u, LPR);
}
template <int LPR>
__device__ __forceinline__ double bcast(double v, int u) {
    if constexpr (LPR == 64) {
        const long long b = __builtin_bit_cast(long long, v);
        const int lo = __builtin_amdgcn_readlane((int)(b & 0xffffffffll), u);
        const int hi = __builtin_amdgcn_readlane((int)(b >> 32), u);
        return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
    } else {
        return __shfl(v, u, LPR);
    }
}

// acc = sum_k a_k X[j_k, c..c+1] over row `row`, in column order.  The row's
// (column, value) pairs are fetched BATCH at a time with one coalesced load
// (lane u of the group holds entry u) and broadcast, so all gathers of X for
// the batch are in flight together.  xs receives X[row, c..c+1] (the gather
// of the diagonal entry; self tells whether the row has one), which spares
// the dot product a second load of the row.  after_index() issues the
// caller's own loads for the row once the first batch's pairs are requested:
// a wave waits for its loads in issue order, so loads issued before the
// pairs would delay the gathers that depend on them.  A caller without such
// loads passes NoLoads, which keeps the batch loop in one piece (peeling the
// first batch slowed the one-pair float32 tile by a quarter).
struct NoLoads {
    __device__ void operator()() const {}
};
template <int LPR, int NV, class TV, class TX, class F>
__device__ __forceinline__ void row_product(const int32_t *__restrict__ rp,
                                            const int32_t *__restrict__ ci,
                                            const TV *__restrict__ va,
                                            const TX *__restrict__ X, int ldp, int row,
                                            int lr, const int c[NV], const bool ok[NV],
                                            typename Acc<TV>::type acc[NV],
                                            typename Acc<TX>::type xs[NV], bool &self,
                                            F &&after_index) {
    using XT = typename Acc<TX>::type;   // gathered pairs stay in storage precision
    constexpr int BATCH = LPR < 8 ? LPR : 8;
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[v] = Acc<TV>::zero();
    self = false;
    if constexpr (LPR == 64) {
        // one row per wave: the row's pointers and (column, value) pairs are
        // wave-uniform and come through scalar loads, whose waits are apart
        // from those of the vector loads and stores
        const int rw = __builtin_amdgcn_readfirstlane(row);
        const int s = rp[rw], e = rp[rw + 1];
        after_index();
        for (int kb = s; kb < e; kb += 8) {
            const int cnt = e - kb;
            int jj[8];
            TV a[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                const int k = min(kb + u, e - 1);
                jj[u] = ci[k];
                a[u] = va[k];
            }
            XT x[8][NV];
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    if (u < cnt && ok[v])
                        ldpair(X + (size_t)jj[u] * ldp + c[v], x[u][v]);
                    else
                        x[u][v] = Acc<TX>::zero();
                }
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                if (u < cnt) {
#pragma unroll
                    for (int v = 0; v < NV; ++v) {
                        acc[v].x = fma(a[u], (TV)x[u][v].x, acc[v].x);
                        acc[v].y = fma(a[u], (TV)x[u][v].y, acc[v].y);
                    }
                    if (jj[u] == rw) {
                        self = true;
#pragma unroll
                        for (int v = 0; v < NV; ++v) xs[v] = x[u][v];
                    }
                }
            }
        }
        return;
    }
    constexpr bool PEEL = !std::is_same<std::decay_t<F>, NoLoads>::value;
    const int s = rp[row], e = rp[row + 1];
    // the first batch's (column, value) pairs, then the caller's loads
    int jv = row;
    TV av = TV(0);
    if (PEEL) {
        if (lr < BATCH && lr < e - s) {
            jv = __builtin_nontemporal_load(ci + s + lr);
            av = __builtin_nontemporal_load(va + s + lr);
        }
        after_index();
    }
    for (int kb = s; kb < e; kb += BATCH) {
        const int cnt = e - kb;
        if (!PEEL || kb != s) {
            jv = row;
            av = TV(0);
            if (lr < BATCH && lr < cnt) {
                jv = __builtin_nontemporal_load(ci + kb + lr);
                av = __builtin_nontemporal_load(va + kb + lr);
            }
        }
        XT x[BATCH][NV];
        int jj[BATCH];
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            jj[u] = bcast<LPR>(jv, u);
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                if (u < cnt && ok[v])
                    ldpair(X + (size_t)jj[u] * ldp + c[v], x[u][v]);
                else
                    x[u][v] = Acc<TX>::zero();
            }
        }
#pragma unroll
        for (int u = 0; u < BATCH; ++u) {
            const TV a = bcast<LPR>(av, u);
            if (u < cnt) {
#pragma unroll
                for (int v = 0; v < NV; ++v) {
                    acc[v].x = fma(a, (TV)x[u][v].x, acc[v].x);
                    acc[v].y = fma(a, (TV)x[u][v].y, acc[v].y);
                }
                if (jj[u] == row) {
                    self = true;
#pragma unroll
                    for (int v = 0; v < NV; ++v) xs[v] = x[u][v];
                }
            }
        }
    }
}

// Sum NQ per-lane partials over the block's rows (fixed order) and store them
// column-major: part[q][col * nrt + rt].
template <int LPR, int NV, int NQ>
__device__ __forceinline__ void block_partials(const Geom &g, const Lane<LPR, NV> &ln, int cc,
                                               int prow, const double2 (&acc)[NQ][NV],
                                               double *const (&part)[NQ], bool quad = false) {
    constexpr int RS = Lane<LPR, NV>::RSTEP;
    constexpr int CW = Lane<LPR, NV>::CW;
    __shared__ double red[NQ][RS][CW];
#pragma unroll
    for (int q = 0; q < NQ; ++q)
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            const int cl = quad ? 4 * ln.lr + 2 * v : 2 * (ln.lr + LPR * v);
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
            part[q][(size_t)col * g.nrt + prow] = s;
        }
    }
}

// Dot products of the SpMM whose value does not depend on how rows are
// grouped into partial sums (the tile, the block that took a row).  Every
// term t is pre-rounded on two fixed grids (the extraction of Demmel and
// Nguyen's reproducible summation): with a per-column bound on the sum of
// |t| (2^e >= bound), m1 = 1.5 2^(e+1) and m2 = m1 2^(ceil(log2 n)-52),
// q1 = (m1 + t) - m1 is t on the grid ulp(m1), q2 = (m2 + r) - m2 the rest
// r = t - q1 on the grid ulp(m2).  Sums of up to n such values stay exact in
// FP64, so the two fold sums are the same in any order; the dot is their sum.
// The dropped remainder is at most n ulp(m2) / 2 = 2^-60 bound for n <= 2^22.
__device__ __forceinline__ double fold_grid(double bound) {
    int e = 0;
    (void)frexp(bound > 1e-280 ? bound : 1e-280, &e);   // bound <= 2^e
    return ldexp(1.5, e + 1);
}

// m2 = m1 f2 with f2 = 2^(ceil(log2 n) - 52), the same for every column.
__device__ __forceinline__ void fold_add(double u, double v, double m1, double f2, double &s1,
                                         double &s2) {
#pragma clang fp contract(off)
    const double t = u * v;
    const double m2 = m1 * f2;
    const double q1 = (m1 + t) - m1;
    const double r = t - q1;
    const double q2 = (m2 + r) - m2;
    s1 = s1 + q1;
    s2 = s2 + q2;
}

// The rows a block's lanes process, calling f(row) for each: rows base + slot
// with base = rs + first + j stride.
template <int LPR, int NV, class F>
__device__ __forceinline__ void for_rows(const Sched &sc, const Lane<LPR, NV> &ln, F &&f) {
    for (int base = sc.rs + sc.first; base < sc.re; base += sc.stride) {
        const int row = base + ln.slot;
        if (row < sc.re) f(row);
    }
}

// Rows of a float32 SpMM with two column pairs per lane, when the padded
// width is a multiple of 4: lane lr owns the four adjacent columns
// c0 = cc CW + 4 lr .. c0 + 3 and gathers them with one 16-byte load (the
// pair layout needs two 8-byte loads per row).  Products, their order and
// the dot terms are those of row_product; the partials use the quad map.
typedef float fvec4 __attribute__((ext_vector_type(4)));
template <int LPR, class TV, bool WITH_DOT>
__device__ __forceinline__ void spmm_rows_quad(const Geom &g, const Sched &sc,
                                               const Lane<LPR, 2> &ln,
                                               const int32_t *__restrict__ rp,
                                               const int32_t *__restrict__ ci,
                                               const TV *__restrict__ va,
                                               const float *__restrict__ X,
                                               float *__restrict__ Y, const double *m1,
                                               double f2, double2 (&dotacc)[2][2]) {
    using AT = typename Acc<TV>::type;
    constexpr int BATCH = LPR < 8 ? LPR : 8;
    constexpr int CW = Lane<LPR, 2>::CW;
    const int lr = ln.lr;
    const int c0 = sc.cc * CW + 4 * lr;
    const bool ok = c0 < g.ldp;
    for_rows<LPR, 2>(sc, ln, [&](int row) {
        AT acc[2] = {Acc<TV>::zero(), Acc<TV>::zero()};
        fvec4 xs = {0.f, 0.f, 0.f, 0.f};
        bool self = false;
        const int s = rp[row], e = rp[row + 1];
        for (int kb = s; kb < e; kb += BATCH) {
            const int cnt = e - kb;
            int jv = row;
            TV av = TV(0);
            if (lr < BATCH && lr < cnt) {
                jv = __builtin_nontemporal_load(ci + kb + lr);
                av = __builtin_nontemporal_load(va + kb + lr);
            }
            fvec4 x[BATCH];
            int jj[BATCH];
#pragma unroll
            for (int u = 0; u < BATCH; ++u) {
                jj[u] = bcast<LPR>(jv, u);
                if (u < cnt && ok)
                    x[u] = *reinterpret_cast<const fvec4 *>(X + (size_t)jj[u] * g.ldp + c0);
                else
                    x[u] = fvec4{0.f, 0.f, 0.f, 0.f};
            }
#pragma unroll
            for (int u = 0; u < BATCH; ++u) {
                const TV a = bcast<LPR>(av, u);
                if (u < cnt) {
                    acc[0].x = fma(a, (TV)x[u].x, acc[0].x);
                    acc[0].y = fma(a, (TV)x[u].y, acc[0].y);
                    acc[1].x = fma(a, (TV)x[u].z, acc[1].x);
                    acc[1].y = fma(a, (TV)x[u].w, acc[1].y);
                    if (jj[u] == row) {
                        self = true;
                        xs = x[u];
                    }
                }
            }
        }
        if (!ok) return;
        float *y = Y + (size_t)row * g.ldp + c0;
        const fvec4 q4 = {(float)acc[0].x, (float)acc[0].y, (float)acc[1].x, (float)acc[1].y};
        if (WITH_DOT) {
            fvec4 xr = xs;
            if (!self) xr = *reinterpret_cast<const fvec4 *>(X + (size_t)row * g.ldp + c0);
            const int cl = 4 * lr;
            fold_add((double)xr.x, (double)q4.x, m1[cl], f2, dotacc[0][0].x, dotacc[1][0].x);
            fold_add((double)xr.y, (double)q4.y, m1[cl + 1], f2, dotacc[0][0].y, dotacc[1][0].y);
            fold_add((double)xr.z, (double)q4.z, m1[cl + 2], f2, dotacc[0][1].x, dotacc[1][1].x);
            fold_add((double)xr.w, (double)q4.w, m1[cl + 3], f2, dotacc[0][1].y, dotacc[1][1].y);
        }
        __builtin_nontemporal_store(q4, reinterpret_cast<fvec4 *>(y));
    });
}

// ---------------------------------------------------------------------------

// Y = A X; with WITH_DOT also the partials of sum_i X[i,c] Y[i,c] (in FP64,
// with Y as stored).
// Three waves per SIMD for the SpMMs of up to two column pairs per lane (the
// gathers need waves in flight more than registers).
template <int NV>
constexpr int spmm_waves() { return NV <= 2 ? 3 : 1; }

template <int LPR, int NV, class TV, class TX, bool WITH_DOT>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(spmm_waves<NV>())))
void k_spmm(Geom g, const int32_t *__restrict__ rp,
                                                const int32_t *__restrict__ ci,
                                                const TV *__restrict__ va,
                                                const TX *__restrict__ X, TX *__restrict__ Y,
                                                double *part, const double *__restrict__ bound) {
    using AT = typename Acc<TV>::type;
    using XT = typename Acc<TX>::type;
    Sched sc;
    if (!block_sched<Lane<LPR, NV>::RSTEP>(g, sc)) return;
    Lane<LPR, NV> ln(g, sc.cc);
    constexpr int CW = Lane<LPR, NV>::CW;
    __shared__ double m1[WITH_DOT ? CW : 1];   // first fold grid of the chunk's columns
    double2 dotacc[2][NV];                     // the two fold sums
    const double f2 = ldexp(1.0, g.cl2n - 52);
#pragma unroll
    for (int v = 0; v < NV; ++v) dotacc[0][v] = dotacc[1][v] = make_double2(0.0, 0.0);
    if (WITH_DOT) {
        for (int i = threadIdx.x; i < CW; i += BLOCK) {
            const int col = sc.cc * CW + i;
            m1[i] = col < g.ldp ? fold_grid(bound[col]) : 0.0;
        }
        __syncthreads();
    }
    bool quad = false;
    if constexpr (std::is_same<TX, float>::value && NV == 2) {
        if ((g.ldp & 3) == 0 &&
            ((reinterpret_cast<uintptr_t>(X) | reinterpret_cast<uintptr_t>(Y)) & 15) == 0) {
            quad = true;
            spmm_rows_quad<LPR, TV, WITH_DOT>(g, sc, ln, rp, ci, va, X, Y, m1, f2, dotacc);
        }
    }
    if (!quad) for_rows<LPR, NV>(sc, ln, [&](int row) {
        AT acc[NV];
        XT xs[NV];
        bool self;
        row_product<LPR, NV, TV, TX>(rp, ci, va, X, g.ldp, row, ln.lr, ln.c, ln.ok, acc, xs, self,
                                     NoLoads{});
        // Dot terms (and the load of a row without a diagonal entry) before
        // the stores: one counter tracks a wave's loads and stores in flight,
        // so waiting for a load issued after a store waits for the store too.
        if (WITH_DOT) {
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                if (!ln.ok[v]) continue;
                XT xr = xs[v];
                if (!self) ldpair(X + (size_t)row * g.ldp + ln.c[v], xr);
                const double2 p = wide(xr);
                const double2 q = as_stored(acc[v], (const TX *)Y);
                const int cl = 2 * (ln.lr + LPR * v);
                fold_add(p.x, q.x, m1[cl], f2, dotacc[0][v].x, dotacc[1][v].x);
                fold_add(p.y, q.y, m1[cl + 1], f2, dotacc[0][v].y, dotacc[1][v].y);
            }
        }
#pragma unroll
        for (int v = 0; v < NV; ++v)
            if (ln.ok[v]) stpair_nt(Y + (size_t)row * g.ldp + ln.c[v], acc[v]);
    });
    if (WITH_DOT) {
        double *const parts[2] = {part, part + (size_t)g.nrt * g.ldp};
        block_partials<LPR, NV, 2>(g, ln, sc.cc, sc.prow, dotacc, parts, quad);
    }
}

// SpMM of the single-reduction PCG (FP64): W = A D^-1 R through the values
// vs = a_ij / d_j, then S = W + beta S in place, and the partials of
// delta = sum_i (D^-1 R)[i,c] W[i,c] (R of the own row comes from the gather
// of the diagonal entry).  beta == nullptr: S = W.
template <int LPR, int NV>
__global__ __launch_bounds__(BLOCK) __attribute__((amdgpu_waves_per_eu(spmm_waves<NV>())))
void k_spmm_sr(Geom g, const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci,
                                                   const double *__restrict__ vs,
                                                   const double *__restrict__ dinv,
                                                   const double *__restrict__ R,
                                                   const double *__restrict__ beta,
                                                   double *__restrict__ S, double *part,
                                                   const double *__restrict__ bound) {
    Sched sc;
    if (!block_sched<Lane<LPR, NV>::RSTEP>(g, sc)) return;
    Lane<LPR, NV> ln(g, sc.cc);
    double2 be[NV];
    constexpr int CW = Lane<LPR, NV>::CW;
    __shared__ double m1[CW];   // first fold grid of the chunk's columns
    double2 dotacc[2][NV];      // the two fold sums
    const double f2 = ldexp(1.0, g.cl2n - 52);
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        be[v] = (ln.ok[v] && beta) ? ld2(beta + ln.c[v]) : make_double2(0.0, 0.0);
        dotacc[0][v] = dotacc[1][v] = make_double2(0.0, 0.0);
    }
    for (int i = threadIdx.x; i < CW; i += BLOCK) {
        const int col = sc.cc * CW + i;
        m1[i] = col < g.ldp ? fold_grid(bound[col]) : 0.0;
    }
    __syncthreads();
    for_rows<LPR, NV>(sc, ln, [&](int row) {
        // the row's S entries and D^-1 are requested after its column
        // indices and before its gathers
        double2 so[NV];
        double di;
        double2 acc[NV], xs[NV];
        bool self;
        row_product<LPR, NV, double, double>(
            rp, ci, vs, R, g.ldp, row, ln.lr, ln.c, ln.ok, acc, xs, self, [&] {
#pragma unroll
                for (int v = 0; v < NV; ++v)
                    so[v] = (ln.ok[v] && beta) ? ldn2(S + (size_t)row * g.ldp + ln.c[v])
                                               : make_double2(0.0, 0.0);
                di = dinv[row];
            });
        // Dot terms (and the load of a row without a diagonal entry) before
        // the stores: one counter tracks a wave's loads and stores in flight,
        // so waiting for a load issued after a store waits for the store too.
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (!ln.ok[v]) continue;
            double2 xr = xs[v];
            if (!self) xr = ld2(R + (size_t)row * g.ldp + ln.c[v]);
            const int cl = 2 * (ln.lr + LPR * v);
            fold_add(xr.x * di, acc[v].x, m1[cl], f2, dotacc[0][v].x, dotacc[1][v].x);
            fold_add(xr.y * di, acc[v].y, m1[cl + 1], f2, dotacc[0][v].y, dotacc[1][v].y);
        }
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (!ln.ok[v]) continue;
            double2 sn;
            sn.x = fma(be[v].x, so[v].x, acc[v].x);
            sn.y = fma(be[v].y, so[v].y, acc[v].y);
            stn2(S + (size_t)row * g.ldp + ln.c[v], sn);
        }
    });
    double *const parts[2] = {part, part + (size_t)g.nrt * g.ldp};
    block_partials<LPR, NV, 2>(g, ln, sc.cc, sc.prow, dotacc, parts);
}

// Ring SpMM of the single-reduction PCG: the same products and dot partials
// as k_spmm_sr, with the gathered rows of R served from LDS.
//
// Each block sweeps one contiguous range of solver rows for one 16-column
// chunk, RING_G rows per step.  The rows [s - RING_H, s + RING_G + RING_H)
// around step s stay in an LDS ring (in the solver order every mesh
// neighbour of a row lies within a pencil layer, at most RING_H rows away,
// except across the pencil's side faces), and the rows that the step's rows
// reference outside that window -- the side-face neighbours, listed per step
// by k_ring_halo -- are staged in LDS beside it.  While a step is computed
// from LDS, the next step's new ring rows, halo rows, matrix entries, S and
// D^-1 are already on their way into registers; the indices they depend on
// (row pointers, halo lists) are fetched one step earlier still.  A
// reference found in neither (a halo list cut at RING_HMAX rows) is gathered
// from memory.  Each entry of A D^-1 R is formed in CSR order with the same
// fused multiply-adds as in k_spmm_sr, and delta is summed on the fold
// grids, so S and the dot products are bitwise those of every other tile.
constexpr int RING_RPL = 2;                         // rows per lane group per step
constexpr int RING_HPL = 3;                         // halo rows per lane group per step
constexpr int RING_G = 32 * RING_RPL;               // rows per step (32 lane groups)
constexpr int RING_H = 64;                          // window reach below and above a step
constexpr int RING_ROWS = RING_G + 2 * RING_H;      // rows held in the LDS ring
constexpr int RING_HMAX = 32 * RING_HPL;            // halo rows staged per step
constexpr int RING_HSEARCH = 128;                   // halo list in LDS, padded to a power of 2
constexpr int RING_SORT = 1024;                     // halo candidates sorted per step
static_assert(RING_HMAX <= RING_HSEARCH, "halo search");

// Halo list of every step: the distinct columns, ascending, that rows
// [s, s + RING_G) reference outside [s - RING_H, s + RING_G + RING_H); the
// first RING_HMAX of them, the rest of the list INT_MAX.  slow[step] = 1
// where the list was cut or a row has more than 8 entries: such steps take
// the ring kernel's path that reads memory inside the row loop.  One block
// per step.
__global__ __launch_bounds__(256) void k_ring_halo(const int32_t *__restrict__ rp,
                                                   const int32_t *__restrict__ ci, int n,
                                                   int32_t *__restrict__ halo,
                                                   int32_t *__restrict__ slow) {
    static_assert(RING_G * 4 <= 256 * 1, "one thread quarter per row");
    __shared__ int list[RING_SORT];
    __shared__ int cnt, longrow;
    const int step = blockIdx.x;
    const int s0 = step * RING_G;
    if (threadIdx.x == 0) cnt = longrow = 0;
    __syncthreads();
    const int row = s0 + (int)(threadIdx.x >> 2);
    if (row < n && (int)(threadIdx.x >> 2) < RING_G) {
        if ((threadIdx.x & 3) == 0 && rp[row + 1] - rp[row] > 8) longrow = 1;
        const int lo = s0 - RING_H, hi = s0 + RING_G + RING_H;
        for (int q = rp[row] + (int)(threadIdx.x & 3); q < rp[row + 1]; q += 4) {
            const int col = ci[q];
            if (col < lo || col >= hi) {
                const int p = atomicAdd(&cnt, 1);
                if (p < RING_SORT) list[p] = col;
            }
        }
    }
    __syncthreads();
    const int m = min(cnt, RING_SORT);
    for (int i = threadIdx.x; i < RING_SORT; i += blockDim.x)
        if (i >= m) list[i] = INT_MAX;
    __syncthreads();
    for (int k = 2; k <= RING_SORT; k <<= 1)        // bitonic sort, ascending
        for (int j = k >> 1; j > 0; j >>= 1) {
            for (int i = threadIdx.x; i < RING_SORT; i += blockDim.x) {
                const int l = i ^ j;
                if (l > i) {
                    const int x = list[i], y = list[l];
                    if ((x > y) == ((i & k) == 0)) {
                        list[i] = y;
                        list[l] = x;
                    }
                }
            }
            __syncthreads();
        }
    if (threadIdx.x == 0) {
        int32_t *h = halo + (size_t)step * RING_HMAX;
        int out = 0, cut = cnt > RING_SORT;
        for (int i = 0; i < m; ++i)
            if (i == 0 || list[i] != list[i - 1]) {
                if (out == RING_HMAX) {
                    cut = 1;
                    break;
                }
                h[out++] = list[i];
            }
        for (; out < RING_HMAX; ++out) h[out] = INT_MAX;
        slow[step] = cut || longrow;
    }
}

// A lane of the ring SpMM owns 16 bytes of a row's chunk: RingT<TX>::CPL
// columns of the block vector type TX, kept in LDS and in registers as the
// raw 16 bytes (a double2, or four floats in a double2's bits).
template <class TX>
struct RingT;
template <>
struct RingT<double> {
    static constexpr int CPL = 2;
};
template <>
struct RingT<float> {
    static constexpr int CPL = 4;
};

// The lane's 16 bytes of row `row` (columns c.. of the chunk), 0 where the
// lane or the row lies outside the block.  Columns come in pairs (ldp is
// even), so a lane whose last pair lies past ldp loads only its first.
template <class TX>
__device__ __forceinline__ double2 ring_row(const TX *__restrict__ X, int row, int n, int ldp,
                                            int c, bool ok) {
    double2 v = make_double2(0.0, 0.0);
    if (!(ok && row >= 0 && row < n)) return v;
    const TX *p = X + (size_t)row * ldp + c;
    if constexpr (sizeof(TX) == 8) {
        v = ld2(p);
    } else {
        const float2 a = *reinterpret_cast<const float2 *>(p);
        const float2 b = c + 2 < ldp ? *reinterpret_cast<const float2 *>(p + 2)
                                     : make_float2(0.f, 0.f);
        v = make_double2(__builtin_bit_cast(double, a), __builtin_bit_cast(double, b));
    }
    return v;
}

// The lane's columns of a 16-byte unit, widened to double.
template <class TX>
__device__ __forceinline__ void ring_cols(double2 v, double (&x)[RingT<TX>::CPL]) {
    if constexpr (sizeof(TX) == 8) {
        x[0] = v.x;
        x[1] = v.y;
    } else {
        const float2 a = __builtin_bit_cast(float2, v.x), b = __builtin_bit_cast(float2, v.y);
        x[0] = a.x;
        x[1] = a.y;
        x[2] = b.x;
        x[3] = b.y;
    }
}

// X[col, chunk] for the ring SpMM at a step whose window starts at lo: from
// the ring when col lies in the window, else from the staged halo rows
// (lower bound in the sorted, INT_MAX-padded halo list), else from memory.
template <class TX>
__device__ __forceinline__ double2 ring_fetch(const double2 (*ring)[8], const double2 (*hrow)[8],
                                              const int *hidx, const TX *__restrict__ X, int col,
                                              int lo, int pr, int n, int ldp, int c, bool ok) {
    if ((unsigned)(col - lo) < (unsigned)RING_ROWS) return ring[col % RING_ROWS][pr];
    int p = 0;
#pragma unroll
    for (int w = RING_HSEARCH / 2; w > 0; w >>= 1)
        if (hidx[p + w - 1] < col) p += w;
    if (hidx[p] == col) return hrow[p][pr];
    return ring_row(X, col, n, ldp, c, ok);
}

// The same where every reference is known to be in the window or the halo.
__device__ __forceinline__ double2 ring_fetch_staged(const double2 (*ring)[8],
                                                     const double2 (*hrow)[8], const int *hidx,
                                                     int col, int lo, int pr) {
    if ((unsigned)(col - lo) < (unsigned)RING_ROWS) return ring[col % RING_ROWS][pr];
    int p = 0;
#pragma unroll
    for (int w = RING_HSEARCH / 2; w > 0; w >>= 1)
        if (hidx[p + w - 1] < col) p += w;
    return hrow[p][pr];
}

// The next step's loads of one lane: matrix entry (lane pr of the row's
// group holds entry pr), D^-1 and the old S of each of its rows.
template <int CPL>
struct RingRows {
    int ci[RING_RPL];
    double va[RING_RPL], di[RING_RPL];
    double s[RING_RPL][CPL];
    int rp[RING_RPL][2];
};

// Ring SpMM in two forms, on block vectors of type TX (16 columns of double
// or 32 of float per chunk):
//   SR (single-reduction PCG, FP64): Y = A D^-1 X + beta Y in place with the
//      values a_ij / d_j, and the partials of delta = sum (D^-1 X) . W;
//   !SR (classic PCG): Y = A X with the values a_ij, and the partials of
//      sum X . Y with X and Y as stored.
// Block b runs on XCD b mod 8; the ncc chunk blocks of one row range are
// numbered consecutively on one XCD, so that they run together and share
// the range's matrix entries (and halo rows) in that XCD's L2.
template <class TX, bool SR>
__global__ __launch_bounds__(BLOCK) void k_spmm_ring(Geom g, const int32_t *__restrict__ halo,
                                                     const int32_t *__restrict__ slow,
                                                     const int32_t *__restrict__ rp,
                                                     const int32_t *__restrict__ ci,
                                                     const double *__restrict__ vals,
                                                     const double *__restrict__ dinv,
                                                     const TX *__restrict__ X,
                                                     const double *__restrict__ beta,
                                                     TX *__restrict__ Y, double *part,
                                                     const double *__restrict__ bound) {
    constexpr int CPL = RingT<TX>::CPL;
    constexpr int CW = 8 * CPL;                 // chunk width
    static_assert(!SR || sizeof(TX) == 8, "the single-reduction form is FP64");
    static_assert(2 * 32 * CW * sizeof(double) <= RING_ROWS * 8 * sizeof(double2),
                  "the ring doubles as the partial-sum buffer");
    if (g.gate && *g.gate == 0) return;
    const int bx = blockIdx.x;
    const int j = bx >> 3;
    const int cc = j % g.ncc;
    const int range = (j / g.ncc) * 8 + (bx & 7);
    if (range >= g.nrt) return;
    const int a = range * g.rb;                 // a multiple of RING_G
    const int e = min(g.n, a + g.rb);
    const int n = g.n, ldp = g.ldp;
    const int rl = threadIdx.x >> 3, pr = threadIdx.x & 7;   // lane group (rows rl + 32 k), unit
    const int c = cc * CW + CPL * pr;           // the lane's first column
    const bool ok = c < ldp;

    __shared__ double2 ring[RING_ROWS][8];
    __shared__ double2 hrow[RING_HMAX][8];
    __shared__ int hidx[RING_HSEARCH];
    __shared__ double m1[CW];                   // first fold grid of the chunk's columns
    const double f2 = ldexp(1.0, g.cl2n - 52);
    double be[CPL];
#pragma unroll
    for (int u = 0; u < CPL; ++u) be[u] = (SR && beta && c + u < ldp) ? beta[c + u] : 0.0;

    // loads of step t's entries, D^-1 and S (row pointers already known)
    auto load_rows = [&](int t, RingRows<CPL> &q) {
#pragma unroll
        for (int k = 0; k < RING_RPL; ++k) {
            q.ci[k] = 0;
            q.va[k] = 0.0;
            q.di[k] = 0.0;
#pragma unroll
            for (int u = 0; u < CPL; ++u) q.s[k][u] = 0.0;
            const int row = t + rl + 32 * k;
            if (row < e) {
                if (pr < q.rp[k][1] - q.rp[k][0]) {
                    q.ci[k] = ci[q.rp[k][0] + pr];
                    q.va[k] = vals[q.rp[k][0] + pr];
                }
                if constexpr (SR) {
                    q.di[k] = dinv[row];
                    if (ok && beta) {
                        const double2 v = ldn2(Y + (size_t)row * ldp + c);
                        q.s[k][0] = v.x;
                        q.s[k][1] = v.y;
                    }
                }
            }
        }
    };
    auto load_rp = [&](int t, int (&r)[RING_RPL][2]) {
#pragma unroll
        for (int k = 0; k < RING_RPL; ++k) {
            const int row = min(t + rl + 32 * k, n);
            r[k][0] = rp[row];
            r[k][1] = rp[min(row + 1, n)];
        }
    };

    // window and halo of the first step
    if (threadIdx.x < CW) {
        const int col = cc * CW + threadIdx.x;
        m1[threadIdx.x] = col < ldp ? fold_grid(bound[col]) : 0.0;
    }
    for (int i = threadIdx.x; i < RING_ROWS * 8; i += BLOCK) {
        const int row = a - RING_H + (i >> 3);
        if (row >= 0) {
            const int cu = cc * CW + CPL * (i & 7);
            ring[row % RING_ROWS][i & 7] = ring_row(X, row, n, ldp, cu, cu < ldp);
        }
    }
    for (int i = threadIdx.x; i < RING_HSEARCH; i += BLOCK)
        hidx[i] = i < RING_HMAX ? halo[(size_t)(a / RING_G) * RING_HMAX + i] : INT_MAX;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < RING_HPL; ++k) {
        const int h = hidx[rl + 32 * k];
        hrow[rl + 32 * k][pr] = ring_row(X, h != INT_MAX ? h : -1, n, ldp, c, ok);
    }
    RingRows<CPL> cur, nxt;
    load_rp(a, cur.rp);
    load_rp(a + RING_G, nxt.rp);
    load_rows(a, cur);
    int hi_n[RING_HPL];                          // halo indices of the next step
#pragma unroll
    for (int k = 0; k < RING_HPL; ++k)
        hi_n[k] = a + RING_G < e ? halo[(size_t)(a / RING_G + 1) * RING_HMAX + rl + 32 * k]
                                 : INT_MAX;
    int slow_c = slow[a / RING_G];               // this step's and the next step's path
    int slow_n = a + RING_G < e ? slow[a / RING_G + 1] : 0;
    __syncthreads();

    double dot0[CPL], dot1[CPL];                 // the two fold sums of the dot product
#pragma unroll
    for (int u = 0; u < CPL; ++u) dot0[u] = dot1[u] = 0.0;
    for (int s = a; s < e; s += RING_G) {
        const int t = s + RING_G;               // the next step
        const bool has_t = t < e;
        // next step: new ring rows, halo rows, entries, S, D^-1; the step
        // after: row pointers, halo indices and path
        double2 rn[RING_RPL], hn[RING_HPL];
        int hi_nn[RING_HPL], rp_nn[RING_RPL][2], slow_nn = 0;
#pragma unroll
        for (int k = 0; k < RING_RPL; ++k) {
            rn[k] = make_double2(0.0, 0.0);
            rp_nn[k][0] = rp_nn[k][1] = 0;
        }
#pragma unroll
        for (int k = 0; k < RING_HPL; ++k) {
            hn[k] = make_double2(0.0, 0.0);
            hi_nn[k] = INT_MAX;
        }
        if (has_t) {
#pragma unroll
            for (int k = 0; k < RING_RPL; ++k)
                rn[k] = ring_row(X, t + RING_H + rl + 32 * k, n, ldp, c, ok);
#pragma unroll
            for (int k = 0; k < RING_HPL; ++k)
                hn[k] = ring_row(X, hi_n[k] != INT_MAX ? hi_n[k] : -1, n, ldp, c, ok);
            load_rows(t, nxt);
            const int u = t + RING_G;
            if (u < e) {
#pragma unroll
                for (int k = 0; k < RING_HPL; ++k)
                    hi_nn[k] = halo[(size_t)(u / RING_G) * RING_HMAX + rl + 32 * k];
                slow_nn = slow[u / RING_G];
            }
            load_rp(u, rp_nn);
        }

        // this step, from LDS: rows of up to 8 entries whose references are
        // all staged take the path that reads no memory (the entries and S
        // came in with the previous step); the others read their entries
        // and unstaged references inside the row loop
        const int lo = s - RING_H;
#pragma unroll
        for (int k = 0; k < RING_RPL; ++k) {
            const int row = s + rl + 32 * k;
            if (row >= e) continue;
            double acc[CPL];
#pragma unroll
            for (int u = 0; u < CPL; ++u) acc[u] = 0.0;
            if (!slow_c) {
                const int cnt = cur.rp[k][1] - cur.rp[k][0];
                for (int q = 0; q < cnt; ++q) {
                    const int col = __shfl(cur.ci[k], q, 8);
                    const double av = __shfl(cur.va[k], q, 8);
                    double xv[CPL];
                    ring_cols<TX>(ring_fetch_staged(ring, hrow, hidx, col, lo, pr), xv);
#pragma unroll
                    for (int u = 0; u < CPL; ++u) acc[u] = fma(av, xv[u], acc[u]);
                }
            } else {
                for (int q = cur.rp[k][0]; q < cur.rp[k][1]; ++q) {
                    const int col = ci[q];
                    const double av = vals[q];
                    double xv[CPL];
                    ring_cols<TX>(ring_fetch(ring, hrow, hidx, X, col, lo, pr, n, ldp, c, ok), xv);
#pragma unroll
                    for (int u = 0; u < CPL; ++u) acc[u] = fma(av, xv[u], acc[u]);
                }
            }
            if (ok) {
                double xs[CPL];                 // the row itself lies in the window
                ring_cols<TX>(ring[row % RING_ROWS][pr], xs);
                TX *y = Y + (size_t)row * ldp + c;
                if constexpr (SR) {
                    double2 sn;
                    sn.x = fma(be[0], cur.s[k][0], acc[0]);
                    sn.y = fma(be[1], cur.s[k][1], acc[1]);
                    stn2(y, sn);
                    const int cl = CPL * pr;
                    fold_add(xs[0] * cur.di[k], acc[0], m1[cl], f2, dot0[0], dot1[0]);
                    fold_add(xs[1] * cur.di[k], acc[1], m1[cl + 1], f2, dot0[1], dot1[1]);
                } else {
#pragma unroll
                    for (int u = 0; u < CPL; u += 2) {
                        if (c + u >= ldp) break;
                        const double2 q2 = make_double2(acc[u], acc[u + 1]);
                        stpair_nt(y + u, q2);
                        const double2 qs = as_stored(q2, (const TX *)y);
                        const int cl = CPL * pr + u;
                        fold_add(xs[u], qs.x, m1[cl], f2, dot0[u], dot1[u]);
                        fold_add(xs[u + 1], qs.y, m1[cl + 1], f2, dot0[u + 1], dot1[u + 1]);
                    }
                }
            }
        }
        __syncthreads();
        if (has_t) {   // the slots of rows [s - RING_H, s - RING_H + RING_G) are free now
#pragma unroll
            for (int k = 0; k < RING_RPL; ++k)
                ring[(t + RING_H + rl + 32 * k) % RING_ROWS][pr] = rn[k];
#pragma unroll
            for (int k = 0; k < RING_HPL; ++k) {
                hrow[rl + 32 * k][pr] = hn[k];
                if (pr == 0) hidx[rl + 32 * k] = hi_n[k];
            }
        }
        __syncthreads();
        cur = nxt;
        slow_c = slow_n;
        slow_n = slow_nn;
#pragma unroll
        for (int k = 0; k < RING_RPL; ++k) {
            nxt.rp[k][0] = rp_nn[k][0];
            nxt.rp[k][1] = rp_nn[k][1];
        }
#pragma unroll
        for (int k = 0; k < RING_HPL; ++k) hi_n[k] = hi_nn[k];
    }

    // partials of the range, summed over the block's lane groups in a fixed
    // order (the ring serves as the buffer: the loop ended on a barrier)
    double(*red)[32][CW] = reinterpret_cast<double(*)[32][CW]>(&ring[0][0]);
#pragma unroll
    for (int u = 0; u < CPL; ++u) {
        red[0][rl][CPL * pr + u] = dot0[u];
        red[1][rl][CPL * pr + u] = dot1[u];
    }
    __syncthreads();
    if (threadIdx.x < 2 * CW) {
        const int q = threadIdx.x / CW, cl = threadIdx.x % CW;
        const int col = cc * CW + cl;
        if (col < ldp) {
            double sum = 0.0;
            for (int k = 0; k < 32; ++k) sum += red[q][k][cl];
            part[(size_t)q * g.nrt * ldp + (size_t)col * g.nrt + range] = sum;
        }
    }
}

// Rows per lane per step in the streaming kernels (measured best on gfx950:
// the residual update gains from more loads in flight).
template <class TP>
constexpr int unroll_update() { return 8; }                           // k_update
constexpr int UNROLL_P = 4;                                           // k_pupdate

// Load form of the streaming kernels.  FP32 vectors are loaded without a
// guard, from addresses clamped into the block's rows and the padded columns,
// and out-of-range entries are masked afterwards: a guarded load that widens
// to double waits for its own data inside the guard, so only one or two loads
// per wave would be in flight.  FP64 vectors keep the guarded form, which
// measures faster for them.
template <class TP>
constexpr bool clamp_loads() { return sizeof(TP) == 4; }

// Rout = R - alpha Q (Rout == R: in place); partials r.D^-1 r and r.r of
// the new residual.  (X is updated lazily from the ring of the last LAZY
// search directions.)  Each entry is read and written by the same lane, so
// the in-place form is safe.
template <int LPR, int NV, class TP>
__global__ __launch_bounds__(BLOCK) void k_update(Geom g, const double *__restrict__ alpha,
                                                  const double *__restrict__ dinv,
                                                  const TP *R, const TP *__restrict__ Q,
                                                  TP *Rout, double *prz, double *prr) {
    constexpr int UR = unroll_update<TP>();
    constexpr bool CL = clamp_loads<TP>();
    Sched sc;
    if (!block_sched<Lane<LPR, NV>::RSTEP>(g, sc)) return;
    Lane<LPR, NV> ln(g, sc.cc);
    double2 acc[2][NV];
    double2 al[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) {
        acc[0][v] = acc[1][v] = make_double2(0.0, 0.0);
        al[v] = ln.ok[v] ? ld2(alpha + ln.c[v]) : make_double2(0.0, 0.0);
    }
    const int r1 = sc.re;
    for (int base = sc.rs + sc.first + ln.slot; base - ln.slot < r1; base += UR * sc.stride) {
        double2 r[UR][NV], q[UR][NV];
        double di[UR];
#pragma unroll
        for (int u = 0; u < UR; ++u) {
            const int row = base + u * sc.stride;
            const bool rv = CL || row < r1;
            const int rl = CL ? min(row, r1 - 1) : row;
            di[u] = rv ? dinv[rl] : 0.0;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const size_t o = (size_t)rl * g.ldp + (CL ? ln.cs[v] : ln.c[v]);
                const bool on = CL || (rv && ln.ok[v]);
                r[u][v] = on ? ldn2(R + o) : make_double2(0.0, 0.0);
                q[u][v] = on ? ldn2(Q + o) : make_double2(0.0, 0.0);
            }
        }
#pragma unroll
        for (int u = 0; u < UR; ++u) {
            const int row = base + u * sc.stride;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                if (!(row < r1 && ln.ok[v])) continue;
                double2 rr = r[u][v];
                rr.x = fma(-al[v].x, q[u][v].x, rr.x);
                rr.y = fma(-al[v].y, q[u][v].y, rr.y);
                rr = as_stored(rr, R);   // the dots see r as stored
                stn2(Rout + (size_t)row * g.ldp + ln.c[v], rr);
                acc[0][v].x = fma(rr.x, rr.x * di[u], acc[0][v].x);
                acc[0][v].y = fma(rr.y, rr.y * di[u], acc[0][v].y);
                acc[1][v].x = fma(rr.x, rr.x, acc[1][v].x);
                acc[1][v].y = fma(rr.y, rr.y, acc[1][v].y);
            }
        }
    }
    double *const parts[2] = {prz, prr};
    block_partials<LPR, NV, 2>(g, ln, sc.cc, sc.prow, acc, parts);
}

// X is updated every LAZY iterations from a ring of the last LAZY search
// directions (classic form) or residuals (single-reduction form); the host
// checks convergence every CHECK_MIN iterations or more.
constexpr int LAZY = 16;
constexpr int CHECK_MIN = 8;
template <class TP>
struct Ring {
    const TP *p[LAZY];
};

// X += sum_{j < cnt} alpha_j P_j (in ring order: the iterations' order), one
// pass over X per window of up to LAZY iterations.  Fixed geometry (32 lanes
// x 2 pairs per row, 128-column chunks, as the single-reduction flush); the
// window's step lengths of the block's columns sit in LDS and the directions
// are read eight at a time.  FP32 rings: unconditional loads from clamped
// addresses (slots past cnt read slot 0, cnt >= 1), masked at the store, as
// in k_update.
template <class TP>
__global__ __launch_bounds__(BLOCK) void k_xflush(Geom g, int cnt, const double *__restrict__ alphas,
                                                  Ring<TP> ring, double *__restrict__ X) {
    constexpr int LPR = 32, NV = 2;
    constexpr int CP = Lane<LPR, NV>::CW / 2;
    constexpr int HALF = LAZY / 2;
    constexpr bool CL = clamp_loads<TP>();
    __shared__ double2 cf[LAZY][CP];
    Sched sc;
    if (!block_sched<Lane<LPR, NV>::RSTEP>(g, sc)) return;   // whole block
    Lane<LPR, NV> ln(g, sc.cc);
    for (int i = threadIdx.x; i < LAZY * CP; i += BLOCK) {
        const int j = i / CP, cp = i % CP;
        const int col = sc.cc * 2 * CP + 2 * cp;
        cf[j][cp] = (j < cnt && col < g.ldp) ? ld2(alphas + (size_t)j * g.ldp + col)
                                             : make_double2(0.0, 0.0);
    }
    __syncthreads();
    __builtin_assume(cnt >= 1);   // the host launches no empty flush
    for (int base = sc.rs + sc.first; base < sc.re; base += sc.stride) {
        const int row = base + ln.slot;
        if (!CL && row >= sc.re) continue;
        const int rl = CL ? min(row, sc.re - 1) : row;
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (!CL && !ln.ok[v]) continue;
            const int cp = ln.lr + LPR * v;
            const size_t o = (size_t)rl * g.ldp + (CL ? ln.cs[v] : ln.c[v]);
            double2 x = ldn2(X + o);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                double2 p[HALF];
#pragma unroll
                for (int j = 0; j < HALF; ++j) {
                    const int jj = h * HALF + j;
                    p[j] = CL ? ldn2(ring.p[jj < cnt ? jj : 0] + o)
                              : (jj < cnt ? ldn2(ring.p[jj] + o) : make_double2(0.0, 0.0));
                }
#pragma unroll
                for (int j = 0; j < HALF; ++j) {
                    const int jj = h * HALF + j;
                    if (jj < cnt) {
                        const double2 a = cf[jj][cp];
                        x.x = fma(a.x, p[j].x, x.x);
                        x.y = fma(a.y, p[j].y, x.y);
                    }
                }
            }
            if (!CL || (row < sc.re && ln.ok[v])) stn2(X + o, x);
        }
    }
}

// Lazy search directions of the single-reduction PCG (FP64): for the
// iterations j < cnt of the window, in order, P = D^-1 R_j + beta_j P and
// X += alpha_j P, with the same fused multiply-adds as the direction update
// and the X flush of the classic form; one pass over P and X per window of
// up to LAZY iterations.  The window's step lengths and betas of the
// block's columns sit in LDS (LAZY of each per column pair would not fit
// in registers); the residuals are read eight at a time.
template <int LPR, int NV>
__global__ __launch_bounds__(BLOCK) void k_pflush(Geom g, int cnt, const double *__restrict__ alphas,
                                                  const double *__restrict__ betas,
                                                  Ring<double> ring,
                                                  const double *__restrict__ dinv,
                                                  double *__restrict__ P,
                                                  double *__restrict__ X) {
    constexpr int CP = Lane<LPR, NV>::CW / 2;   // column pairs of the chunk
    constexpr int HALF = LAZY / 2;
    __shared__ double2 cf[2][LAZY][CP];
    Sched sc;
    if (!block_sched<Lane<LPR, NV>::RSTEP>(g, sc)) return;   // whole block
    Lane<LPR, NV> ln(g, sc.cc);
    for (int i = threadIdx.x; i < 2 * LAZY * CP; i += BLOCK) {
        const int q = i / (LAZY * CP), j = (i / CP) % LAZY, cp = i % CP;
        const int col = sc.cc * 2 * CP + 2 * cp;
        cf[q][j][cp] = (j < cnt && col < g.ldp)
                           ? ld2((q ? betas : alphas) + (size_t)j * g.ldp + col)
                           : make_double2(0.0, 0.0);
    }
    __syncthreads();
    for (int base = sc.rs + sc.first; base < sc.re; base += sc.stride) {
        const int row = base + ln.slot;
        if (row >= sc.re) continue;
        const double di = dinv[row];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (!ln.ok[v]) continue;
            const int cp = ln.lr + LPR * v;
            const size_t o = (size_t)row * g.ldp + ln.c[v];
            double2 p = ldn2(P + o);
            double2 x = ldn2(X + o);
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                double2 r[HALF];
#pragma unroll
                for (int j = 0; j < HALF; ++j)
                    r[j] = h * HALF + j < cnt ? ldn2(ring.p[h * HALF + j] + o)
                                              : make_double2(0.0, 0.0);
#pragma unroll
                for (int j = 0; j < HALF; ++j) {
                    const int jj = h * HALF + j;
                    if (jj < cnt) {
                        const double2 a = cf[0][jj][cp], b = cf[1][jj][cp];
                        p.x = fma(b.x, p.x, r[j].x * di);
                        p.y = fma(b.y, p.y, r[j].y * di);
                        x.x = fma(a.x, p.x, x.x);
                        x.y = fma(a.y, p.y, x.y);
                    }
                }
            }
            stn2(P + o, p);
            stn2(X + o, x);
        }
    }
}

// Pout = D^-1 R + beta Pin (beta == nullptr: Pout = D^-1 R).
template <int LPR, int NV, class TP>
__global__ __launch_bounds__(BLOCK) void k_pupdate(Geom g, const double *__restrict__ beta,
                                                   const double *__restrict__ dinv,
                                                   const TP *__restrict__ R,
                                                   const TP *__restrict__ P,
                                                   TP *__restrict__ Pout) {
    constexpr bool CL = clamp_loads<TP>();
    Sched sc;
    if (!block_sched<Lane<LPR, NV>::RSTEP>(g, sc)) return;
    Lane<LPR, NV> ln(g, sc.cc);
    double2 be[NV];
#pragma unroll
    for (int v = 0; v < NV; ++v)
        be[v] = (ln.ok[v] && beta) ? ld2(beta + ln.c[v]) : make_double2(0.0, 0.0);
    const int r1 = sc.re;
    for (int base = sc.rs + sc.first + ln.slot; base - ln.slot < r1; base += UNROLL_P * sc.stride) {
        double2 r[UNROLL_P][NV], p[UNROLL_P][NV];
        double di[UNROLL_P];
#pragma unroll
        for (int u = 0; u < UNROLL_P; ++u) {
            const int row = base + u * sc.stride;
            const bool rv = CL || row < r1;
            const int rl = CL ? min(row, r1 - 1) : row;
            di[u] = rv ? dinv[rl] : 0.0;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                const size_t o = (size_t)rl * g.ldp + (CL ? ln.cs[v] : ln.c[v]);
                const bool on = CL || (rv && ln.ok[v]);
                r[u][v] = on ? ldn2(R + o) : make_double2(0.0, 0.0);
                p[u][v] = (on && beta) ? ldn2(P + o) : make_double2(0.0, 0.0);
            }
        }
#pragma unroll
        for (int u = 0; u < UNROLL_P; ++u) {
            const int row = base + u * sc.stride;
#pragma unroll
            for (int v = 0; v < NV; ++v) {
                if (!(row < r1 && ln.ok[v])) continue;
                double2 pn;
                if (beta) {
                    pn.x = fma(be[v].x, p[u][v].x, r[u][v].x * di[u]);
                    pn.y = fma(be[v].y, p[u][v].y, r[u][v].y * di[u]);
                } else {
                    pn = make_double2(r[u][v].x * di[u], r[u][v].y * di[u]);
                }
                stn2(Pout + (size_t)row * g.ldp + ln.c[v], pn);
            }
        }
    }
}

// R = B - Q (Q may be null: R = B).  Partials: b.b, r.D^-1 r, r.r.  R may be
// null (only the partials are wanted: true residual).  Solver row r takes the
// right-hand side of node perm[r].
template <int LPR, int NV, class TR>
__global__ __launch_bounds__(BLOCK) void k_residual(Geom g, const int32_t *__restrict__ perm,
                                                    const int32_t *__restrict__ bp,
                                                    const int32_t *__restrict__ bc,
                                                    const double *__restrict__ bv,
                                                    const int32_t *__restrict__ colmap,
                                                    const double *__restrict__ dinv,
                                                    const double *__restrict__ Q,
                                                    TR *__restrict__ R, double *pbb,
                                                    double *prz, double *prr) {
    Sched sc;
    if (!block_sched<Lane<LPR, NV>::RSTEP>(g, sc)) return;
    Lane<LPR, NV> ln(g, sc.cc);
    double2 acc[3][NV];
#pragma unroll
    for (int v = 0; v < NV; ++v) acc[0][v] = acc[1][v] = acc[2][v] = make_double2(0.0, 0.0);
    for (int base = sc.rs + sc.first; base < sc.re; base += sc.stride) {
        const int row = base + ln.slot;
        if (row >= sc.re) continue;
        const double di = dinv[row];
        const int node = perm[row];
        const int s = bp[node], e = bp[node + 1];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
            if (!ln.ok[v]) continue;
            double2 b = make_double2(0.0, 0.0);
            for (int k = s; k < e; ++k) {
                const int l = colmap ? colmap[bc[k]] : bc[k];
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
            if (R) {
                r = as_stored(r, (const TR *)R);   // the dots see r as stored
                st2(R + o, r);
            }
            acc[0][v].x = fma(b.x, b.x, acc[0][v].x);
            acc[0][v].y = fma(b.y, b.y, acc[0][v].y);
            acc[1][v].x = fma(r.x, r.x * di, acc[1][v].x);
            acc[1][v].y = fma(r.y, r.y * di, acc[1][v].y);
            acc[2][v].x = fma(r.x, r.x, acc[2][v].x);
            acc[2][v].y = fma(r.y, r.y, acc[2][v].y);
        }
    }
    double *const parts[3] = {pbb, prz, prr};
    block_partials<LPR, NV, 3>(g, ln, sc.cc, sc.prow, acc, parts);
}

// ---------------------------------------------------------------------------
// Per-column reductions (one block per column, fixed order).

struct Scal {
    double *rho, *alpha, *beta, *bb, *rr;
    double *tt;                       // per-column stop level for ||r||^2
    double *bd;                       // per-column bound on sum |t| of the SpMM's dot
    const double *kappa;              // max_i sum_j |a_ij| / d_i (device scalar)
    int32_t *iters, *active, *flag;   // flag[0]: breakdown
    const int32_t *gate;              // as Geom::gate
};

constexpr int RED = 256;

// The mixed-precision solve replaces the recurrence residual by the FP64
// true residual after every MIXED_REPLACE-th iteration (a multiple of LAZY).
constexpr int MIXED_REPLACE = 64;

__device__ __forceinline__ double col_sum(const double *part, int nrt, int c) {
    __shared__ double s[RED];
    double acc = 0.0;
    for (int k = threadIdx.x; k < nrt; k += RED) acc += part[(size_t)c * nrt + k];
    s[threadIdx.x] = acc;
    __syncthreads();
    for (int off = RED / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    const double r = s[0];
    __syncthreads();
    return r;
}

// A dot product of the SpMM from its two fold partials (exact sums).
__device__ __forceinline__ double col_sum2(const double *part, int nrt, int ldp, int c) {
    const double s1 = col_sum(part, nrt, c);
    const double s2 = col_sum(part + (size_t)nrt * ldp, nrt, c);
    return s1 + s2;
}

// Bounds of the SpMM's dot for the fold grids.  With z = D^-1 r and w = A z,
// sum_i |z_i w_i| <= sum_ij |a_ij| |z_i| |z_j| <= sum_i z_i^2 sum_j |a_ij|
// <= kappa gamma, gamma = r.D^-1 r: so 2 kappa gamma bounds the single-
// reduction delta and the first p.Ap (p = z).  Later p.Ap of the classic
// form take 2^16 times the previous one (no a-priori bound; an exceeded
// bound only makes the sum depend on the grouping again).
__device__ __forceinline__ double bound_z(const Scal &sc, double gamma) {
    return 2.0 * sc.kappa[0] * gamma;
}

// tt = max(tol^2 ||b||^2, eta^2 ||r||^2): eta = 0 runs to the tolerance; the
// mixed-precision mode uses eta > 0 so that each float32 cycle only reduces
// its starting residual by eta before the FP64 refinement step.
__global__ __launch_bounds__(RED) void k_red_init(Scal sc, const double *pbb, const double *prz,
                                                  const double *prr, int nrt, int L,
                                                  double tol2, double eta2) {
    const int c = blockIdx.x;
    const double bb = col_sum(pbb, nrt, c);
    const double rz = col_sum(prz, nrt, c);
    const double rr = col_sum(prr, nrt, c);
    if (threadIdx.x == 0) {
        sc.bb[c] = bb;
        sc.rho[c] = rz;
        sc.rr[c] = rr;
        sc.bd[c] = bound_z(sc, rz);
        sc.tt[c] = fmax(tol2 * bb, eta2 * rr);
        sc.iters[c] = 0;
        sc.alpha[c] = 0.0;
        sc.beta[c] = 0.0;
        sc.active[c] = (c < L && bb > 0.0 && rr > tol2 * bb) ? 1 : 0;
    }
}

__global__ __launch_bounds__(RED) void k_red_alpha(Scal sc, double *alpha, const double *ppq,
                                                   int nrt, int ldp) {
    const int c = blockIdx.x;
    if (sc.gate && *sc.gate == 0) return;
    const double pq = col_sum2(ppq, nrt, ldp, c);
    if (threadIdx.x == 0) {
        double a = 0.0;
        if (sc.active[c]) {
            if (pq > 0.0) {
                a = sc.rho[c] / pq;
                sc.bd[c] = 65536.0 * pq;
            } else {
                sc.active[c] = 0;
                sc.flag[0] = 1;
            }
        }
        alpha[c] = a;
    }
}

// Step length of the single-reduction form: with gamma = r.D^-1 r (rho) and
// delta = (D^-1 r).A(D^-1 r), p.Ap = delta - beta gamma / alpha_prev, so
// alpha = gamma / (delta - beta gamma / alpha_prev) (= gamma / delta when
// beta = 0).  sc.alpha keeps alpha_prev.
__global__ __launch_bounds__(RED) void k_red_alpha_sr(Scal sc, double *alpha, const double *pdelta,
                                                      int nrt, int ldp) {
    const int c = blockIdx.x;
    if (sc.gate && *sc.gate == 0) return;
    const double delta = col_sum2(pdelta, nrt, ldp, c);
    if (threadIdx.x == 0) {
        double a = 0.0;
        if (sc.active[c]) {
            const double b = sc.beta[c], gam = sc.rho[c];
            const double pap = b == 0.0 ? delta : delta - b * gam / sc.alpha[c];
            if (pap > 0.0) {
                a = gam / pap;
            } else {
                sc.active[c] = 0;
                sc.flag[0] = 1;
            }
        }
        alpha[c] = a;
        sc.alpha[c] = a;
    }
}

// beta = rz / rho of the new residual; bslot (optional) keeps a copy in the
// ring of step coefficients.
__global__ __launch_bounds__(RED) void k_red_beta(Scal sc, const double *prz, const double *prr,
                                                  int nrt, double *bslot, int sr) {
    const int c = blockIdx.x;
    if (sc.gate && *sc.gate == 0) return;
    const double rz = col_sum(prz, nrt, c);
    const double rr = col_sum(prr, nrt, c);
    if (threadIdx.x == 0) {
        double b = 0.0;
        if (sc.active[c]) {
            sc.iters[c] += 1;
            sc.rr[c] = rr;
            if (rr <= sc.tt[c]) {
                sc.active[c] = 0;
            } else {
                b = rz / sc.rho[c];
                sc.rho[c] = rz;
                if (sr) sc.bd[c] = bound_z(sc, rz);
            }
        }
        sc.beta[c] = b;
        if (bslot) bslot[c] = b;
    }
}

// Iterative refinement: after the true residual R = B - A X (FP64) is formed,
// columns whose true residual misses the tolerance restart with P = D^-1 R.
__global__ __launch_bounds__(RED) void k_red_refine(Scal sc, const double *prz,
                                                    const double *prr, int nrt, int L,
                                                    double tol2, double eta2) {
    const int c = blockIdx.x;
    const double rz = col_sum(prz, nrt, c);
    const double rr = col_sum(prr, nrt, c);
    if (threadIdx.x == 0) {
        const int again = (c < L && sc.bb[c] > 0.0 && rr > tol2 * sc.bb[c]) ? 1 : 0;
        sc.active[c] = again;
        sc.rr[c] = rr;
        if (again) {
            sc.rho[c] = rz;
            sc.bd[c] = bound_z(sc, rz);
            sc.tt[c] = fmax(tol2 * sc.bb[c], eta2 * rr);
        }
        sc.alpha[c] = 0.0;
        sc.beta[c] = 0.0;
    }
}

__global__ __launch_bounds__(RED) void k_red_sum(const double *part, int nrt, double *out) {
    const int c = blockIdx.x;
    const double s = col_sum(part, nrt, c);
    if (threadIdx.x == 0) out[c] = s;
}

// kappa = max over solver rows of sum_j |a_ij| / d_i (a maximum: the same in
// any order).  Partial maxima per block, then one block.
constexpr int KAPPA_BLOCKS = 256;
__global__ __launch_bounds__(RED) void k_kappa_part(const int32_t *rp, const double *va,
                                                    const double *dinv, int32_t n,
                                                    double *part) {
    __shared__ double s[RED];
    double m = 0.0;
    for (int64_t r = (int64_t)blockIdx.x * RED + threadIdx.x; r < n;
         r += (int64_t)gridDim.x * RED) {
        double a = 0.0;
        for (int32_t k = rp[r]; k < rp[r + 1]; ++k) a += fabs(va[k]);
        m = fmax(m, a * dinv[r]);
    }
    s[threadIdx.x] = m;
    __syncthreads();
    for (int off = RED / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__global__ __launch_bounds__(RED) void k_kappa_final(const double *part, int np, double *kappa) {
    __shared__ double s[RED];
    double m = 0.0;
    for (int k = threadIdx.x; k < np; k += RED) m = fmax(m, part[k]);
    s[threadIdx.x] = m;
    __syncthreads();
    for (int off = RED / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] = fmax(s[threadIdx.x], s[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) kappa[0] = s[0] > 0.0 ? s[0] : 1.0;
}

// Gate of a batched head at the end of a replayed chunk: 1 while any column
// is active.  The next chunk's kernels read it before doing anything, so a
// head that has converged costs the replays still queued only their
// launches.  out (optional) receives (gate, breakdown flag) for the host.
__global__ __launch_bounds__(RED) void k_gate(const int32_t *active, int ldp, const int32_t *flag,
                                             int32_t *gate, int32_t *out) {
    __shared__ int any;
    if (threadIdx.x == 0) any = 0;
    __syncthreads();
    int a = 0;
    for (int c = threadIdx.x; c < ldp; c += RED) a |= active[c] != 0;
    if (a) atomicOr(&any, 1);
    __syncthreads();
    if (threadIdx.x == 0) {
        *gate = any;
        if (out) {
            out[0] = any;
            out[1] = *flag;
        }
    }
}

// ---------------------------------------------------------------------------
// Tile table and dispatch

struct TileCfg {
    int lpr, nv, front;
    const char *name;
    int ring = 0;   // 1: the LDS ring SpMM (single-reduction FP64 form only)
};

constexpr TileCfg kTiles[] = {
    {64, 1, 0, "lpr64_nv1_cw128"},       {64, 2, 0, "lpr64_nv2_cw256"},
    {32, 1, 0, "lpr32_nv1_cw64"},        {32, 2, 0, "lpr32_nv2_cw128"},
    {16, 1, 0, "lpr16_nv1_cw32"},        {16, 2, 0, "lpr16_nv2_cw64"},
    {8, 1, 0, "lpr8_nv1_cw16"},          {8, 2, 0, "lpr8_nv2_cw32"},
    {4, 1, 0, "lpr4_nv1_cw8"},           {64, 4, 0, "lpr64_nv4_cw512"},
    {64, 1, 1, "lpr64_nv1_cw128_front"}, {64, 2, 1, "lpr64_nv2_cw256_front"},
    {32, 1, 1, "lpr32_nv1_cw64_front"},  {32, 2, 1, "lpr32_nv2_cw128_front"},
    {16, 1, 1, "lpr16_nv1_cw32_front"},  {16, 2, 1, "lpr16_nv2_cw64_front"},
    {8, 1, 1, "lpr8_nv1_cw16_front"},    {8, 2, 1, "lpr8_nv2_cw32_front"},
    {8, 1, 0, "ring_g64_cw16", 1},
};
constexpr int NTILES = sizeof(kTiles) / sizeof(kTiles[0]);
static_assert(NTILES <= 32, "residency cache size");
static_assert(RING_G == 64, "the ring tile's name gives its step");

#define ZI_TILE_SWITCH(tile, FN, ...)                       \
    switch (kTiles[tile].lpr * 8 + kTiles[tile].nv) {       \
        case 64 * 8 + 1: FN<64, 1>(__VA_ARGS__); break;     \
        case 64 * 8 + 2: FN<64, 2>(__VA_ARGS__); break;     \
        case 32 * 8 + 1: FN<32, 1>(__VA_ARGS__); break;     \
        case 32 * 8 + 2: FN<32, 2>(__VA_ARGS__); break;     \
        case 16 * 8 + 1: FN<16, 1>(__VA_ARGS__); break;     \
        case 16 * 8 + 2: FN<16, 2>(__VA_ARGS__); break;     \
        case 8 * 8 + 1: FN<8, 1>(__VA_ARGS__); break;       \
        case 8 * 8 + 2: FN<8, 2>(__VA_ARGS__); break;       \
        case 4 * 8 + 1: FN<4, 1>(__VA_ARGS__); break;       \
        default: FN<64, 4>(__VA_ARGS__); break;             \
    }

// Default tile without autotuning: the cooperative-front schedule with the
// narrowest column chunk that holds every column, two column pairs per lane
// where that chunk width allows it (measured fastest on the 2 mm sphere for
// 64-256 columns); below 16 columns the chunk-schedule lpr4 tile.
int auto_tile(int ldp) {
    int best = -1, bestcw = 1 << 30, bestnv = 0;
    for (int t = 0; t < NTILES; ++t) {
        if (!kTiles[t].front) continue;
        const int cw = 2 * kTiles[t].lpr * kTiles[t].nv;
        if (cw < ldp) continue;
        if (cw < bestcw || (cw == bestcw && kTiles[t].nv > bestnv)) {
            best = t;
            bestcw = cw;
            bestnv = kTiles[t].nv;
        }
    }
    if (ldp <= 8) return 8;           // lpr4_nv1_cw8
    return best >= 0 ? best : 9;      // wider than any front tile: lpr64_nv4_cw512
}

// resident: blocks of the kernel that one XCD holds at once (0: no cap).  In
// the cooperative front every block of a unit must be resident: a block
// walks its unit's whole row range, so blocks that only start when earlier
// ones have finished would sweep the range a second time, behind the first
// front, and fetch every shared neighbour row again.
constexpr int SLAB_STEPS = 64;
// ring_cw: the ring tile's chunk width (16 columns of double, 32 of float).
Geom make_geom(int n, int ldp, int tile, int resident = 0, int slabs = 1, int ring_cw = 16) {
    const TileCfg &t = kTiles[tile];
    const int cw = t.ring ? ring_cw : 2 * t.lpr * t.nv;
    const int rstep = WAVES * (64 / t.lpr);
    Geom g{};
    g.n = n;
    g.ldp = ldp;
    g.cl2n = 1;
    while ((1ll << g.cl2n) < (long long)n) ++g.cl2n;
    g.ncc = (ldp + cw - 1) / cw;
    g.front = t.front;
    if (t.ring) {
        // one block per (row range, chunk), as many as the chip holds at once
        // (at most TARGET_BLOCKS); ranges of whole steps, at least four
        const int target = std::max(1, (resident > 0 ? std::min(8 * resident, TARGET_BLOCKS)
                                                      : TARGET_BLOCKS) / g.ncc);
        int rb = (n + target - 1) / target;
        rb = std::max(4 * RING_G, ((rb + RING_G - 1) / RING_G) * RING_G);
        g.rb = rb;
        g.nrt = (n + rb - 1) / rb;
        g.nb = g.ncc * g.nrt;
        g.nb_pad = 8 * g.ncc * ((g.nrt + 7) / 8);
        g.slabs = 1;
    } else if (!t.front) {
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
        g.slabs = 1;
    } else {
        g.P = g.ncc >= 8 ? 1 : 8 / g.ncc;          // row parts per column chunk
        g.U = g.ncc * g.P;                         // units (chunk, part)
        const int groups = (n + g.P - 1) / g.P / rstep + 1;   // row groups per unit
        int B = TARGET_BLOCKS / g.U;
        if (resident > 0) B = std::min(B, resident / ((g.U + 7) / 8));
        if (B < 1) B = 1;
        if (B > groups) B = groups;
        g.B = B;
        // a slab spans at least SLAB_STEPS steps of the front: shorter sweeps
        // do not drift, and each slab costs a launch
        const int part = (n + g.P - 1) / g.P;
        g.slabs = std::max(1, std::min(slabs, part / (B * rstep * SLAB_STEPS)));
        g.slab = (part + g.slabs - 1) / g.slabs;
        g.nrt = g.slabs * g.P * B;
        g.nb = ((g.U + 7) / 8) * 8 * B;            // units padded to XCD multiples
        g.nb_pad = g.nb;
    }
    return g;
}

// Blocks of BLOCK threads that one XCD (a eighth of the CUs) holds at once
// for a kernel, from its register and LDS use.
int cus_per_xcd() {
    int dev = 0, cu = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cu < 8)
        return 1;
    return cu / 8;
}

template <class K>
int resident_per_xcd(K kern) {
    int nb = 0;
    if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kern, BLOCK, 0) != hipSuccess || nb < 1)
        nb = 1;
    return nb * cus_per_xcd();
}

// Kernels whose front geometry is capped by their own residency.
enum class GK { SPMM_SR, SPMM_DOT64, SPMM_DOT32, SPMM64, SPMM32F, UPDATE64, UPDATE32,
                PUPDATE64, PUPDATE32, RESIDUAL64, RESIDUAL32, COUNT };

template <int LPR, int NV>
void occupancy_of(GK k, int *out);

int resident_blocks(GK k, int tile) {
    static std::mutex mu;
    static int cache[(int)GK::COUNT][32] = {};
    std::lock_guard<std::mutex> lk(mu);
    int &r = cache[(int)k][tile];
    if (r == 0) {
        if (kTiles[tile].ring)
            r = k == GK::SPMM_DOT32   ? resident_per_xcd(k_spmm_ring<float, false>)
                : k == GK::SPMM_DOT64 ? resident_per_xcd(k_spmm_ring<double, false>)
                                      : resident_per_xcd(k_spmm_ring<double, true>);
        else
            ZI_TILE_SWITCH(tile, occupancy_of, k, &r);
    }
    return r;
}

// The SpMM of the solve runs as SPMM_SLABS launches, each over one slab of
// every unit's rows: the unit's blocks walk their rows as one front, but over
// a long range they drift apart and the neighbour rows they share leave L2
// between uses; a kernel boundary every slab lines the front up again.  On
// the 1 mm sphere (256 columns) 8 slabs took the SpMM from 5.60 to 5.43 ms
// (4: 5.43, 16: 5.47).  Slabs never change a result: the dot products are
// summed on fixed grids.
constexpr int MAX_SLABS = 16;
constexpr int SPMM_SLABS = 8;
int spmm_slabs(GK k) {
    return (k == GK::SPMM_SR || k == GK::SPMM_DOT64 || k == GK::SPMM_DOT32) ? SPMM_SLABS : 1;
}

Geom make_geom_for(GK k, int n, int ldp, int tile) {
    return make_geom(n, ldp, tile, resident_blocks(k, tile), std::min(MAX_SLABS, spmm_slabs(k)),
                     k == GK::SPMM_DOT32 ? 32 : 16);
}

template <int LPR, int NV, class TV, class TX>
void launch_spmm(const Geom &g, hipStream_t s, const int32_t *rp, const int32_t *ci,
                 const TV *va, const TX *X, TX *Y, double *part,
                 const double *bound = nullptr) {
    Geom gs = g;
    for (gs.cur = 0; gs.cur < g.slabs; ++gs.cur) {
        if (part)
            hipLaunchKernelGGL((k_spmm<LPR, NV, TV, TX, true>), dim3(g.nb_pad), dim3(BLOCK), 0, s,
                               gs, rp, ci, va, X, Y, part, bound);
        else
            hipLaunchKernelGGL((k_spmm<LPR, NV, TV, TX, false>), dim3(g.nb_pad), dim3(BLOCK), 0,
                               s, gs, rp, ci, va, X, Y, part, bound);
    }
}

template <int LPR, int NV, class TP>
void launch_update(const Geom &g, hipStream_t s, const double *alpha, const double *dinv,
                   const TP *R, const TP *Q, TP *Rout, double *prz, double *prr) {
    hipLaunchKernelGGL((k_update<LPR, NV, TP>), dim3(g.nb_pad), dim3(BLOCK), 0, s, g, alpha, dinv,
                       R, Q, Rout, prz, prr);
}

template <int LPR, int NV>
void launch_spmm_sr(const Geom &g, hipStream_t s, const int32_t *rp, const int32_t *ci,
                    const double *vs, const double *dinv, const double *R, const double *beta,
                    double *S, double *part, const double *bound) {
    Geom gs = g;
    for (gs.cur = 0; gs.cur < g.slabs; ++gs.cur)
        hipLaunchKernelGGL((k_spmm_sr<LPR, NV>), dim3(g.nb_pad), dim3(BLOCK), 0, s, gs, rp, ci,
                           vs, dinv, R, beta, S, part, bound);
}

// halo: the system's ring lists (ring_halo), followed by the steps' path
// flags.  SR: Y = A D^-1 X + beta Y (vals = a_ij / d_j); else Y = A X.
template <class TX, bool SR>
void launch_spmm_ring(const Geom &g, hipStream_t s, const int32_t *halo, const int32_t *rp,
                      const int32_t *ci, const double *vals, const double *dinv, const TX *X,
                      const double *beta, TX *Y, double *part, const double *bound) {
    const size_t steps = ((size_t)g.n + RING_G - 1) / RING_G;
    hipLaunchKernelGGL((k_spmm_ring<TX, SR>), dim3(g.nb_pad), dim3(BLOCK), 0, s, g, halo,
                       halo + steps * RING_HMAX, rp, ci, vals, dinv, X, beta, Y, part, bound);
}

// Halo lists of the ring SpMM (one per RING_G rows of the solver's matrix),
// built once per system.
zi_status ensure_ring(zi_system *sys, hipStream_t s) {
    if (sys->ring_halo) return ZI_OK;
    const int steps = (sys->n + RING_G - 1) / RING_G;
    int32_t *h = nullptr;   // lists, then one path flag per step
    ZI_TRY(sys->pool.alloc(&h, (size_t)std::max(steps, 1) * (RING_HMAX + 1)));
    if (steps > 0) {
        hipLaunchKernelGGL(k_ring_halo, dim3(steps), dim3(256), 0, s, sys->sp_ptr, sys->sp_col,
                           sys->n, h, h + (size_t)steps * RING_HMAX);
        ZI_HIP(hipGetLastError());
    }
    sys->ring_halo = h;
    return ZI_OK;
}

template <int LPR, int NV>
void occupancy_of(GK k, int *out) {
    switch (k) {
        case GK::SPMM_SR: *out = resident_per_xcd(k_spmm_sr<LPR, NV>); break;
        case GK::SPMM_DOT64:
            *out = resident_per_xcd(k_spmm<LPR, NV, double, double, true>);
            break;
        case GK::SPMM_DOT32:
            *out = resident_per_xcd(k_spmm<LPR, NV, double, float, true>);
            break;
        case GK::SPMM64: *out = resident_per_xcd(k_spmm<LPR, NV, double, double, false>); break;
        case GK::SPMM32F: *out = resident_per_xcd(k_spmm<LPR, NV, float, float, false>); break;
        case GK::UPDATE64: *out = resident_per_xcd(k_update<LPR, NV, double>); break;
        case GK::UPDATE32: *out = resident_per_xcd(k_update<LPR, NV, float>); break;
        case GK::PUPDATE64: *out = resident_per_xcd(k_pupdate<LPR, NV, double>); break;
        case GK::PUPDATE32: *out = resident_per_xcd(k_pupdate<LPR, NV, float>); break;
        case GK::RESIDUAL64: *out = resident_per_xcd(k_residual<LPR, NV, double>); break;
        default: *out = resident_per_xcd(k_residual<LPR, NV, float>); break;
    }
}

// The flush writes no partial sums, so it runs with its own geometry: the
// cooperative front of 32 lanes x 2 pairs per row (128-column chunks), the
// fastest for it on the 2 mm sphere, whatever tile the SpMM uses.
constexpr int FLUSH_TILE = 13;   // lpr32_nv2_cw128_front
// Residual update, direction update, residual b - A x and the lazy-P flush
// run with one geometry for a given column count and precision, whatever
// the SpMM tile: 128-column front chunks of 32 lanes x 2 pairs from 128
// columns up, else the narrowest front tile that holds every column (no idle
// lanes on 32-96 column blocks).  Float32 blocks of more than 128 columns
// take 256-column chunks, a row of up to 1 KB per lane group (the float32
// residual update at 1 mm, 256 columns: 1.97 against 2.05 ms).
constexpr int STREAM_TILE_F32 = 11;   // lpr64_nv2_cw256_front
int stream_tile(int ldp, bool f32 = false) {
    if (f32 && ldp > 128) return STREAM_TILE_F32;
    return ldp >= 128 ? FLUSH_TILE : auto_tile(ldp);
}
static_assert(kTiles[STREAM_TILE_F32].lpr == 64 && kTiles[STREAM_TILE_F32].nv == 2 &&
                  kTiles[STREAM_TILE_F32].front == 1,
              "float32 streaming geometry");
static_assert(kTiles[FLUSH_TILE].lpr == 32 && kTiles[FLUSH_TILE].nv == 2 &&
                  kTiles[FLUSH_TILE].front == 1,
              "flush geometry");

template <class TP>
void launch_xflush(int n, int ldp, const int32_t *gate, hipStream_t s, int cnt,
                   const double *alphas, Ring<TP> ring,
                   double *X) {
    static const int res = resident_per_xcd(k_xflush<TP>);
    Geom g = make_geom(n, ldp, FLUSH_TILE, res);
    g.gate = gate;
    hipLaunchKernelGGL((k_xflush<TP>), dim3(g.nb_pad), dim3(BLOCK), 0, s, g, cnt, alphas, ring,
                       X);
}

template <int LPR, int NV>
void launch_pflush_t(int n, int ldp, int tile, const int32_t *gate, hipStream_t s, int cnt,
                     const double *alphas, const double *betas, Ring<double> ring,
                     const double *dinv, double *P, double *X) {
    static const int res = resident_per_xcd(k_pflush<LPR, NV>);
    Geom g = make_geom(n, ldp, tile, res);
    g.gate = gate;
    hipLaunchKernelGGL((k_pflush<LPR, NV>), dim3(g.nb_pad), dim3(BLOCK), 0, s, g, cnt, alphas,
                       betas, ring, dinv, P, X);
}

void launch_pflush(int n, int ldp, const int32_t *gate, hipStream_t s, int cnt,
                   const double *alphas, const double *betas, Ring<double> ring,
                   const double *dinv, double *P, double *X) {
    const int tile = stream_tile(ldp);
    ZI_TILE_SWITCH(tile, launch_pflush_t, n, ldp, tile, gate, s, cnt, alphas, betas, ring, dinv,
                   P, X);
}

template <int LPR, int NV, class TP>
void launch_pupdate(const Geom &g, hipStream_t s, const double *beta, const double *dinv,
                    const TP *R, const TP *P, TP *Pout) {
    hipLaunchKernelGGL((k_pupdate<LPR, NV, TP>), dim3(g.nb_pad), dim3(BLOCK), 0, s, g, beta, dinv,
                       R, P, Pout);
}


template <int LPR, int NV, class TR>
void launch_residual(const Geom &g, hipStream_t s, const zi_system *sys, const int32_t *colmap,
                     const double *dinv, const double *Q, TR *R, double *pbb, double *prz,
                     double *prr) {
    hipLaunchKernelGGL((k_residual<LPR, NV, TR>), dim3(g.nb_pad), dim3(BLOCK), 0, s, g, sys->perm,
                       sys->b_ptr, sys->b_col, sys->b_val, colmap, dinv, Q, R, pbb, prz, prr);
}

__global__ void k_to_f32(const double *a, int64_t n, float *b) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}

// Values of A D^-1: vs[k] = va[k] dinv[ci[k]].
__global__ void k_scale_cols(const double *va, const int32_t *ci, const double *dinv, int64_t nnz,
                             double *vs) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < nnz) vs[k] = va[k] * dinv[ci[k]];
}

// Preconditioner in solver row order: dinv[r] = 1 / d[perm[r]].
__global__ void k_dinv(const double *d, const int32_t *perm, int32_t n, double *dinv) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) dinv[r] = 1.0 / d[perm[r]];
}

}  // namespace

// ---------------------------------------------------------------------------
// Workspace

struct zi_solver_ws {
    int ldp = 0, nrt_cap = 0;
    double *X = nullptr, *R = nullptr, *Q = nullptr, *dinv = nullptr;
    double *P[LAZY] = {};   // search-direction ring (classic: 0..7); lazy P and residual ring
    double *aring = nullptr;                                  // LAZY x ldp step lengths
    double *aflush = nullptr;                                 // LAZY x ldp scratch
    double *bring = nullptr;                                  // LAZY x ldp betas (single-reduction)
    double *bflush = nullptr;                                 // LAZY x ldp scratch
    double *vs = nullptr;                                     // values of A D^-1
    double *part[3] = {nullptr, nullptr, nullptr};   // 2 x nrt x ldp each (two folds)
    double *kap = nullptr;      // kappa and its block partial maxima
    int32_t *gate = nullptr;    // batched heads: any column active at the last chunk end
    double *sc_d = nullptr;     // rho alpha beta bb rr tt bd (7 ldp)
    int32_t *sc_i = nullptr;    // iters active (2 ldp) + flag
    std::vector<hipEvent_t> ev;
    zi::Pool pool;
    int32_t *h_pin = nullptr;   // pinned host copy of active (ldp) + flag
    ~zi_solver_ws() {
        for (auto e : ev) (void)hipEventDestroy(e);
        if (h_pin) (void)hipHostFree(h_pin);
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
    ws->pool.cached = true;
    const size_t blk = (size_t)sys->n * ldp;
    zi_status st = ZI_OK;
    for (int j = 0; j < LAZY; ++j) {
        if ((st = ws->pool.alloc(&ws->P[j], blk)) != ZI_OK) {
            delete ws;
            return st;
        }
    }
    if ((st = ws->pool.alloc(&ws->X, blk)) != ZI_OK || (st = ws->pool.alloc(&ws->R, blk)) != ZI_OK ||
        (st = ws->pool.alloc(&ws->aring, (size_t)LAZY * ldp)) != ZI_OK ||
        (st = ws->pool.alloc(&ws->aflush, (size_t)LAZY * ldp)) != ZI_OK ||
        (st = ws->pool.alloc(&ws->bring, (size_t)LAZY * ldp)) != ZI_OK ||
        (st = ws->pool.alloc(&ws->bflush, (size_t)LAZY * ldp)) != ZI_OK ||
        (st = ws->pool.alloc(&ws->vs, (size_t)std::max<int64_t>(sys->sp_nnz, 1))) != ZI_OK ||
        (st = ws->pool.alloc(&ws->Q, blk)) != ZI_OK ||
        (st = ws->pool.alloc(&ws->dinv, (size_t)sys->n)) != ZI_OK ||
        (st = ws->pool.alloc(&ws->sc_d, (size_t)7 * ldp)) != ZI_OK ||
        (st = ws->pool.alloc(&ws->kap, (size_t)KAPPA_BLOCKS + 1)) != ZI_OK ||
        (st = ws->pool.alloc(&ws->gate, 1)) != ZI_OK ||
        (st = ws->pool.alloc(&ws->sc_i, (size_t)2 * ldp + 1)) != ZI_OK) {
        delete ws;
        return st;
    }
    for (int q = 0; q < 3; ++q) {
        if ((st = ws->pool.alloc(&ws->part[q], (size_t)2 * nrt_max * ldp)) != ZI_OK) {
            delete ws;
            return st;
        }
    }
    if (hipHostMalloc(reinterpret_cast<void **>(&ws->h_pin), sizeof(int32_t) * (ldp + 1)) !=
        hipSuccess) {
        ws->h_pin = nullptr;
        delete ws;
        set_error("hipHostMalloc of %zu bytes failed", sizeof(int32_t) * (ldp + 1));
        return ZI_ENOMEM;
    }
    ws->ldp = ldp;
    ws->nrt_cap = nrt_max;
    sys->ws = ws;
    return ZI_OK;
}

// Partial-sum rows per column that any geometry of these sizes uses: a
// residency cap only lowers B, and slabs multiply P B by at most MAX_SLABS.
int max_nrt(int n, int ldp) {
    int m = 1;
    for (int t = 0; t < NTILES; ++t) {
        const Geom g = make_geom(n, ldp, t);
        m = std::max(m, g.front ? MAX_SLABS * g.nrt : g.nrt);
        if (kTiles[t].ring) m = std::max(m, make_geom(n, ldp, t, 0, 1, 32).nrt);
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

namespace {

// One transfer-matrix solve split into phases, so that the iteration loop can
// be replayed as a hipGraph and several systems can share one graph.
struct SolveCtx {
    zi_system *sys = nullptr;
    zi_solver_ws *ws = nullptr;
    Geom g{};                 // SpMM (the tile); partials of red_alpha
    // The streaming kernels run with one fixed geometry whatever the tile, so
    // their partial sums (and all results) do not depend on the tile.
    Geom gu{};                // residual update; partials of red_beta
    Geom gp{};                // direction update (classic form)
    Geom gr{};                // residual b - A x; partials of red_init, red_refine
    int32_t *gate = nullptr;      // batched heads: the head's gate (null: not gated)
    int32_t *gate_out = nullptr;  // batched heads: (gate, breakdown) for the host
    int tile = 0, ldp = 0, L = 0, maxit = 0, check = 0;
    int stile = 0;            // the streaming kernels' tile (a function of ldp)
    int rtile = 0;            // tile and geometry of the product A X of the true residual
    Geom grt{};               // (the SpMM tile's, or the streaming tile's for the ring tile)
    double tol = 0, tol2 = 0;
    double eta2 = 0;          // inner-cycle reduction (squared); 0 = run to tol
    bool mixed = false, timing = false;
    bool sr = false;          // single-reduction form (FP64)
    Scal sc{};
    EventTimer timer{nullptr};
    // event pairs per timed kernel: spmm_pq, update, pupdate, xflush
    std::vector<hipEvent_t> ev[4];
    int calls[4] = {0, 0, 0, 0};   // launches of the same kernels
    int it = 0;               // iterations of the block loop so far
    int flushed = 0;          // iterations whose steps are already in X
    int refinements = 0;
    int32_t *colmap = nullptr;   // electrode -> solved column (or -1), if a subset
    bool any_active = true;
    bool done = false;        // no further iterations wanted
    int32_t h_flag = 0;
    std::vector<int32_t> h_active;
    std::chrono::steady_clock::time_point t_start;
    template <class TP>
    TP *P(int k) const { return reinterpret_cast<TP *>(ws->P[k % LAZY]); }
    double *alpha(int k) const { return ws->aring + (size_t)(k % LAZY) * ldp; }
    // Single-reduction form: residual r_k in a ring of LAZY blocks (R,
    // P[1..15]; slot 0 is R, where the initial residual is formed), the lazy
    // search direction in P[0], S = A p in Q, the betas beside the step lengths.
    double *Rsr(int k) const { return k % LAZY == 0 ? ws->R : ws->P[k % LAZY]; }
    double *beta_slot(int k) const { return ws->bring + (size_t)(k % LAZY) * ldp; }
};

// A batched head's gate is opened for work the host enqueues outside the
// replays (set-up, refinement, the final flush and residual); k_gate then
// sets it from the active flags.
zi_status open_gate(SolveCtx &c, hipStream_t s) {
    return c.gate ? fill_i32(c.gate, 1, 1, s) : ZI_OK;
}

// The active flags (ldp) and the breakdown flag are adjacent: one copy into
// the workspace's pinned buffer, read after the stream has been synchronised.
zi_status enqueue_read_active(SolveCtx &c, hipStream_t s) {
    ZI_HIP(hipMemcpyAsync(c.ws->h_pin, c.sc.active, sizeof(int32_t) * (c.ldp + 1),
                          hipMemcpyDeviceToHost, s));
    return ZI_OK;
}

void take_active(SolveCtx &c) {
    c.h_flag = c.ws->h_pin[c.ldp];
    c.any_active = false;
    for (int k = 0; k < c.ldp; ++k) {
        c.h_active[k] = c.ws->h_pin[k];
        c.any_active = c.any_active || c.h_active[k];
    }
}

zi_status read_active(SolveCtx &c, hipStream_t s) {
    ZI_TRY(enqueue_read_active(c, s));
    ZI_HIP(hipStreamSynchronize(s));
    take_active(c);
    return ZI_OK;
}

// Kernel timing samples one iteration in TIMING_STRIDE (events between
// dependent kernels add a few microseconds each); the statistics report the
// sampled launches and their total time.
constexpr int TIMING_STRIDE = 8;

struct Timed {
    SolveCtx &c;
    int which;
    hipStream_t s;
    hipEvent_t e1 = nullptr;
    zi_status st = ZI_OK;
    bool on;
    Timed(SolveCtx &c_, int w, hipStream_t s_, bool sample)
        : c(c_), which(w), s(s_), on(c_.timing && sample) {
        ++c.calls[which];
        if (!on) return;
        hipEvent_t e0;
        if ((st = c.timer.get(&e0)) != ZI_OK || (st = c.timer.get(&e1)) != ZI_OK) return;
        c.ev[which].push_back(e0);
        c.ev[which].push_back(e1);
        (void)hipEventRecord(e0, s);
    }
    ~Timed() {
        if (on && e1) (void)hipEventRecord(e1, s);
    }
};

zi_status true_residual(SolveCtx &c, hipStream_t s, bool write_r);

// X += sum of the pending steps alpha_j P_j (iterations flushed .. it_end-1).
template <class TP>
zi_status enqueue_flush(SolveCtx &c, int it_end, hipStream_t s) {
    const int cnt = it_end - c.flushed;
    if (cnt <= 0) return ZI_OK;
    Ring<TP> ring;
    for (int j = 0; j < LAZY; ++j) ring.p[j] = c.P<TP>(c.flushed + j);
    // the alpha slots of iterations flushed.. are (flushed + j) % LAZY; the
    // ring is rotated so that entry j is iteration flushed + j
    double *al = c.ws->aring;
    const int first = c.flushed % LAZY;
    {
        Timed t(c, 3, s, cnt == LAZY);
        ZI_TRY(t.st);
        if (first == 0) {
            launch_xflush<TP>(c.sys->n, c.ldp, c.gate, s, cnt, (const double *)al, ring,
                              c.ws->X);
        } else {
            // the step lengths are rotated into a contiguous scratch block
            for (int j = 0; j < cnt; ++j)
                ZI_HIP(hipMemcpyAsync(c.ws->aflush + (size_t)j * c.ldp, c.alpha(c.flushed + j),
                                      sizeof(double) * c.ldp, hipMemcpyDeviceToDevice, s));
            launch_xflush<TP>(c.sys->n, c.ldp, c.gate, s, cnt, (const double *)c.ws->aflush, ring,
                              c.ws->X);
        }
    }
    ZI_HIP(hipGetLastError());
    c.flushed = it_end;
    return ZI_OK;
}

// Enqueue iteration k (no host synchronisation): SpMM with p.q, alpha, the
// residual update, every LAZY-th iteration the X flush, beta and the next
// direction into the ring.  TP is the element type of P and Q; the matrix
// values are FP64 in both modes.  replace_r: after the flush, overwrite r by the
// FP64 true residual b - A x before beta (a reliable update: the search
// direction is kept, only the drift of the recurrence is removed).
template <class TP>
zi_status enqueue_iteration(SolveCtx &c, int k, const double *va, hipStream_t s,
                            bool replace_r) {
    zi_solver_ws *ws = c.ws;
    const Geom &g = c.g;
    const int tile = c.tile;
    TP *Pk = c.P<TP>(k), *Pn = c.P<TP>(k + 1);
    TP *Q = reinterpret_cast<TP *>(ws->Q);
    double *al = c.alpha(k);
    {
        Timed t(c, 0, s, k % TIMING_STRIDE == 0);
        ZI_TRY(t.st);
        if (kTiles[tile].ring)
            launch_spmm_ring<TP, false>(g, s, c.sys->ring_halo, c.sys->sp_ptr, c.sys->sp_col, va,
                                        nullptr, (const TP *)Pk, nullptr, Q, ws->part[0],
                                        (const double *)c.sc.bd);
        else
            ZI_TILE_SWITCH(tile, launch_spmm, g, s, c.sys->sp_ptr, c.sys->sp_col, va,
                           (const TP *)Pk, Q, ws->part[0], (const double *)c.sc.bd);
    }
    hipLaunchKernelGGL(k_red_alpha, dim3(c.ldp), dim3(RED), 0, s, c.sc, al, ws->part[0], g.nrt,
                       c.ldp);
    {
        Timed t(c, 1, s, k % TIMING_STRIDE == 0);
        ZI_TRY(t.st);
        ZI_TILE_SWITCH(c.stile, launch_update, c.gu, s, (const double *)al,
                       (const double *)ws->dinv, (const TP *)ws->R, (const TP *)Q,
                       reinterpret_cast<TP *>(ws->R), ws->part[1], ws->part[2]);
    }
    if ((k + 1) % LAZY == 0 || replace_r) ZI_TRY(enqueue_flush<TP>(c, k + 1, s));
    // a reliable update rewrites the partials of part[0..2] with c.gr's layout
    const int nrt_beta = replace_r ? c.gr.nrt : c.gu.nrt;
    if (replace_r) ZI_TRY(true_residual(c, s, true));
    hipLaunchKernelGGL(k_red_beta, dim3(c.ldp), dim3(RED), 0, s, c.sc, ws->part[1], ws->part[2],
                       nrt_beta, (double *)nullptr, 0);
    {
        Timed t(c, 2, s, k % TIMING_STRIDE == 0);
        ZI_TRY(t.st);
        ZI_TILE_SWITCH(c.stile, launch_pupdate, c.gp, s, (const double *)c.sc.beta,
                       (const double *)ws->dinv, (const TP *)ws->R, (const TP *)Pk, Pn);
    }
    ZI_HIP(hipGetLastError());
    return ZI_OK;
}

// Single-reduction form: X += alpha_j P_j with P_j = D^-1 R_j + beta_j P_{j-1}
// for the pending iterations flushed .. it_end-1, one pass over P and X.
zi_status enqueue_flush_sr(SolveCtx &c, int it_end, hipStream_t s) {
    const int cnt = it_end - c.flushed;
    if (cnt <= 0) return ZI_OK;
    Ring<double> ring;
    for (int j = 0; j < LAZY; ++j) ring.p[j] = c.Rsr(c.flushed + j);
    const double *al = c.ws->aring, *bt = c.ws->bring;
    if (c.flushed % LAZY != 0) {   // rotate the coefficients into contiguous blocks
        for (int j = 0; j < cnt; ++j) {
            ZI_HIP(hipMemcpyAsync(c.ws->aflush + (size_t)j * c.ldp, c.alpha(c.flushed + j),
                                  sizeof(double) * c.ldp, hipMemcpyDeviceToDevice, s));
            ZI_HIP(hipMemcpyAsync(c.ws->bflush + (size_t)j * c.ldp, c.beta_slot(c.flushed + j),
                                  sizeof(double) * c.ldp, hipMemcpyDeviceToDevice, s));
        }
        al = c.ws->aflush;
        bt = c.ws->bflush;
    }
    {
        Timed t(c, 2, s, cnt == LAZY);
        ZI_TRY(t.st);
        launch_pflush(c.sys->n, c.ldp, c.gate, s, cnt, al, bt, ring, (const double *)c.ws->dinv,
                      c.ws->P[0], c.ws->X);
    }
    ZI_HIP(hipGetLastError());
    c.flushed = it_end;
    return ZI_OK;
}

// Iteration k of the single-reduction form (Chronopoulos and Gear's PCG: one
// reduction point per iteration, the same iterates as the classic form in
// exact arithmetic).  With r_k, gamma_k = r_k.D^-1 r_k and beta_k known:
//   S = A D^-1 r_k + beta_k S and delta_k;  alpha_k;  [lazy P, X flush];
//   r_{k+1} = r_k - alpha_k S with gamma_{k+1}, ||r_{k+1}||^2;  beta_{k+1}.
// The flush of a window runs before the update that overwrites the ring slot
// of the window's first residual.
zi_status enqueue_iteration_sr(SolveCtx &c, int k, hipStream_t s) {
    zi_solver_ws *ws = c.ws;
    const Geom &g = c.g;
    const int tile = c.tile;
    double *al = c.alpha(k);
    {
        Timed t(c, 0, s, k % TIMING_STRIDE == 0);
        ZI_TRY(t.st);
        if (kTiles[tile].ring)
            launch_spmm_ring<double, true>(g, s, c.sys->ring_halo, c.sys->sp_ptr,
                                           c.sys->sp_col, (const double *)ws->vs,
                                           (const double *)ws->dinv, (const double *)c.Rsr(k),
                                           (const double *)c.sc.beta, ws->Q, ws->part[0],
                                           (const double *)c.sc.bd);
        else
            ZI_TILE_SWITCH(tile, launch_spmm_sr, g, s, c.sys->sp_ptr, c.sys->sp_col,
                           (const double *)ws->vs, (const double *)ws->dinv,
                           (const double *)c.Rsr(k), (const double *)c.sc.beta, ws->Q,
                           ws->part[0], (const double *)c.sc.bd);
    }
    hipLaunchKernelGGL(k_red_alpha_sr, dim3(c.ldp), dim3(RED), 0, s, c.sc, al, ws->part[0], g.nrt,
                       c.ldp);
    if ((k + 1) % LAZY == 0) ZI_TRY(enqueue_flush_sr(c, k + 1, s));
    {
        Timed t(c, 1, s, k % TIMING_STRIDE == 0);
        ZI_TRY(t.st);
        ZI_TILE_SWITCH(c.stile, launch_update, c.gu, s, (const double *)al,
                       (const double *)ws->dinv, (const double *)c.Rsr(k),
                       (const double *)ws->Q, c.Rsr(k + 1), ws->part[1], ws->part[2]);
    }
    hipLaunchKernelGGL(k_red_beta, dim3(c.ldp), dim3(RED), 0, s, c.sc, ws->part[1], ws->part[2],
                       c.gu.nrt, c.beta_slot(k + 1), 1);
    ZI_HIP(hipGetLastError());
    return ZI_OK;
}

// Iterations it .. it+count-1.  In the mixed-precision mode iteration k is a
// reliable update when (k + 1) % MIXED_REPLACE == 0.
zi_status enqueue_iterations(SolveCtx &c, int count, hipStream_t s) {
    const int it0 = c.it;
    for (int j = 0; j < count; ++j) {
        if (c.sr) {
            ZI_TRY(enqueue_iteration_sr(c, it0 + j, s));
        } else if (c.mixed) {
            ZI_TRY(enqueue_iteration<float>(c, it0 + j, c.sys->sp_val, s,
                                            (it0 + j + 1) % MIXED_REPLACE == 0));
        } else {
            ZI_TRY(enqueue_iteration<double>(c, it0 + j, c.sys->sp_val, s, false));
        }
    }
    return ZI_OK;
}

zi_status flush_all(SolveCtx &c, hipStream_t s) {
    if (c.sr) return enqueue_flush_sr(c, c.it, s);
    if (c.mixed) return enqueue_flush<float>(c, c.it, s);
    return enqueue_flush<double>(c, c.it, s);
}

// R = B - A X in FP64 with its partials (b.b, r.D^-1 r, r.r) in part[0..2].
// Q is used as FP64 scratch (its float32 half is rewritten by the next SpMM).
zi_status true_residual(SolveCtx &c, hipStream_t s, bool write_r) {
    zi_solver_ws *ws = c.ws;
    ZI_TILE_SWITCH(c.rtile, launch_spmm, c.grt, s, c.sys->sp_ptr, c.sys->sp_col,
                   (const double *)c.sys->sp_val, (const double *)ws->X, ws->Q, (double *)nullptr);
    if (c.mixed) {   // R holds float32 in the mixed mode
        ZI_TILE_SWITCH(c.stile, launch_residual, c.gr, s, c.sys, (const int32_t *)c.colmap,
                       ws->dinv, ws->Q, write_r ? reinterpret_cast<float *>(ws->R) : nullptr,
                       ws->part[0], ws->part[1], ws->part[2]);
    } else {
        ZI_TILE_SWITCH(c.stile, launch_residual, c.gr, s, c.sys, (const int32_t *)c.colmap,
                       ws->dinv, ws->Q, write_r ? ws->R : nullptr, ws->part[0], ws->part[1],
                       ws->part[2]);
    }
    ZI_HIP(hipGetLastError());
    return ZI_OK;
}

// P_it = D^-1 R (start or restart of the search directions).
zi_status enqueue_restart_direction(SolveCtx &c, hipStream_t s) {
    if (c.mixed) {
        float *p = c.P<float>(c.it);
        ZI_TILE_SWITCH(c.stile, launch_pupdate, c.gp, s, (const double *)nullptr,
                       (const double *)c.ws->dinv, (const float *)c.ws->R, (const float *)p, p);
    } else {
        double *p = c.P<double>(c.it);
        ZI_TILE_SWITCH(c.stile, launch_pupdate, c.gp, s, (const double *)nullptr,
                       (const double *)c.ws->dinv, (const double *)c.ws->R, (const double *)p,
                       p);
    }
    ZI_HIP(hipGetLastError());
    return ZI_OK;
}

int pick_tile(const zi_system *sys, int ldp, int precision, int requested) {
    if (requested >= 0) return requested;
    if (sys->tuned_ldp[precision] == ldp && sys->tuned_tile[precision] >= 0)
        return sys->tuned_tile[precision];
    return auto_tile(ldp);
}

// Validate options, prepare the workspace and enqueue the initial state:
// X = x0 or 0, R = B - A X, the per-column scalars and P = D^-1 R.
// graphs: the iterations will be replayed as captured chunks (zi_solve_impl
// with opts.graph, and every batch).
zi_status solve_begin(zi_system *sys, const zi_solve_opts *o, SolveCtx &c, hipStream_t s,
                      bool graphs, bool gated = false) {
    c.t_start = std::chrono::steady_clock::now();
    const int n = sys->n;
    const int L = o->columns ? o->n_columns : sys->L;
    const int ldp = L + (L & 1);
    if (o->columns) {
        if (o->n_columns < 1 || o->n_columns > sys->L) {
            set_error("n_columns must be in [1, n_electrodes]");
            return ZI_EINVAL;
        }
        std::vector<int32_t> map(sys->L, -1);
        for (int k = 0; k < o->n_columns; ++k) {
            const int l = o->columns[k];
            if (l < 0 || l >= sys->L || map[l] >= 0) {
                set_error("columns[%d] = %d out of range or repeated", k, l);
                return ZI_EINVAL;
            }
            map[l] = k;
        }
        if (!sys->colmap) ZI_TRY(sys->pool.alloc(&sys->colmap, (size_t)sys->L));
        ZI_HIP(hipMemcpyAsync(sys->colmap, map.data(), sizeof(int32_t) * sys->L,
                              hipMemcpyHostToDevice, s));
        c.colmap = sys->colmap;
    }
    if (o->precond != ZI_PREC_JACOBI && o->precond != ZI_PREC_LDP) {
        set_error("unknown preconditioner %d", o->precond);
        return ZI_EINVAL;
    }
    if (o->precision != ZI_FP64 && o->precision != ZI_FP32_SPMM_IR) {
        set_error("unknown precision %d", o->precision);
        return ZI_EINVAL;
    }
    const int tile = pick_tile(sys, ldp, o->precision, o->tile);
    if (tile >= NTILES) {
        set_error("tile %d out of range", tile);
        return ZI_EINVAL;
    }
    if (o->form != ZI_PCG_AUTO && o->form != ZI_PCG_CLASSIC && o->form != ZI_PCG_SINGLE) {
        set_error("unknown PCG form %d", o->form);
        return ZI_EINVAL;
    }
    c.mixed = o->precision == ZI_FP32_SPMM_IR;
    if (c.mixed && o->form == ZI_PCG_SINGLE) {
        set_error("the single-reduction PCG form is FP64 only");
        return ZI_EINVAL;
    }
    c.sr = !c.mixed && o->form != ZI_PCG_CLASSIC;
    if (kTiles[tile].ring) ZI_TRY(ensure_ring(sys, s));
    ZI_TRY(ensure_ws(sys, ldp, max_nrt(n, ldp)));
    zi_solver_ws *ws = sys->ws;
    c.sys = sys;
    c.ws = ws;
    c.g = make_geom_for(c.sr ? GK::SPMM_SR : c.mixed ? GK::SPMM_DOT32 : GK::SPMM_DOT64, n, ldp,
                        tile);
    c.stile = stream_tile(ldp, c.mixed);
    c.rtile = kTiles[tile].ring ? c.stile : tile;
    c.grt = kTiles[tile].ring ? make_geom_for(GK::SPMM64, n, ldp, c.rtile) : c.g;
    c.gu = make_geom_for(c.mixed ? GK::UPDATE32 : GK::UPDATE64, n, ldp, c.stile);
    c.gp = make_geom_for(c.mixed ? GK::PUPDATE32 : GK::PUPDATE64, n, ldp, c.stile);
    c.gr = make_geom_for(c.mixed ? GK::RESIDUAL32 : GK::RESIDUAL64, n, ldp, c.stile);
    if (gated) {
        c.gate = ws->gate;
        c.g.gate = c.gu.gate = c.gp.gate = c.gr.gate = c.grt.gate = c.gate;
        ZI_TRY(open_gate(c, s));
    }
    c.tile = tile;
    c.ldp = ldp;
    c.L = L;
    c.maxit = o->maxit > 0 ? o->maxit : 50000;
    c.check = o->check_every > 0 ? o->check_every : 8;
    c.check = ((c.check + CHECK_MIN - 1) / CHECK_MIN) * CHECK_MIN;
    // a replayed graph chunk must end on an X flush (every LAZY iterations)
    if (graphs) c.check = ((c.check + LAZY - 1) / LAZY) * LAZY;
    if (c.mixed) {   // a divisor of MIXED_REPLACE: captured chunks repeat per phase
        int q = graphs ? LAZY : CHECK_MIN;
        while (q < c.check && q < MIXED_REPLACE) q *= 2;
        c.check = q;
    }
    c.tol = o->tol > 0 ? o->tol : 1e-8;
    c.tol2 = c.tol * c.tol;
    if (!(o->refine_eta >= 0.0 && o->refine_eta < 1.0)) {
        set_error("refine_eta must be in [0, 1) (got %g)", o->refine_eta);
        return ZI_EINVAL;
    }
    c.eta2 = c.mixed ? o->refine_eta * o->refine_eta : 0.0;
    c.timing = o->timing != 0 && o->graph == 0;
    c.timer = EventTimer{&ws->ev};
    c.h_active.assign(ldp, 0);
    Scal &sc = c.sc;
    sc.rho = ws->sc_d;
    sc.alpha = ws->sc_d + ldp;
    sc.beta = ws->sc_d + 2 * ldp;
    sc.bb = ws->sc_d + 3 * ldp;
    sc.rr = ws->sc_d + 4 * ldp;
    sc.tt = ws->sc_d + 5 * ldp;
    sc.bd = ws->sc_d + 6 * ldp;
    sc.kappa = ws->kap;
    sc.gate = c.gate;
    sc.iters = ws->sc_i;
    sc.active = ws->sc_i + ldp;
    sc.flag = ws->sc_i + 2 * ldp;

    hipLaunchKernelGGL(k_dinv, dim3((n + 255) / 256), dim3(256), 0, s,
                       o->precond == ZI_PREC_LDP ? sys->absrow : sys->diag, sys->perm, n,
                       ws->dinv);
    hipLaunchKernelGGL(k_kappa_part, dim3(KAPPA_BLOCKS), dim3(RED), 0, s,
                       (const int32_t *)sys->sp_ptr, (const double *)sys->sp_val,
                       (const double *)ws->dinv, n, ws->kap + 1);
    hipLaunchKernelGGL(k_kappa_final, dim3(1), dim3(RED), 0, s, (const double *)(ws->kap + 1),
                       KAPPA_BLOCKS, ws->kap);
    ZI_TRY(fill_i32(sc.flag, 0, 1, s));
    ZI_TRY(fill_f64(ws->X, 0.0, (size_t)n * ldp, s));
    if (o->x0) {
        ZI_TRY(gather_rows(o->x0, L, sys->perm, ws->X, ldp, n, L, s));
        ZI_TRY(true_residual(c, s, true));
    } else {
        if (c.mixed) {
            ZI_TILE_SWITCH(c.stile, launch_residual, c.gr, s, sys, (const int32_t *)c.colmap,
                           ws->dinv, (const double *)nullptr, reinterpret_cast<float *>(ws->R),
                           ws->part[0], ws->part[1], ws->part[2]);
        } else {
            ZI_TILE_SWITCH(c.stile, launch_residual, c.gr, s, sys, (const int32_t *)c.colmap,
                           ws->dinv, (const double *)nullptr, ws->R, ws->part[0], ws->part[1],
                           ws->part[2]);
        }
    }
    hipLaunchKernelGGL(k_red_init, dim3(ldp), dim3(RED), 0, s, sc, ws->part[0], ws->part[1],
                       ws->part[2], c.gr.nrt, L, c.tol2, c.eta2);
    if (c.sr) {
        // A D^-1, and zero S, lazy P and beta_0 (beta_0 = 0 multiplies them)
        const int64_t nnz = sys->sp_nnz;
        if (nnz > 0)
            hipLaunchKernelGGL(k_scale_cols, dim3((unsigned)((nnz + 255) / 256)), dim3(256), 0, s,
                               (const double *)sys->sp_val, (const int32_t *)sys->sp_col,
                               (const double *)ws->dinv, nnz, ws->vs);
        ZI_TRY(fill_f64(ws->Q, 0.0, (size_t)n * ldp, s));
        ZI_TRY(fill_f64(ws->P[0], 0.0, (size_t)n * ldp, s));
        ZI_TRY(fill_f64(ws->bring, 0.0, (size_t)LAZY * ldp, s));
    } else {
        ZI_TRY(enqueue_restart_direction(c, s));
    }
    if (c.gate)
        hipLaunchKernelGGL(k_gate, dim3(1), dim3(RED), 0, s, (const int32_t *)sc.active, ldp,
                           (const int32_t *)sc.flag, c.gate, (int32_t *)nullptr);
    ZI_TRY(read_active(c, s));
    c.done = !c.any_active;
    return ZI_OK;
}

// After the recurrence of every column has converged: in the mixed mode run
// one FP64 refinement step (true residual, restart of the columns that miss
// the tolerance).  Sets c.done when nothing is left to iterate.
zi_status solve_after_converged(SolveCtx &c, hipStream_t s) {
    if (c.h_flag || c.it >= c.maxit || !c.mixed) {
        c.done = true;
        return ZI_OK;
    }
    ZI_TRY(open_gate(c, s));
    ZI_TRY(flush_all(c, s));
    ZI_TRY(true_residual(c, s, true));
    hipLaunchKernelGGL(k_red_refine, dim3(c.ldp), dim3(RED), 0, s, c.sc, c.ws->part[1],
                       c.ws->part[2], c.gr.nrt, c.L, c.tol2, c.eta2);
    if (c.gate)
        hipLaunchKernelGGL(k_gate, dim3(1), dim3(RED), 0, s, (const int32_t *)c.sc.active, c.ldp,
                           (const int32_t *)c.sc.flag, c.gate, (int32_t *)nullptr);
    ZI_HIP(hipGetLastError());
    ZI_TRY(read_active(c, s));
    if (!c.any_active) {
        c.done = true;
        return ZI_OK;
    }
    ++c.refinements;
    return enqueue_restart_direction(c, s);
}

// Host check after a chunk, once the active flags have been taken.
zi_status solve_check_taken(SolveCtx &c, hipStream_t s) {
    if (c.h_flag || c.it >= c.maxit) {
        c.done = true;
        return ZI_OK;
    }
    if (!c.any_active) return solve_after_converged(c, s);
    return ZI_OK;
}

zi_status solve_check(SolveCtx &c, hipStream_t s) {
    ZI_TRY(read_active(c, s));
    return solve_check_taken(c, s);
}

// Host copies of a solve's final counts and norms (ldp entries each, and the
// breakdown flag), written by solve_end_enqueue, read by solve_end_finish
// once the stream has drained.
struct EndCopy {
    int32_t *iters = nullptr, *flag = nullptr;
    double *rr = nullptr, *bb = nullptr, *tr = nullptr;
    static size_t bytes(int ldp) { return (size_t)ldp * (sizeof(int32_t) + 3 * sizeof(double)) + 8; }
    void carve(void *p, int ldp) {   // from bytes(ldp) host bytes at p (8-byte aligned)
        char *q = static_cast<char *>(p);
        rr = reinterpret_cast<double *>(q);
        bb = rr + ldp;
        tr = bb + ldp;
        iters = reinterpret_cast<int32_t *>(tr + ldp);
        flag = iters + ldp;
    }
};

// The final flush, T in the caller's order and the statistics' copies, queued.
zi_status solve_end_enqueue(SolveCtx &c, double *T, zi_solve_stats *st, hipStream_t s,
                            const EndCopy &h) {
    zi_solver_ws *ws = c.ws;
    const int n = c.sys->n, L = c.L, ldp = c.ldp;
    const bool timing = c.timing;
    c.timing = false;
    ZI_TRY(open_gate(c, s));
    ZI_TRY(flush_all(c, s));
    c.timing = timing;
    ZI_TRY(gather_rows(ws->X, ldp, c.sys->iperm, T, L, n, L, s));
    ZI_HIP(hipMemcpyAsync(h.iters, c.sc.iters, sizeof(int32_t) * ldp, hipMemcpyDeviceToHost, s));
    ZI_HIP(hipMemcpyAsync(h.rr, c.sc.rr, sizeof(double) * ldp, hipMemcpyDeviceToHost, s));
    ZI_HIP(hipMemcpyAsync(h.bb, c.sc.bb, sizeof(double) * ldp, hipMemcpyDeviceToHost, s));
    if (st && st->relres_true) {
        ZI_TRY(true_residual(c, s, false));
        hipLaunchKernelGGL(k_red_sum, dim3(ldp), dim3(RED), 0, s, ws->part[2], c.gr.nrt,
                           c.sc.alpha);   // alpha reused as scratch
        ZI_HIP(hipGetLastError());
        ZI_HIP(hipMemcpyAsync(h.tr, c.sc.alpha, sizeof(double) * ldp, hipMemcpyDeviceToHost, s));
    }
    ZI_HIP(hipMemcpyAsync(h.flag, c.sc.flag, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    return ZI_OK;
}

zi_status solve_end_finish(SolveCtx &c, zi_solve_stats *st, const EndCopy &h);

zi_status solve_end(SolveCtx &c, double *T, zi_solve_stats *st, hipStream_t s) {
    std::vector<double> buf((EndCopy::bytes(c.ldp) + 7) / 8);
    EndCopy h;
    h.carve(buf.data(), c.ldp);
    ZI_TRY(solve_end_enqueue(c, T, st, s, h));
    ZI_HIP(hipStreamSynchronize(s));
    return solve_end_finish(c, st, h);
}

// Statistics and status of a solve from its host copies.
zi_status solve_end_finish(SolveCtx &c, zi_solve_stats *st, const EndCopy &h) {
    const int n = c.sys->n, L = c.L, ldp = c.ldp;
    const int32_t *h_iters = h.iters;
    const double *h_rr = h.rr, *h_bb = h.bb, *h_true = h.tr;
    const int32_t h_flag = *h.flag;
    if (st) {
        for (int k = 0; k < L; ++k) {
            if (st->iters) st->iters[k] = h_iters[k];
            const double bn = h_bb[k] > 0 ? h_bb[k] : 1.0;
            if (st->relres_rec) st->relres_rec[k] = h_bb[k] > 0 ? std::sqrt(h_rr[k] / bn) : 0.0;
            if (st->relres_true) st->relres_true[k] = h_bb[k] > 0 ? std::sqrt(h_true[k] / bn) : 0.0;
        }
        st->block_iters = c.it;
        st->refinements = c.refinements;
        st->tile = c.tile;
        st->n_kernels = 0;
        if (c.timing) {
            const int64_t pe = c.mixed ? 4 : 8;   // bytes of a P, Q or R entry
            const int64_t ne = (int64_t)n * ldp;
            const int64_t abytes = (int64_t)c.sys->sp_nnz * 12 + (int64_t)(n + 1) * 4;
            static const char *names_classic[4] = {"spmm_pq", "update", "pupdate", "xflush"};
            static const char *names_sr[3] = {"spmm_sr", "update", "pflush"};
            const int64_t bytes_classic[4] = {
                abytes + 2 * pe * ne,                      // read P, write Q
                3 * pe * ne + (int64_t)n * 8,              // r/w R, read Q, D^-1
                3 * pe * ne + (int64_t)n * 8,              // read R, P; write P; D^-1
                (16 + LAZY * pe) * ne};                    // r/w X, read LAZY directions
            const int64_t bytes_sr[3] = {
                abytes + 24 * ne + (int64_t)n * 8,         // read R; r/w S; D^-1
                24 * ne + (int64_t)n * 8,                  // read R, S; write R; D^-1
                (32 + LAZY * 8) * ne + (int64_t)n * 8};   // r/w P, X; read LAZY residuals
            const char *const *names = c.sr ? names_sr : names_classic;
            const int64_t *bytes = c.sr ? bytes_sr : bytes_classic;
            st->n_kernels = c.sr ? 3 : 4;
            for (int q = 0; q < st->n_kernels; ++q) {
                double ms = 0;
                for (size_t k = 0; k + 1 < c.ev[q].size(); k += 2) {
                    float a = 0;
                    ZI_HIP(hipEventElapsedTime(&a, c.ev[q][k], c.ev[q][k + 1]));
                    ms += a;
                }
                st->kernel_name[q] = names[q];
                st->kernel_ms[q] = ms;
                st->kernel_launches[q] = (int32_t)(c.ev[q].size() / 2);
                st->kernel_calls[q] = c.calls[q];
                st->kernel_bytes[q] = bytes[q];
            }
        }
        st->seconds = std::chrono::duration<double>(std::chrono::steady_clock::now() - c.t_start).count();
    }
    if (h_flag) {
        set_error("PCG breakdown: p^T A p <= 0 (matrix not positive definite)");
        return ZI_EBREAKDOWN;
    }
    if (c.any_active) {
        set_error("PCG did not reach tol %.3g within %d iterations", c.tol, c.maxit);
        return ZI_ENOTCONV;
    }
    return ZI_OK;
}

// Capture `count` iterations of every listed solve into one graph: one
// branch per solve (its own stream), forked from and joined back to the
// internal capture stream `origin` (never the caller's stream, which may be
// the null stream).  The graph is launched on the caller's stream.
// Captured chunks of check iterations.  In the mixed mode the reliable updates
// fall on fixed iterations, so a chunk's graph depends on its phase in the
// MIXED_REPLACE cycle: one graph per phase.
struct GraphSet {
    std::vector<hipGraphExec_t> ex;
    ~GraphSet() { clear(); }
    void clear() {
        for (auto e : ex)
            if (e) (void)hipGraphExecDestroy(e);
        ex.clear();
    }
    void reset(const SolveCtx &c) {
        clear();
        ex.assign(c.mixed ? MIXED_REPLACE / c.check : 1, nullptr);
    }
    // As reset, but the old graphs may still be executing (a replay is kept
    // queued): they go to `grave`, destroyed once the stream has drained.
    void retire(const SolveCtx &c, std::vector<hipGraphExec_t> &grave) {
        for (auto e : ex)
            if (e) grave.push_back(e);
        ex.assign(c.mixed ? MIXED_REPLACE / c.check : 1, nullptr);
    }
    static int phase(const SolveCtx &c) {
        return c.mixed ? (c.it % MIXED_REPLACE) / c.check : 0;
    }
};

zi_status capture_graph(std::vector<SolveCtx *> &cs, std::vector<hipStream_t> &streams,
                        int count, hipStream_t origin, hipGraphExec_t *exec) {
    hipEvent_t fork, join_ev;
    ZI_HIP(hipEventCreateWithFlags(&fork, hipEventDisableTiming));
    std::vector<hipEvent_t> joins(cs.size());
    for (auto &e : joins) ZI_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipGraph_t graph;
    ZI_HIP(hipStreamBeginCapture(origin, hipStreamCaptureModeThreadLocal));
    zi_status st = ZI_OK;
    if (hipEventRecord(fork, origin) != hipSuccess) st = ZI_EDEVICE;
    for (size_t k = 0; k < cs.size() && st == ZI_OK; ++k) {
        if (hipStreamWaitEvent(streams[k], fork, 0) != hipSuccess) {
            st = ZI_EDEVICE;
            break;
        }
        const int flushed = cs[k]->flushed;
        st = enqueue_iterations(*cs[k], count, streams[k]);
        cs[k]->flushed = flushed;   // the replays, not the capture, advance it
        if (st == ZI_OK && cs[k]->gate)
            hipLaunchKernelGGL(k_gate, dim3(1), dim3(RED), 0, streams[k],
                               (const int32_t *)cs[k]->sc.active, cs[k]->ldp,
                               (const int32_t *)cs[k]->sc.flag, cs[k]->gate, cs[k]->gate_out);
        if (st == ZI_OK && hipEventRecord(joins[k], streams[k]) != hipSuccess) st = ZI_EDEVICE;
        if (st == ZI_OK && hipStreamWaitEvent(origin, joins[k], 0) != hipSuccess) st = ZI_EDEVICE;
    }
    hipError_t ee = hipStreamEndCapture(origin, &graph);
    (void)join_ev;
    if (st == ZI_OK && ee != hipSuccess) {
        set_error("hipStreamEndCapture failed: %s", hipGetErrorString(ee));
        st = ZI_EDEVICE;
    }
    if (st == ZI_OK) {
        hipError_t ie = hipGraphInstantiate(exec, graph, nullptr, nullptr, 0);
        if (ie != hipSuccess) {
            set_error("hipGraphInstantiate failed: %s", hipGetErrorString(ie));
            st = ZI_EDEVICE;
        }
    }
    if (ee == hipSuccess) (void)hipGraphDestroy(graph);
    (void)hipEventDestroy(fork);
    for (auto &e : joins) (void)hipEventDestroy(e);
    if (st == ZI_EDEVICE && zi::g_err_empty()) set_error("graph capture failed");
    return st;
}

}  // namespace

zi_status zi_solve_impl(zi_system *sys, const zi_solve_opts *o, double *T, zi_solve_stats *st,
                        hipStream_t s) {
    SolveCtx c;
    ZI_TRY(solve_begin(sys, o, c, s, o->graph != 0));
    if (o->graph) {
        std::vector<SolveCtx *> cs{&c};
        hipStream_t side, cap;
        ZI_HIP(hipStreamCreateWithFlags(&side, hipStreamNonBlocking));
        ZI_HIP(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking));
        std::vector<hipStream_t> streams{side};
        GraphSet gs;
        gs.reset(c);
        zi_status r = ZI_OK;
        while (!c.done && r == ZI_OK) {
            const int chunk = c.check;
            if (c.maxit - c.it < chunk) {   // the tail runs eagerly
                r = enqueue_iterations(c, c.maxit - c.it, s);
                if (r != ZI_OK) break;
                c.it = c.maxit;
                r = solve_check(c, s);
                continue;
            }
            hipGraphExec_t &exec = gs.ex[GraphSet::phase(c)];
            if (!exec) {
                r = capture_graph(cs, streams, chunk, cap, &exec);
                if (r != ZI_OK) break;
            }
            if (hipGraphLaunch(exec, s) != hipSuccess) {
                set_error("hipGraphLaunch failed");
                r = ZI_EDEVICE;
                break;
            }
            c.it += chunk;
            c.flushed = c.it;   // every chunk ends on an X flush (chunk % LAZY == 0)
            r = solve_check(c, s);
        }
        gs.clear();
        (void)hipStreamDestroy(side);
        (void)hipStreamDestroy(cap);
        ZI_TRY(r);
    } else {
        while (!c.done) {
            const int chunk = std::min(c.check, c.maxit - c.it);
            ZI_TRY(enqueue_iterations(c, chunk, s));
            c.it += chunk;
            ZI_TRY(solve_check(c, s));
        }
    }
    return solve_end(c, T, st, s);
}

zi_status zi_solve_batch_impl(zi_system *const *systems, int32_t nsys, const zi_solve_opts *o,
                              double *const *T, zi_solve_stats *st, hipStream_t s) {
    // (gate, breakdown flag) of every head after a replay, and two pinned
    // host copies: the host reads one replay's copy while the next runs.
    // After them in the same pinned block: every head's final statistics.
    size_t end_bytes = 0;
    for (int k = 0; k < nsys; ++k) {
        const int L = o->columns ? o->n_columns : systems[k]->L;
        end_bytes += EndCopy::bytes(L + (L & 1));
    }
    const size_t flag_bytes = ((sizeof(int32_t) * 4 * nsys + 7) / 8) * 8;
    int32_t *gates_d = nullptr, *gates_h = nullptr;
    ZI_HIP(hipMalloc(reinterpret_cast<void **>(&gates_d), sizeof(int32_t) * 2 * nsys));
    if (hipHostMalloc(reinterpret_cast<void **>(&gates_h), flag_bytes + end_bytes) !=
        hipSuccess) {
        (void)hipFree(gates_d);
        set_error("hipHostMalloc of the batch flags failed");
        return ZI_ENOMEM;
    }
    struct Bufs {
        int32_t *d, *h;
        ~Bufs() {
            (void)hipFree(d);
            (void)hipHostFree(h);
        }
    } bufs{gates_d, gates_h};
    std::vector<SolveCtx> cs(nsys);
    for (int k = 0; k < nsys; ++k) {
        ZI_TRY(solve_begin(systems[k], o, cs[k], s, true, true));
        cs[k].timing = false;   // events cannot be captured
        cs[k].gate_out = gates_d + 2 * k;
    }
    ZI_TRY(fill_i32(gates_d, 0, (size_t)2 * nsys, s));
    // Heads are captured in groups of BATCH_GROUP, each group's graph launched
    // on a stream of its own, forked from and joined back to the caller's
    // stream.  A head that has converged stays in its group's graph, gated
    // (its kernels return at once), so finishing heads cost no new capture; a
    // group is captured again only for a head that is not in its graph or
    // whose iteration phase moved (a refinement restart).
    constexpr int BATCH_GROUP = 8;
    const int ngroups = (nsys + BATCH_GROUP - 1) / BATCH_GROUP;
    // one stream per system (capture branches), per group (launch) + capture origin
    std::vector<hipStream_t> streams(nsys + ngroups + 1);
    for (auto &x : streams) ZI_HIP(hipStreamCreateWithFlags(&x, hipStreamNonBlocking));
    std::vector<hipEvent_t> events(ngroups + 3);   // joins, fork, flags copied (2)
    for (auto &e : events) ZI_HIP(hipEventCreateWithFlags(&e, hipEventDisableTiming));
    hipStream_t cap = streams[nsys + ngroups];
    struct Guard {
        std::vector<hipStream_t> &v;
        std::vector<hipEvent_t> &e;
        ~Guard() {
            for (auto x : v) (void)hipStreamDestroy(x);
            for (auto x : e) (void)hipEventDestroy(x);
        }
    } guard{streams, events};
    const int chunk = cs[0].check;   // same options for every system
    std::vector<GraphSet> gsets(ngroups);
    std::vector<hipGraphExec_t> grave;   // replaced graphs, destroyed after the last sync
    std::vector<std::vector<int>> last(ngroups);
    std::vector<int> epoch(nsys, 0);   // bumped when the host restarts a head (refinement)
    struct Replay {
        bool live = false;
        std::vector<int> heads, epochs;
    } rp[2];
    zi_status r = ZI_OK;

    auto members = [&]() {
        std::vector<int> m;
        for (int k = 0; k < nsys; ++k)
            if (!cs[k].done && cs[k].maxit - cs[k].it >= chunk) m.push_back(k);
        return m;
    };
    // Replay one chunk of every member (all groups), then copy the flags.
    auto launch = [&](const std::vector<int> &mem, int p) -> zi_status {
        std::vector<int> gm;
        ZI_HIP(hipEventRecord(events[ngroups], s));
        for (int grp = 0; grp < ngroups; ++grp) {
            gm.clear();
            for (int k : mem)
                if (k / BATCH_GROUP == grp) gm.push_back(k);
            if (gm.empty()) continue;
            bool covered = !last[grp].empty();
            for (int k : gm)
                covered = covered &&
                          std::find(last[grp].begin(), last[grp].end(), k) != last[grp].end();
            // the graph's active heads advance together: the first gives the phase
            const int ph = GraphSet::phase(cs[gm[0]]);
            if (covered && !gsets[grp].ex[ph] && gm != last[grp])
                covered = false;   // a new capture leaves the converged heads out
            if (!covered) {   // the last replay may still run the old graphs
                gsets[grp].retire(cs[gm[0]], grave);
                last[grp] = gm;
            }
            hipGraphExec_t &exec = gsets[grp].ex[ph];
            if (!exec) {
                std::vector<SolveCtx *> sel;
                std::vector<hipStream_t> ss;
                for (int k : last[grp]) {
                    sel.push_back(&cs[k]);
                    ss.push_back(streams[k]);
                }
                ZI_TRY(capture_graph(sel, ss, chunk, cap, &exec));
            }
            hipStream_t ls = streams[nsys + grp];
            if (hipStreamWaitEvent(ls, events[ngroups], 0) != hipSuccess ||
                hipGraphLaunch(exec, ls) != hipSuccess ||
                hipEventRecord(events[grp], ls) != hipSuccess ||
                hipStreamWaitEvent(s, events[grp], 0) != hipSuccess) {
                set_error("hipGraphLaunch failed");
                return ZI_EDEVICE;
            }
        }
        for (int k : mem) {
            cs[k].it += chunk;
            cs[k].flushed = cs[k].it;   // every chunk ends on a flush
        }
        ZI_HIP(hipMemcpyAsync(gates_h + (size_t)p * 2 * nsys, gates_d,
                              sizeof(int32_t) * 2 * nsys, hipMemcpyDeviceToHost, s));
        ZI_HIP(hipEventRecord(events[ngroups + 1 + p], s));
        rp[p].live = true;
        rp[p].heads = mem;
        rp[p].epochs.clear();
        for (int k : mem) rp[p].epochs.push_back(epoch[k]);
        return ZI_OK;
    };
    // Solves within one chunk of maxit finish on their own (no graph).
    auto tails = [&]() -> zi_status {
        for (int k = 0; k < nsys; ++k) {
            if (cs[k].done || cs[k].maxit - cs[k].it >= chunk) continue;
            ZI_TRY(open_gate(cs[k], s));
            while (!cs[k].done) {
                const int rest = cs[k].maxit - cs[k].it;
                ZI_TRY(enqueue_iterations(cs[k], rest, s));
                cs[k].it += rest;
                ZI_TRY(solve_check(cs[k], s));
            }
        }
        return ZI_OK;
    };

    int par = 0;
    r = tails();
    if (r == ZI_OK) {
        const std::vector<int> m = members();
        if (!m.empty()) r = launch(m, par);
    }
    while (r == ZI_OK && rp[par].live) {
        // The next replay is queued before this one's flags are read, with the
        // members as known now: a head found converged below is still in it,
        // gated, and costs only its launches.
        const std::vector<int> next = members();
        if (!next.empty()) r = launch(next, par ^ 1);
        if (r != ZI_OK) break;
        if (hipEventSynchronize(events[ngroups + 1 + par]) != hipSuccess) {
            set_error("hipEventSynchronize failed");
            r = ZI_EDEVICE;
            break;
        }
        const int32_t *gh = gates_h + (size_t)par * 2 * nsys;
        for (size_t j = 0; j < rp[par].heads.size() && r == ZI_OK; ++j) {
            const int k = rp[par].heads[j];
            // flags of a replay launched before the head was restarted are stale
            if (cs[k].done || rp[par].epochs[j] != epoch[k]) continue;
            cs[k].any_active = gh[2 * k] != 0;
            cs[k].h_flag = gh[2 * k + 1];
            if (!cs[k].any_active && rp[par ^ 1].live) {
                const auto &q = rp[par ^ 1].heads;
                if (std::find(q.begin(), q.end(), k) != q.end()) {
                    // the queued replay found the head's gate closed and did
                    // nothing for it: its iteration count (which fixes the
                    // ring slots and the reliable-update phase) goes back, and
                    // its group is captured again without it (a recapture of
                    // a few milliseconds costs less than the gated launches
                    // of a head that stays in its group's graph)
                    cs[k].it -= chunk;
                    cs[k].flushed = cs[k].it;
                    last[k / BATCH_GROUP].clear();
                }
            }
            const int ref = cs[k].refinements;
            r = solve_check_taken(cs[k], s);
            if (cs[k].refinements != ref) ++epoch[k];
        }
        rp[par].live = false;
        if (r == ZI_OK) r = tails();
        par ^= 1;
        if (r == ZI_OK && !rp[par].live) {   // nothing queued: heads restarted since
            const std::vector<int> m = members();
            if (!m.empty()) r = launch(m, par);
        }
    }
    // Every head's final flush, T and statistics are queued behind the last
    // replay; the graphs are destroyed (milliseconds of host work each) once
    // the replays have run, while the GPU works on the heads' ends.
    hipEvent_t replays_done = events[ngroups + 1];
    const bool ev_ok = hipEventRecord(replays_done, s) == hipSuccess;
    std::vector<EndCopy> ends(nsys);
    char *endbuf = reinterpret_cast<char *>(gates_h) + flag_bytes;
    for (size_t k = 0, off = 0; r == ZI_OK && k < (size_t)nsys; ++k) {
        ends[k].carve(endbuf + off, cs[k].ldp);
        off += EndCopy::bytes(cs[k].ldp);
        r = solve_end_enqueue(cs[k], T[k], st ? &st[k] : nullptr, s, ends[k]);
    }
    if (!ev_ok || hipEventSynchronize(replays_done) != hipSuccess)
        (void)hipStreamSynchronize(s);   // no replay left running before graphs are destroyed
    for (auto &g : gsets) g.clear();
    for (auto e : grave) (void)hipGraphExecDestroy(e);
    const bool synced = hipStreamSynchronize(s) == hipSuccess;
    zi_status worst = r;
    if (r == ZI_OK && !synced) {
        set_error("hipStreamSynchronize failed");
        worst = ZI_EDEVICE;
    }
    if (worst == ZI_OK)
        for (int k = 0; k < nsys; ++k) {
            const zi_status e = solve_end_finish(cs[k], st ? &st[k] : nullptr, ends[k]);
            if (e != ZI_OK && worst == ZI_OK) worst = e;
        }
    return worst;
}

zi_status zi_autotune_impl(zi_system *sys, int32_t precision, int32_t *best, double *ms_out,
                           hipStream_t s) {
    const int n = sys->n, L = sys->L, ldp = L + (L & 1);
    if (precision != ZI_FP64 && precision != ZI_FP32_SPMM_IR) {
        set_error("unknown precision %d", precision);
        return ZI_EINVAL;
    }
    ZI_TRY(ensure_ws(sys, ldp, max_nrt(n, ldp)));
    zi_solver_ws *ws = sys->ws;
    const size_t blk = (size_t)n * ldp;
    // smooth, finite operands: blocks of ones, step lengths and betas 0.5,
    // D^-1 = 1 (the values only have to keep every kernel's arithmetic finite)
    for (int j = 0; j < LAZY; ++j) ZI_TRY(fill_f64(ws->P[j], 1.0, blk, s));
    ZI_TRY(fill_f64(ws->R, 1.0, blk, s));
    ZI_TRY(fill_f64(ws->Q, 0.0, blk, s));   // also 0.0f as a float block
    ZI_TRY(fill_f64(ws->X, 0.0, blk, s));
    ZI_TRY(fill_f64(ws->dinv, 1.0, (size_t)n, s));
    ZI_TRY(fill_f64(ws->aring, 0.5, (size_t)LAZY * ldp, s));
    ZI_TRY(fill_f64(ws->bring, 0.5, (size_t)LAZY * ldp, s));
    if (precision == ZI_FP32_SPMM_IR) {
        hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((blk + 255) / 256)), dim3(256), 0, s, ws->R,
                           (int64_t)blk, reinterpret_cast<float *>(ws->P[0]));
        hipLaunchKernelGGL(k_to_f32, dim3((unsigned)((blk + 255) / 256)), dim3(256), 0, s, ws->P[1],
                           (int64_t)blk, reinterpret_cast<float *>(ws->R));
    }
    ZI_HIP(hipGetLastError());
    hipEvent_t e0, e1;
    ZI_HIP(hipEventCreate(&e0));
    ZI_HIP(hipEventCreate(&e1));
    int bt = 0;
    double bms = 1e30;
    // Each tile is scored by the iteration's SpMM, the best of three launches
    // after a warm-up: the other kernels of an iteration run with one fixed
    // geometry whatever the tile.
    const bool f32 = precision == ZI_FP32_SPMM_IR;
    ZI_TRY(ensure_ring(sys, s));
    for (int t = 0; t < NTILES; ++t) {
        const Geom gs = make_geom_for(f32 ? GK::SPMM_DOT32 : GK::SPMM_SR, n, ldp, t);
        double total = 0.0;
        const int kinds = 1;
        for (int kind = 0; kind < kinds; ++kind) {
            double tmin = 1e30;
            for (int rep = 0; rep < 4; ++rep) {
                ZI_HIP(hipEventRecord(e0, s));
                if (precision == ZI_FP32_SPMM_IR) {
                    float *P0 = reinterpret_cast<float *>(ws->P[0]);
                    float *P1 = reinterpret_cast<float *>(ws->P[1]);
                    float *Qf = reinterpret_cast<float *>(ws->Q);
                    float *Rf = reinterpret_cast<float *>(ws->R);
                    (void)kind;
                    (void)P1;
                    (void)Rf;
                    if (kTiles[t].ring)
                        launch_spmm_ring<float, false>(gs, s, sys->ring_halo, sys->sp_ptr,
                                                       sys->sp_col, (const double *)sys->sp_val,
                                                       nullptr, (const float *)P0, nullptr, Qf,
                                                       ws->part[0], (const double *)ws->aring);
                    else
                        ZI_TILE_SWITCH(t, launch_spmm, gs, s, sys->sp_ptr, sys->sp_col,
                                       (const double *)sys->sp_val, (const float *)P0, Qf,
                                       ws->part[0], (const double *)ws->aring);
                } else if (kTiles[t].ring) {
                    launch_spmm_ring<double, true>(gs, s, sys->ring_halo, sys->sp_ptr,
                                                   sys->sp_col, (const double *)sys->sp_val,
                                                   (const double *)ws->dinv,
                                                   (const double *)ws->P[0],
                                                   (const double *)ws->bring, ws->Q, ws->part[0],
                                                   (const double *)ws->aring);
                } else {   // the FP64 solve's default (single-reduction) kernels
                    ZI_TILE_SWITCH(t, launch_spmm_sr, gs, s, sys->sp_ptr, sys->sp_col,
                                   (const double *)sys->sp_val, (const double *)ws->dinv,
                                   (const double *)ws->P[0], (const double *)ws->bring, ws->Q,
                                   ws->part[0], (const double *)ws->aring);
                }
                ZI_HIP(hipGetLastError());
                ZI_HIP(hipEventRecord(e1, s));
                ZI_HIP(hipEventSynchronize(e1));
                float ms = 0;
                ZI_HIP(hipEventElapsedTime(&ms, e0, e1));
                if (rep > 0) tmin = std::min(tmin, (double)ms);   // first run warms up
            }
            total += tmin;   // the flushes have their own geometry: not scored
        }
        if (ms_out) ms_out[t] = total;
        if (total < bms) {
            bms = total;
            bt = t;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    sys->tuned_tile[precision] = bt;
    sys->tuned_ldp[precision] = ldp;
    if (best) *best = bt;
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
    if (kTiles[tile].ring) {
        set_error("tile %s serves the solver's products only", kTiles[tile].name);
        return ZI_EINVAL;
    }
    const int n = sys->n;
    const Geom g = make_geom_for(GK::SPMM64, n, k, tile);
    Pool tmp;   // the blocks in solver row order
    double *Xp = nullptr, *Yp = nullptr;
    ZI_TRY(tmp.alloc(&Xp, (size_t)n * k));
    ZI_TRY(tmp.alloc(&Yp, (size_t)n * k));
    ZI_TRY(gather_rows(X, k, sys->perm, Xp, k, n, k, s));
    hipEvent_t e0, e1;
    ZI_HIP(hipEventCreate(&e0));
    ZI_HIP(hipEventCreate(&e1));
    ZI_HIP(hipEventRecord(e0, s));
    ZI_TILE_SWITCH(tile, launch_spmm, g, s, sys->sp_ptr, sys->sp_col, (const double *)sys->sp_val,
                   (const double *)Xp, Yp, (double *)nullptr);
    ZI_HIP(hipGetLastError());
    ZI_HIP(hipEventRecord(e1, s));
    ZI_TRY(gather_rows(Yp, k, sys->iperm, Y, k, n, k, s));
    ZI_HIP(hipStreamSynchronize(s));
    float t = 0;
    ZI_HIP(hipEventElapsedTime(&t, e0, e1));
    if (ms) *ms = t;
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    return ZI_OK;
}

namespace zi {

// Y = A X for a float32 CSR matrix and n x ld float32 row-major blocks (ld
// even), used by the warm-start network's graph aggregation.
zi_status spmm_f32(const int32_t *rp, const int32_t *ci, const float *va, const float *X, float *Y,
                   int32_t n, int32_t ld, hipStream_t s) {
    const int tile = auto_tile(ld);
    const Geom g = make_geom_for(GK::SPMM32F, n, ld, tile);
    ZI_TILE_SWITCH(tile, launch_spmm, g, s, rp, ci, va, X, Y, (double *)nullptr);
    ZI_HIP(hipGetLastError());
    return ZI_OK;
}

}  // namespace zi
