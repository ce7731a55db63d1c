// Assembly of the grounded CEM system of Eq. (u_system), App. A.1.
//
// Design (deterministic, no floating-point atomics):
//   1. validate indices / conductivity / coordinates (direct reads only);
//   2. per-tet geometry: gradients of the linear basis functions and the 10
//      unique entries of the element stiffness matrix;
//   3. node -> tet incidence by counting sort, each node's list ascending;
//   4. CSR structure: per node, the sorted set of vertices of its incident
//      tets (thread-private sorted list in LDS), scan, fill;
//   5. values by a row-owned gather: node i sums K^e_{ij} of its incident
//      tets in ascending tet order (no colouring, no atomics);
//   6. boundary faces by bucketing the 4e faces on their smallest edge (an
//      index into the CSR) and counting the third vertex;
//   7. CEM: triangle areas, contact areas, surface mass into A, B node-major
//      and electrode-major, all in fixed orders;
//   8. ground node (smallest admissible) and the symmetric ground fix.
#include <algorithm>
#include <climits>
#include <cmath>
#include <cstring>

#include "zi_internal.h"

namespace {

using namespace zi;

inline unsigned grid_for(size_t n, int threads) {
    return (unsigned)((n + threads - 1) / threads);
}

__device__ __forceinline__ int sym10(int a, int b) {
    // (0,0)0 (0,1)1 (0,2)2 (0,3)3 (1,1)4 (1,2)5 (1,3)6 (2,2)7 (2,3)8 (3,3)9
    if (a > b) {
        int t = a;
        a = b;
        b = t;
    }
    return a == 0 ? b : (a == 1 ? 3 + b : (a == 2 ? 5 + b : 9));
}

__device__ __forceinline__ int32_t find_col(const int32_t *col, int32_t s, int32_t e, int32_t j) {
    // lower_bound of j in col[s, e); returns -1 if absent
    int32_t lo = s, hi = e;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (col[mid] < j)
            lo = mid + 1;
        else
            hi = mid;
    }
    return (lo < e && col[lo] == j) ? lo : -1;
}

// ---------------------------------------------------------------------------
// 1. validation
// ---------------------------------------------------------------------------

__global__ void k_validate_tets(const int32_t *tets, const double *sigma, int ncomp, int32_t e,
                                int32_t n, int *flags) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= e) return;
    int f = 0;
    int v[4];
#pragma unroll
    for (int a = 0; a < 4; ++a) {
        v[a] = tets[4 * t + a];
        if (v[a] < 0 || v[a] >= n) f |= F_TET_INDEX;
    }
    if (v[0] == v[1] || v[0] == v[2] || v[0] == v[3] || v[1] == v[2] || v[1] == v[3] ||
        v[2] == v[3])
        f |= F_TET_INDEX;
    if (ncomp == 1) {
        const double s = sigma[t];
        if (!(s > 0.0) || !isfinite(s)) f |= F_SIGMA;
    } else {
        const double *s = sigma + 6 * t;
        bool ok = true;
        for (int k = 0; k < 6; ++k) ok = ok && isfinite(s[k]);
        // Sylvester: leading minors of [[s11 s12 s13][s12 s22 s23][s13 s23 s33]]
        const double m1 = s[0];
        const double m2 = s[0] * s[1] - s[3] * s[3];
        const double m3 = s[0] * (s[1] * s[2] - s[5] * s[5]) - s[3] * (s[3] * s[2] - s[5] * s[4]) +
                          s[4] * (s[3] * s[5] - s[1] * s[4]);
        if (!ok || !(m1 > 0.0) || !(m2 > 0.0) || !(m3 > 0.0)) f |= F_SIGMA;
    }
    if (f) atomicOr(flags, f);
}

__global__ void k_validate_nodes(const double *nodes, int32_t n, int *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (!isfinite(nodes[3 * i]) || !isfinite(nodes[3 * i + 1]) || !isfinite(nodes[3 * i + 2]))
        atomicOr(flags, F_COORD);
}

__global__ void k_validate_tris(const int32_t *tris, const int32_t *te, int32_t nt, int32_t n,
                                int32_t L, int *flags) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nt) return;
    int f = 0;
    const int a = tris[3 * k], b = tris[3 * k + 1], c = tris[3 * k + 2];
    if (a < 0 || a >= n || b < 0 || b >= n || c < 0 || c >= n || a == b || a == c || b == c)
        f |= F_TRI_INDEX;
    const int l = te[k];
    if (l < 0 || l >= L) f |= F_TRI_ELECTRODE;
    if (f) atomicOr(flags, f);
}

// ---------------------------------------------------------------------------
// 2. element geometry and stiffness
// ---------------------------------------------------------------------------

struct V3 {
    double x, y, z;
};
__device__ __forceinline__ V3 sub(V3 a, V3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ V3 cross(V3 a, V3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double dot(V3 a, V3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ V3 load3(const double *p, int64_t i) {
    return {p[3 * i], p[3 * i + 1], p[3 * i + 2]};
}

// Gradients of psi_0..psi_3 on tet t.  With rows J0 = x1-x0, J1 = x2-x0,
// J2 = x3-x0 the inverse of J has columns (J1xJ2, J2xJ0, J0xJ1)/det, which are
// grad psi_1..3; grad psi_0 = -sum.  Returns det J; sets *degenerate.
__device__ double tet_gradients(const double *nodes, const int32_t *tets, int64_t t, V3 g[4],
                                bool *degenerate) {
    const V3 x0 = load3(nodes, tets[4 * t]), x1 = load3(nodes, tets[4 * t + 1]);
    const V3 x2 = load3(nodes, tets[4 * t + 2]), x3 = load3(nodes, tets[4 * t + 3]);
    const V3 J0 = sub(x1, x0), J1 = sub(x2, x0), J2 = sub(x3, x0);
    const V3 c0 = cross(J1, J2), c1 = cross(J2, J0), c2 = cross(J0, J1);
    const double det = dot(J0, c0);
    double lmax = fmax(fmax(dot(J0, J0), dot(J1, J1)), dot(J2, J2));
    const V3 e12 = sub(x2, x1), e13 = sub(x3, x1), e23 = sub(x3, x2);
    lmax = fmax(lmax, fmax(fmax(dot(e12, e12), dot(e13, e13)), dot(e23, e23)));
    lmax = sqrt(lmax);
    *degenerate = !(fabs(det) > 1e-12 * lmax * lmax * lmax) || !isfinite(det);
    const double inv = 1.0 / det;
    g[1] = {c0.x * inv, c0.y * inv, c0.z * inv};
    g[2] = {c1.x * inv, c1.y * inv, c1.z * inv};
    g[3] = {c2.x * inv, c2.y * inv, c2.z * inv};
    g[0] = {-(g[1].x + g[2].x + g[3].x), -(g[1].y + g[2].y + g[3].y),
            -(g[1].z + g[2].z + g[3].z)};
    return det;
}

__global__ void k_element(const double *nodes, const int32_t *tets, const double *sigma,
                          int ncomp, int32_t e, double *Ke, int *flags) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= e) return;
    V3 g[4];
    bool degenerate;
    const double det = tet_gradients(nodes, tets, t, g, &degenerate);
    if (degenerate) {
        atomicOr(flags, F_DEGENERATE);
        return;
    }
    const double vol = fabs(det) / 6.0;
    V3 sg[4];
    if (ncomp == 1) {
        const double w = vol * sigma[t];
#pragma unroll
        for (int b = 0; b < 4; ++b) sg[b] = {w * g[b].x, w * g[b].y, w * g[b].z};
    } else {
        const double *s = sigma + 6 * t;
#pragma unroll
        for (int b = 0; b < 4; ++b) {
            sg[b] = {vol * (s[0] * g[b].x + s[3] * g[b].y + s[4] * g[b].z),
                     vol * (s[3] * g[b].x + s[1] * g[b].y + s[5] * g[b].z),
                     vol * (s[4] * g[b].x + s[5] * g[b].y + s[2] * g[b].z)};
        }
    }
    double *k = Ke + 10 * t;
    k[0] = dot(g[0], sg[0]);
    k[1] = dot(g[0], sg[1]);
    k[2] = dot(g[0], sg[2]);
    k[3] = dot(g[0], sg[3]);
    k[4] = dot(g[1], sg[1]);
    k[5] = dot(g[1], sg[2]);
    k[6] = dot(g[1], sg[3]);
    k[7] = dot(g[2], sg[2]);
    k[8] = dot(g[2], sg[3]);
    k[9] = dot(g[3], sg[3]);
}

// ---------------------------------------------------------------------------
// 4. CSR structure: one thread per row, private sorted list in LDS
// ---------------------------------------------------------------------------

constexpr int ROW_THREADS = 64;

__global__ __launch_bounds__(ROW_THREADS) void k_row_struct(const int32_t *inc_ptr,
                                                            const int32_t *inc,
                                                            const int32_t *tets, int32_t n,
                                                            int32_t *rowlen,
                                                            const int32_t *row_ptr,
                                                            int32_t *col, int *flags) {
    __shared__ int32_t lst[MAX_NEIGHBOURS * ROW_THREADS];
    const int tid = threadIdx.x;
    const int64_t i = (int64_t)blockIdx.x * ROW_THREADS + tid;
    if (i >= n) return;
    int cnt = 0;
    bool over = false;
    for (int32_t p = inc_ptr[i]; p < inc_ptr[i + 1]; ++p) {
        const int64_t t = inc[p] >> 2;
        for (int b = 0; b < 4; ++b) {
            const int32_t j = tets[4 * t + b];
            int pos = cnt;
            while (pos > 0 && lst[(pos - 1) * ROW_THREADS + tid] > j) --pos;
            if (pos > 0 && lst[(pos - 1) * ROW_THREADS + tid] == j) continue;
            if (cnt == MAX_NEIGHBOURS) {
                over = true;
                continue;
            }
            for (int q = cnt; q > pos; --q)
                lst[q * ROW_THREADS + tid] = lst[(q - 1) * ROW_THREADS + tid];
            lst[pos * ROW_THREADS + tid] = j;
            ++cnt;
        }
    }
    if (over) atomicOr(flags, F_DEGREE);
    if (col == nullptr) {
        rowlen[i] = cnt;
    } else {
        const int32_t base = row_ptr[i];
        for (int q = 0; q < cnt; ++q) col[base + q] = lst[q * ROW_THREADS + tid];
    }
}

// ---------------------------------------------------------------------------
// 5. values: row-owned gather in ascending tet order
// ---------------------------------------------------------------------------

// RV lanes per row; lane j owns the row's entries s + j, s + j + RV, ... and
// adds, over the row's incident tets in ascending tet order, the element
// entry that couples the row to its column.  Every entry is summed in the
// same order as a row-serial loop would (a tet has distinct vertices, so at
// most one of its entries lands on a given column).
constexpr int RV = 16;

__global__ void k_row_values(const int32_t *inc_ptr, const int32_t *inc, const int32_t *tets,
                             const double *Ke, const int32_t *row_ptr, const int32_t *col,
                             double *val, int32_t n) {
    const int64_t gid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t i = gid / RV;
    const int lane = (int)(gid % RV);
    if (i >= n) return;
    const int32_t s = row_ptr[i], e = row_ptr[i + 1];
    const int32_t p0 = inc_ptr[i], p1 = inc_ptr[i + 1];
    for (int32_t q0 = s; q0 < e; q0 += RV) {
        const int32_t q = q0 + lane;
        const int32_t cq = q < e ? col[q] : -1;
        double acc = 0.0;
        for (int32_t p = p0; p < p1; ++p) {
            const int64_t t = inc[p] >> 2;
            const int a = inc[p] & 3;
            const int4 v = *reinterpret_cast<const int4 *>(tets + 4 * t);
            const int b = v.x == cq ? 0 : v.y == cq ? 1 : v.z == cq ? 2 : v.w == cq ? 3 : -1;
            if (b >= 0) acc += Ke[10 * t + sym10(a, b)];
        }
        if (q < e) val[q] = acc;
    }
}

// ---------------------------------------------------------------------------
// 6. boundary faces
// ---------------------------------------------------------------------------

__device__ __forceinline__ void face_vertices(const int32_t *tets, int64_t t, int f, int32_t &a,
                                              int32_t &b, int32_t &c) {
    int32_t v[3];
    int k = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q)
        if (q != f) v[k++] = tets[4 * t + q];
    // sort three
    if (v[0] > v[1]) { int32_t x = v[0]; v[0] = v[1]; v[1] = x; }
    if (v[1] > v[2]) { int32_t x = v[1]; v[1] = v[2]; v[2] = x; }
    if (v[0] > v[1]) { int32_t x = v[0]; v[0] = v[1]; v[1] = x; }
    a = v[0];
    b = v[1];
    c = v[2];
}

__global__ void k_face_keys(const int32_t *tets, int32_t e, const int32_t *row_ptr,
                            const int32_t *col, int32_t *key, int32_t *third) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 4 * (int64_t)e) return;
    int32_t a, b, c;
    face_vertices(tets, k >> 2, (int)(k & 3), a, b, c);
    const int32_t q = find_col(col, row_ptr[a], row_ptr[a + 1], b);   // always present
    key[k] = q < 0 ? 0 : q;
    third[k] = c;
}

__device__ __forceinline__ int count_face(const int32_t *fptr, const int32_t *fitem,
                                          const int32_t *third, int32_t key, int32_t c) {
    int cnt = 0;
    for (int32_t p = fptr[key]; p < fptr[key + 1]; ++p) cnt += third[fitem[p]] == c;
    return cnt;
}

__global__ void k_face_boundary(const int32_t *tets, int32_t e, const int32_t *key,
                                const int32_t *third, const int32_t *fptr,
                                const int32_t *fitem, uint8_t *boundary) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= 4 * (int64_t)e) return;
    if (count_face(fptr, fitem, third, key[k], third[k]) == 1) {
        int32_t a, b, c;
        face_vertices(tets, k >> 2, (int)(k & 3), a, b, c);
        boundary[a] = 1;
        boundary[b] = 1;
        boundary[c] = 1;
    }
}

__global__ void k_tri_check(const int32_t *tris, int32_t nt, const int32_t *row_ptr,
                            const int32_t *col, const int32_t *fptr, const int32_t *fitem,
                            const int32_t *third, uint8_t *on_elec, int *flags) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nt) return;
    int32_t v[3] = {tris[3 * k], tris[3 * k + 1], tris[3 * k + 2]};
    if (v[0] > v[1]) { int32_t x = v[0]; v[0] = v[1]; v[1] = x; }
    if (v[1] > v[2]) { int32_t x = v[1]; v[1] = v[2]; v[2] = x; }
    if (v[0] > v[1]) { int32_t x = v[0]; v[0] = v[1]; v[1] = x; }
    const int32_t key = find_col(col, row_ptr[v[0]], row_ptr[v[0] + 1], v[1]);
    if (key < 0 || count_face(fptr, fitem, third, key, v[2]) != 1) atomicOr(flags, F_TRI_NOT_FACE);
    on_elec[v[0]] = 1;
    on_elec[v[1]] = 1;
    on_elec[v[2]] = 1;
}

__global__ void k_pick_ground(const uint8_t *boundary, const uint8_t *on_elec, int32_t n,
                              int32_t *g) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n && boundary[i] && !on_elec[i]) atomicMin(g, (int32_t)i);
}

// ---------------------------------------------------------------------------
// 7. complete electrode model
// ---------------------------------------------------------------------------

__global__ void k_tri_area(const double *nodes, const int32_t *tris, int32_t nt, double *area) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nt) return;
    const V3 x0 = load3(nodes, tris[3 * k]), x1 = load3(nodes, tris[3 * k + 1]);
    const V3 x2 = load3(nodes, tris[3 * k + 2]);
    const V3 c = cross(sub(x1, x0), sub(x2, x0));
    area[k] = 0.5 * sqrt(dot(c, c));
}

// calA_l = sum of the areas of electrode l's triangles (ascending order).
__global__ void k_contact_area(const int32_t *eptr, const int32_t *etri, const double *area,
                               int32_t L, double *calA, int *flags) {
    const int l = blockIdx.x * blockDim.x + threadIdx.x;
    if (l >= L) return;
    double s = 0.0;
    for (int32_t p = eptr[l]; p < eptr[l + 1]; ++p) s += area[etri[p]];
    if (eptr[l + 1] == eptr[l]) atomicOr(flags, F_EMPTY_ELECTRODE);
    calA[l] = s;
}

// w_F = |F| / (Z_l calA_l) per triangle.
__global__ void k_tri_weight(const double *area, const int32_t *te, const double *Z,
                             const double *calA, int32_t nt, double *w) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nt) return;
    const int l = te[k];
    w[k] = area[k] / (Z[l] * calA[l]);
}

// Surface mass (1 + delta_ij) w_F / 12 into row i, triangles in ascending order.
__global__ void k_row_cem(const int32_t *tptr, const int32_t *titem, const int32_t *tris,
                          const double *w, const int32_t *row_ptr, const int32_t *col,
                          double *val, int32_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t s = row_ptr[i], e = row_ptr[i + 1];
    for (int32_t p = tptr[i]; p < tptr[i + 1]; ++p) {
        const int64_t f = titem[p] / 3;
        const int a = titem[p] % 3;
        const double wf = w[f];
        for (int b = 0; b < 3; ++b) {
            const int32_t q = find_col(col, s, e, tris[3 * f + b]);
            if (q >= 0) val[q] += (a == b ? 2.0 : 1.0) * wf / 12.0;
        }
    }
}

// Node-major B: b_il = sum over the triangles F of e_l containing i of w_F/3.
// Pass 1 (out_col == nullptr) counts distinct electrodes, pass 2 writes them
// ascending with their weights.
constexpr int MAX_NODE_ELECTRODES = 16;

__global__ void k_brow(const int32_t *tptr, const int32_t *titem, const int32_t *te,
                       const double *w, int32_t n, int32_t *blen, const int32_t *b_ptr,
                       int32_t *out_col, int32_t *out_row, double *out_val, int *flags) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int32_t el[MAX_NODE_ELECTRODES];
    double wv[MAX_NODE_ELECTRODES];
    int cnt = 0;
    for (int32_t p = tptr[i]; p < tptr[i + 1]; ++p) {
        const int64_t f = titem[p] / 3;
        const int32_t l = te[f];
        int pos = cnt;
        while (pos > 0 && el[pos - 1] > l) --pos;
        if (pos > 0 && el[pos - 1] == l) {
            wv[pos - 1] += w[f] / 3.0;
            continue;
        }
        if (cnt == MAX_NODE_ELECTRODES) {
            atomicOr(flags, F_DEGREE);
            continue;
        }
        for (int q = cnt; q > pos; --q) {
            el[q] = el[q - 1];
            wv[q] = wv[q - 1];
        }
        el[pos] = l;
        wv[pos] = w[f] / 3.0;
        ++cnt;
    }
    if (out_col == nullptr) {
        blen[i] = cnt;
        return;
    }
    const int32_t base = b_ptr[i];
    for (int q = 0; q < cnt; ++q) {
        out_col[base + q] = el[q];
        out_row[base + q] = (int32_t)i;
        out_val[base + q] = wv[q];
    }
}

// ---------------------------------------------------------------------------
// 8. ground fix and diagonals
// ---------------------------------------------------------------------------

__global__ void k_ground_fix(int32_t g, const int32_t *row_ptr, const int32_t *col,
                             double *val) {
    const int32_t s = row_ptr[g], e = row_ptr[g + 1];
    for (int32_t q = s + threadIdx.x; q < e; q += blockDim.x) {
        const int32_t j = col[q];
        if (j == g) {
            val[q] = 1.0;
        } else {
            val[q] = 0.0;
            const int32_t r = find_col(col, row_ptr[j], row_ptr[j + 1], g);
            if (r >= 0) val[r] = 0.0;
        }
    }
}

__global__ void k_diags(const int32_t *row_ptr, const int32_t *col, const double *val, int32_t n,
                        double *diag, double *absrow) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    double d = 0.0, s = 0.0;
    for (int32_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
        if (col[q] == i) d = val[q];
        s += fabs(val[q]);
    }
    diag[i] = d;
    absrow[i] = s;
}

// Solver copy of A: off-diagonal entries with |a_ij| <= DROP sqrt(|a_ii a_jj|)
// are left out.  DROP = 64 eps is below the rounding error of the assembly
// itself (each entry is a sum of a few element contributions of size ~a_ii),
// so such entries are indistinguishable from zero: on Kuhn meshes with
// isotropic conductivity they are the couplings that vanish exactly in real
// arithmetic and come out as ~1e-17 a_ii in floating point.
constexpr double DROP = 64.0 * 2.220446049250313e-16;

__device__ __forceinline__ bool keep_entry(int64_t i, int32_t j, double v, const double *diag) {
    if (j == i) return true;
    return fabs(v) > DROP * sqrt(fabs(diag[i] * diag[j]));
}

// ---------------------------------------------------------------------------
// solver row order
// ---------------------------------------------------------------------------
// Every PCG iteration multiplies A by an n x L block whose rows are ~L*8 bytes;
// a row's product gathers the rows of its mesh neighbours.  In the order the
// caller numbers the nodes (lexicographic on a grid) neighbours lie a whole
// grid plane apart, far more rows than one XCD's L2 holds, so each row of the
// block is fetched from memory about three times per product.  The solver
// therefore renumbers the nodes: the bounding box is cut into cubic cells of
// the mesh's volume per node (so that a cell holds about one node), the cells
// into pencils of PENCIL x PENCIL cells along z, the pencils are visited in a
// snake order (and z alternates direction from pencil to pencil), and inside
// a pencil the nodes go by z, then y, then x.  Mesh neighbours are then at
// most a pencil layer (about PENCIL^2 rows) apart, except across the side
// faces of a pencil.  Nodes sharing a cell keep their relative order, so the
// permutation is deterministic.
constexpr int PENCIL = 8;

struct CellGrid {
    double lo[3], h;
    int nc[3];          // cells per axis
    int np[2];          // pencils along x and y
};

__global__ void k_bbox_part(const double *nodes, int32_t n, double *part) {
    __shared__ double s[6][256];
    double v[6] = {INFINITY, INFINITY, INFINITY, -INFINITY, -INFINITY, -INFINITY};
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        for (int k = 0; k < 3; ++k) {
            const double x = nodes[3 * i + k];
            v[k] = fmin(v[k], x);
            v[3 + k] = fmax(v[3 + k], x);
        }
    }
    for (int k = 0; k < 6; ++k) s[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            for (int k = 0; k < 3; ++k) {
                s[k][threadIdx.x] = fmin(s[k][threadIdx.x], s[k][threadIdx.x + off]);
                s[3 + k][threadIdx.x] = fmax(s[3 + k][threadIdx.x], s[3 + k][threadIdx.x + off]);
            }
        }
        __syncthreads();
    }
    if (threadIdx.x < 6) part[blockIdx.x * 6 + threadIdx.x] = s[threadIdx.x][0];
}

// Per-block sums of the tet volumes |det J| / 6 (fixed-order tree reduction).
__global__ void k_volume_part(const double *nodes, const int32_t *tets, int32_t e, double *part) {
    __shared__ double s[256];
    double v = 0.0;
    for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < e;
         t += (int64_t)gridDim.x * blockDim.x) {
        const V3 x0 = load3(nodes, tets[4 * t]), x1 = load3(nodes, tets[4 * t + 1]);
        const V3 x2 = load3(nodes, tets[4 * t + 2]), x3 = load3(nodes, tets[4 * t + 3]);
        v += fabs(dot(sub(x1, x0), cross(sub(x2, x0), sub(x3, x0)))) / 6.0;
    }
    s[threadIdx.x] = v;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) s[threadIdx.x] += s[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) part[blockIdx.x] = s[0];
}

__device__ __forceinline__ int cell_of(double x, double lo, double h, int nc) {
    const double t = (x - lo) / h;
    if (!(t > 0.0)) return 0;
    return t >= (double)(nc - 1) ? nc - 1 : (int)t;
}

__global__ void k_cell_key(const double *nodes, int32_t n, CellGrid g, int32_t *key) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int cx = cell_of(nodes[3 * i + 0], g.lo[0], g.h, g.nc[0]);
    const int cy = cell_of(nodes[3 * i + 1], g.lo[1], g.h, g.nc[1]);
    int cz = cell_of(nodes[3 * i + 2], g.lo[2], g.h, g.nc[2]);
    const int px = cx / PENCIL, py = cy / PENCIL;
    const int pid = py * g.np[0] + ((py & 1) ? g.np[0] - 1 - px : px);
    if (pid & 1) cz = g.nc[2] - 1 - cz;
    key[i] = ((pid * g.nc[2] + cz) * PENCIL + cy % PENCIL) * PENCIL + cx % PENCIL;
}

__global__ void k_inverse_perm(const int32_t *perm, int32_t n, int32_t *iperm) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r < n) iperm[perm[r]] = (int32_t)r;
}

// Cell grid for n nodes in the box [lo, hi] of a mesh of volume vol: cells of
// the volume per node (of the box's, where vol is not positive), enlarged
// where the key space would exceed 4 n + 4096 buckets (flat or strongly
// graded meshes).
CellGrid make_cell_grid(const double lo[3], const double hi[3], int32_t n, double vol_mesh,
                        int64_t *buckets) {
    CellGrid g{};
    double ext[3], emax = 0.0;
    for (int k = 0; k < 3; ++k) {
        g.lo[k] = lo[k];
        ext[k] = hi[k] > lo[k] ? hi[k] - lo[k] : 0.0;
        emax = std::max(emax, ext[k]);
    }
    const double floor_ext = emax > 0.0 ? 1e-6 * emax : 1.0;
    double vol = 1.0;
    for (int k = 0; k < 3; ++k) vol *= std::max(ext[k], floor_ext);
    if (vol_mesh > 0.0 && std::isfinite(vol_mesh) && vol_mesh < vol) vol = vol_mesh;
    g.h = std::cbrt(vol / std::max(n, 1));
    if (!(g.h > 0.0) || !std::isfinite(g.h)) g.h = 1.0;
    const int64_t cap = 4 * (int64_t)n + 4096;
    for (;;) {
        int64_t nc[3];
        for (int k = 0; k < 3; ++k)
            nc[k] = std::max<int64_t>(1, (int64_t)std::ceil(ext[k] / g.h));
        const int64_t npx = (nc[0] + PENCIL - 1) / PENCIL, npy = (nc[1] + PENCIL - 1) / PENCIL;
        const int64_t total = npx * npy * nc[2] * PENCIL * PENCIL;
        if (total <= cap) {
            for (int k = 0; k < 3; ++k) g.nc[k] = (int)nc[k];
            g.np[0] = (int)npx;
            g.np[1] = (int)npy;
            *buckets = total;
            return g;
        }
        g.h *= 1.26;
    }
}

// Solver copy of row perm[r], renumbered through iperm, columns ascending.
__global__ void k_nz_count(const int32_t *row_ptr, const int32_t *col, const double *val,
                           const double *diag, const int32_t *perm, int32_t n, int32_t *len) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int32_t i = perm[r];
    int cnt = 0;
    for (int32_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) cnt += keep_entry(i, col[q], val[q], diag);
    len[r] = cnt;
}

__global__ void k_nz_fill(const int32_t *row_ptr, const int32_t *col, const double *val,
                          const double *diag, const int32_t *perm, const int32_t *iperm,
                          int32_t n, const int32_t *sp_ptr, int32_t *sp_col, double *sp_val) {
    const int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n) return;
    const int32_t i = perm[r];
    const int32_t s = sp_ptr[r];
    int32_t o = s;
    for (int32_t q = row_ptr[i]; q < row_ptr[i + 1]; ++q) {
        if (!keep_entry(i, col[q], val[q], diag)) continue;
        const int32_t c = iperm[col[q]];
        const double v = val[q];
        int32_t j = o - 1;
        while (j >= s && sp_col[j] > c) {
            sp_col[j + 1] = sp_col[j];
            sp_val[j + 1] = sp_val[j];
            --j;
        }
        sp_col[j + 1] = c;
        sp_val[j + 1] = v;
        ++o;
    }
}

// ---------------------------------------------------------------------------
// point-dipole source matrix
// ---------------------------------------------------------------------------

__global__ void k_validate_dipoles(const int32_t *dt, int32_t m, int32_t e, int *flags) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j < m && (dt[j] < 0 || dt[j] >= e)) atomicOr(flags, F_DIPOLE_INDEX);
}

__global__ void k_point_dipoles(const double *nodes, const int32_t *tets, const int32_t *dt,
                                int32_t m, int32_t *cp, int32_t *ri, double *gv) {
    const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= m) return;
    const int64_t t = dt[j];
    V3 g[4];
    bool degenerate;
    tet_gradients(nodes, tets, t, g, &degenerate);
    int ord[4] = {0, 1, 2, 3};
    for (int a = 1; a < 4; ++a) {
        int x = ord[a], b = a - 1;
        while (b >= 0 && tets[4 * t + ord[b]] > tets[4 * t + x]) {
            ord[b + 1] = ord[b];
            --b;
        }
        ord[b + 1] = x;
    }
    for (int k = 0; k < 3; ++k) {
        const int64_t c = 3 * j + k;
        cp[c] = (int32_t)(4 * c);
        for (int a = 0; a < 4; ++a) {
            const V3 ga = g[ord[a]];
            ri[4 * c + a] = tets[4 * t + ord[a]];
            gv[4 * c + a] = -(k == 0 ? ga.x : (k == 1 ? ga.y : ga.z));
        }
    }
    if (j == m - 1) cp[3 * m] = (int32_t)(12 * m);
}

// Source matrix of the linearized EIT lead field (App. A.3): column
// p * ne + j holds K1_m U[:, p] on the vertices of tet m = elems[j] (ascending
// rows), K1_m the unit-conductivity element matrix, U = T M^-1 I (n x P).
__global__ void k_eit_columns(const double *nodes, const int32_t *tets, const int32_t *elems,
                              int32_t ne, int32_t P, const double *U, int32_t *cp, int32_t *ri,
                              double *gv) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (int64_t)ne * P) return;
    const int p = (int)(idx / ne);
    const int64_t j = idx - (int64_t)p * ne;
    const int64_t m = elems ? elems[j] : j;
    V3 g[4];
    bool degenerate;
    const double det = tet_gradients(nodes, tets, m, g, &degenerate);
    const double vol = fabs(det) / 6.0;
    double u[4], w[4];
    for (int a = 0; a < 4; ++a) u[a] = U[(size_t)tets[4 * m + a] * P + p];
    for (int a = 0; a < 4; ++a) {
        double acc = 0.0;
        for (int b = 0; b < 4; ++b) acc += vol * dot(g[a], g[b]) * u[b];
        w[a] = acc;
    }
    int ord[4] = {0, 1, 2, 3};
    for (int a = 1; a < 4; ++a) {
        int x = ord[a], b = a - 1;
        while (b >= 0 && tets[4 * m + ord[b]] > tets[4 * m + x]) {
            ord[b + 1] = ord[b];
            --b;
        }
        ord[b + 1] = x;
    }
    cp[idx] = (int32_t)(4 * idx);
    for (int a = 0; a < 4; ++a) {
        ri[4 * idx + a] = tets[4 * m + ord[a]];
        gv[4 * idx + a] = w[ord[a]];
    }
    if (idx == (int64_t)ne * P - 1) cp[(int64_t)ne * P] = (int32_t)(4 * (int64_t)ne * P);
}

// ---------------------------------------------------------------------------
// host orchestration
// ---------------------------------------------------------------------------

zi_status read_flags(const int *dflags, hipStream_t s, int *hflags) {
    ZI_HIP(hipMemcpyAsync(hflags, dflags, sizeof(int), hipMemcpyDeviceToHost, s));
    ZI_HIP(hipStreamSynchronize(s));
    return ZI_OK;
}

zi_status flags_status(int f) {
    if (!f) return ZI_OK;
    const char *what = (f & F_TET_INDEX)       ? "tetrahedron vertex index out of range or repeated"
                       : (f & F_SIGMA)         ? "conductivity not positive (definite) or not finite"
                       : (f & F_COORD)         ? "non-finite node coordinate"
                       : (f & F_DEGENERATE)    ? "degenerate tetrahedron"
                       : (f & F_TRI_INDEX)     ? "electrode triangle index out of range or repeated"
                       : (f & F_TRI_ELECTRODE) ? "tri_electrode out of range"
                       : (f & F_TRI_NOT_FACE)  ? "electrode triangle is not a boundary face"
                       : (f & F_DEGREE)        ? "node degree exceeds the supported maximum"
                       : (f & F_EMPTY_ELECTRODE) ? "an electrode has no triangle"
                                                 : "invalid input";
    set_error("%s (flags 0x%x)", what, f);
    return ZI_EMESH;
}

}  // namespace

zi_status zi_assemble_impl(const zi_mesh *mesh, const zi_electrodes *el, int32_t ground,
                           hipStream_t s, zi_system **out) {
    const int32_t n = mesh->n_nodes, e = mesh->n_tets, L = el->n_electrodes,
                  nt = el->n_tris;
    const int ncomp = mesh->sigma_ncomp;
    for (int l = 0; l < L; ++l) {
        if (!(el->Z[l] > 0.0) || !std::isfinite(el->Z[l])) {
            set_error("contact impedance Z[%d] must be positive and finite", l);
            return ZI_EMESH;
        }
    }
    Pool tmp;
    int *flags = nullptr;
    ZI_TRY(tmp.alloc(&flags, 1));
    ZI_TRY(fill_i32(flags, 0, 1, s));
    int hflags = 0;

    // 1. validation of everything later kernels index with
    hipLaunchKernelGGL(k_validate_tets, dim3(grid_for(e, 256)), dim3(256), 0, s, mesh->tets,
                       mesh->sigma, ncomp, e, n, flags);
    hipLaunchKernelGGL(k_validate_nodes, dim3(grid_for(n, 256)), dim3(256), 0, s, mesh->nodes,
                       n, flags);
    if (nt > 0)
        hipLaunchKernelGGL(k_validate_tris, dim3(grid_for(nt, 256)), dim3(256), 0, s, el->tris,
                           el->tri_electrode, nt, n, L, flags);
    ZI_HIP(hipGetLastError());
    ZI_TRY(read_flags(flags, s, &hflags));
    ZI_TRY(flags_status(hflags));

    zi_system *sys = new zi_system();
    sys->pool.cached = true;
    sys->n = n;
    sys->e = e;
    sys->L = L;
    sys->ntris = nt;
    sys->ncomp = ncomp;
    (void)hipGetDevice(&sys->device);
    struct Guard {
        zi_system *p;
        ~Guard() {
            if (p) delete p;
        }
    } guard{sys};
    Pool &P = sys->pool;

    ZI_TRY(P.alloc(&sys->nodes, (size_t)n * 3));
    ZI_TRY(P.alloc(&sys->tets, (size_t)e * 4));
    ZI_TRY(P.alloc(&sys->sigma, (size_t)e * ncomp));
    ZI_HIP(hipMemcpyAsync(sys->nodes, mesh->nodes, sizeof(double) * n * 3,
                          hipMemcpyDeviceToDevice, s));
    ZI_HIP(hipMemcpyAsync(sys->tets, mesh->tets, sizeof(int32_t) * e * 4,
                          hipMemcpyDeviceToDevice, s));
    ZI_HIP(hipMemcpyAsync(sys->sigma, mesh->sigma, sizeof(double) * e * ncomp,
                          hipMemcpyDeviceToDevice, s));

    // 2. element matrices
    double *Ke = nullptr;
    ZI_TRY(tmp.alloc(&Ke, (size_t)e * 10));
    hipLaunchKernelGGL(k_element, dim3(grid_for(e, 256)), dim3(256), 0, s, sys->nodes, sys->tets,
                       sys->sigma, ncomp, e, Ke, flags);
    ZI_HIP(hipGetLastError());

    // 3. node -> tet incidence (item = 4 t + local vertex), ascending
    int32_t *inc_ptr = nullptr, *inc = nullptr;
    ZI_TRY(tmp.alloc(&inc_ptr, (size_t)n + 1));
    ZI_TRY(tmp.alloc(&inc, (size_t)e * 4));
    ZI_TRY(bucketize(sys->tets, 4 * e, n, inc_ptr, inc, true, tmp, s));

    // 4. CSR structure
    int32_t *rowlen = nullptr;
    ZI_TRY(tmp.alloc(&rowlen, (size_t)n));
    ZI_TRY(P.alloc(&sys->row_ptr, (size_t)n + 1));
    hipLaunchKernelGGL(k_row_struct, dim3(grid_for(n, ROW_THREADS)), dim3(ROW_THREADS), 0, s,
                       inc_ptr, inc, sys->tets, n, rowlen, (const int32_t *)nullptr,
                       (int32_t *)nullptr, flags);
    ZI_HIP(hipGetLastError());
    ZI_TRY(scan_exclusive(rowlen, sys->row_ptr, n, tmp, s));
    int32_t nnz = 0;
    ZI_HIP(hipMemcpyAsync(&nnz, sys->row_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    ZI_TRY(read_flags(flags, s, &hflags));
    ZI_TRY(flags_status(hflags));
    sys->nnz = nnz;
    ZI_TRY(P.alloc(&sys->col, (size_t)nnz));
    ZI_TRY(P.alloc(&sys->val, (size_t)nnz));
    hipLaunchKernelGGL(k_row_struct, dim3(grid_for(n, ROW_THREADS)), dim3(ROW_THREADS), 0, s,
                       inc_ptr, inc, sys->tets, n, rowlen, sys->row_ptr, sys->col, flags);
    ZI_HIP(hipGetLastError());

    // 5. stiffness values
    hipLaunchKernelGGL(k_row_values, dim3(grid_for((size_t)n * RV, 256)), dim3(256), 0, s,
                       inc_ptr, inc, sys->tets, Ke, sys->row_ptr, sys->col, sys->val, n);
    ZI_HIP(hipGetLastError());

    // 6. boundary faces, electrode triangles on faces
    int32_t *fkey = nullptr, *fthird = nullptr, *fptr = nullptr, *fitem = nullptr;
    ZI_TRY(tmp.alloc(&fkey, (size_t)e * 4));
    ZI_TRY(tmp.alloc(&fthird, (size_t)e * 4));
    ZI_TRY(tmp.alloc(&fptr, (size_t)nnz + 1));
    ZI_TRY(tmp.alloc(&fitem, (size_t)e * 4));
    hipLaunchKernelGGL(k_face_keys, dim3(grid_for((size_t)4 * e, 256)), dim3(256), 0, s,
                       sys->tets, e, sys->row_ptr, sys->col, fkey, fthird);
    ZI_HIP(hipGetLastError());
    ZI_TRY(bucketize(fkey, 4 * e, nnz, fptr, fitem, false, tmp, s));
    ZI_TRY(P.alloc(&sys->boundary, (size_t)n));
    uint8_t *on_elec = nullptr;
    ZI_TRY(tmp.alloc(&on_elec, (size_t)n));
    ZI_HIP(hipMemsetAsync(sys->boundary, 0, n, s));
    ZI_HIP(hipMemsetAsync(on_elec, 0, n, s));
    hipLaunchKernelGGL(k_face_boundary, dim3(grid_for((size_t)4 * e, 256)), dim3(256), 0, s,
                       sys->tets, e, fkey, fthird, fptr, fitem, sys->boundary);
    if (nt > 0)
        hipLaunchKernelGGL(k_tri_check, dim3(grid_for(nt, 256)), dim3(256), 0, s, el->tris, nt,
                           sys->row_ptr, sys->col, fptr, fitem, fthird, on_elec, flags);
    ZI_HIP(hipGetLastError());

    // 7. CEM
    int32_t *tris = nullptr, *te = nullptr;
    double *area = nullptr, *w = nullptr, *Zd = nullptr;
    ZI_TRY(tmp.alloc(&tris, (size_t)nt * 3));
    ZI_TRY(tmp.alloc(&te, (size_t)nt));
    ZI_TRY(tmp.alloc(&area, (size_t)nt));
    ZI_TRY(tmp.alloc(&w, (size_t)nt));
    ZI_TRY(tmp.alloc(&Zd, (size_t)L));
    ZI_TRY(P.alloc(&sys->calA, (size_t)L));
    ZI_TRY(P.alloc(&sys->C, (size_t)L));
    if (nt > 0) {
        ZI_HIP(hipMemcpyAsync(tris, el->tris, sizeof(int32_t) * 3 * nt, hipMemcpyDeviceToDevice, s));
        ZI_HIP(hipMemcpyAsync(te, el->tri_electrode, sizeof(int32_t) * nt, hipMemcpyDeviceToDevice, s));
    }
    std::vector<double> Cz(L);
    for (int l = 0; l < L; ++l) Cz[l] = 1.0 / el->Z[l];
    ZI_HIP(hipMemcpyAsync(Zd, el->Z, sizeof(double) * L, hipMemcpyHostToDevice, s));
    ZI_HIP(hipMemcpyAsync(sys->C, Cz.data(), sizeof(double) * L, hipMemcpyHostToDevice, s));
    int32_t *eptr = nullptr, *etri = nullptr;
    ZI_TRY(tmp.alloc(&eptr, (size_t)L + 1));
    ZI_TRY(tmp.alloc(&etri, (size_t)nt));
    ZI_TRY(bucketize(te, nt, L, eptr, etri, true, tmp, s));
    if (nt > 0)
        hipLaunchKernelGGL(k_tri_area, dim3(grid_for(nt, 256)), dim3(256), 0, s, sys->nodes, tris,
                           nt, area);
    hipLaunchKernelGGL(k_contact_area, dim3(grid_for(L, 64)), dim3(64), 0, s, eptr, etri, area, L,
                       sys->calA, flags);
    if (nt > 0)
        hipLaunchKernelGGL(k_tri_weight, dim3(grid_for(nt, 256)), dim3(256), 0, s, area, te, Zd,
                           sys->calA, nt, w);
    ZI_HIP(hipGetLastError());
    ZI_TRY(read_flags(flags, s, &hflags));   // also checks the face test
    ZI_TRY(flags_status(hflags));

    int32_t *tptr = nullptr, *titem = nullptr;
    ZI_TRY(tmp.alloc(&tptr, (size_t)n + 1));
    ZI_TRY(tmp.alloc(&titem, (size_t)nt * 3));
    ZI_TRY(bucketize(tris, 3 * nt, n, tptr, titem, true, tmp, s));
    hipLaunchKernelGGL(k_row_cem, dim3(grid_for(n, 128)), dim3(128), 0, s, tptr, titem, tris, w,
                       sys->row_ptr, sys->col, sys->val, n);
    int32_t *blen = nullptr;
    ZI_TRY(tmp.alloc(&blen, (size_t)n));
    ZI_TRY(P.alloc(&sys->b_ptr, (size_t)n + 1));
    hipLaunchKernelGGL(k_brow, dim3(grid_for(n, 128)), dim3(128), 0, s, tptr, titem, te, w, n,
                       blen, (const int32_t *)nullptr, (int32_t *)nullptr, (int32_t *)nullptr,
                       (double *)nullptr, flags);
    ZI_HIP(hipGetLastError());
    ZI_TRY(scan_exclusive(blen, sys->b_ptr, n, tmp, s));
    int32_t bnnz = 0;
    ZI_HIP(hipMemcpyAsync(&bnnz, sys->b_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    ZI_HIP(hipStreamSynchronize(s));
    sys->b_nnz = bnnz;
    ZI_TRY(P.alloc(&sys->b_col, (size_t)bnnz));
    ZI_TRY(P.alloc(&sys->b_row, (size_t)bnnz));
    ZI_TRY(P.alloc(&sys->b_val, (size_t)bnnz));
    hipLaunchKernelGGL(k_brow, dim3(grid_for(n, 128)), dim3(128), 0, s, tptr, titem, te, w, n,
                       blen, sys->b_ptr, sys->b_col, sys->b_row, sys->b_val, flags);
    ZI_HIP(hipGetLastError());
    ZI_TRY(P.alloc(&sys->e_ptr, (size_t)L + 1));
    ZI_TRY(P.alloc(&sys->e_item, (size_t)bnnz));
    ZI_TRY(bucketize(sys->b_col, bnnz, L, sys->e_ptr, sys->e_item, true, tmp, s));

    // 8. ground node and fix
    int32_t *dg = nullptr;
    ZI_TRY(tmp.alloc(&dg, 1));
    ZI_TRY(fill_i32(dg, INT_MAX, 1, s));
    hipLaunchKernelGGL(k_pick_ground, dim3(grid_for(n, 256)), dim3(256), 0, s, sys->boundary,
                       on_elec, n, dg);
    ZI_HIP(hipGetLastError());
    int32_t gmin = INT_MAX;
    ZI_HIP(hipMemcpyAsync(&gmin, dg, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    ZI_TRY(read_flags(flags, s, &hflags));
    ZI_TRY(flags_status(hflags));
    if (ground < 0) {
        if (gmin == INT_MAX) {
            set_error("no boundary node outside the electrodes to ground");
            return ZI_EMESH;
        }
        sys->ground = gmin;
    } else {
        uint8_t hb = 0, he = 1;
        ZI_HIP(hipMemcpyAsync(&hb, sys->boundary + ground, 1, hipMemcpyDeviceToHost, s));
        ZI_HIP(hipMemcpyAsync(&he, on_elec + ground, 1, hipMemcpyDeviceToHost, s));
        ZI_HIP(hipStreamSynchronize(s));
        if (!hb || he) {
            set_error("ground node %d is not a boundary node outside the electrodes", ground);
            return ZI_EINVAL;
        }
        sys->ground = ground;
    }
    hipLaunchKernelGGL(k_ground_fix, dim3(1), dim3(64), 0, s, sys->ground, sys->row_ptr,
                       sys->col, sys->val);
    ZI_TRY(P.alloc(&sys->diag, (size_t)n));
    ZI_TRY(P.alloc(&sys->absrow, (size_t)n));
    hipLaunchKernelGGL(k_diags, dim3(grid_for(n, 256)), dim3(256), 0, s, sys->row_ptr, sys->col,
                       sys->val, n, sys->diag, sys->absrow);
    ZI_HIP(hipGetLastError());
    {   // solver row order
        constexpr int NBB = 256;
        double *bb = nullptr;
        ZI_TRY(tmp.alloc(&bb, (size_t)NBB * 6));
        double *vb = nullptr;
        ZI_TRY(tmp.alloc(&vb, (size_t)NBB));
        hipLaunchKernelGGL(k_bbox_part, dim3(NBB), dim3(256), 0, s, sys->nodes, n, bb);
        hipLaunchKernelGGL(k_volume_part, dim3(NBB), dim3(256), 0, s, sys->nodes, sys->tets, e,
                           vb);
        ZI_HIP(hipGetLastError());
        std::vector<double> hb((size_t)NBB * 6), hv((size_t)NBB);
        ZI_HIP(hipMemcpyAsync(hb.data(), bb, sizeof(double) * NBB * 6, hipMemcpyDeviceToHost, s));
        ZI_HIP(hipMemcpyAsync(hv.data(), vb, sizeof(double) * NBB, hipMemcpyDeviceToHost, s));
        ZI_HIP(hipStreamSynchronize(s));
        double vol_mesh = 0.0;
        for (int b = 0; b < NBB; ++b) vol_mesh += hv[b];
        double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
        for (int b = 0; b < NBB; ++b)
            for (int k = 0; k < 3; ++k) {
                lo[k] = std::min(lo[k], hb[b * 6 + k]);
                hi[k] = std::max(hi[k], hb[b * 6 + 3 + k]);
            }
        int64_t nbk = 0;
        const CellGrid cg = make_cell_grid(lo, hi, n, vol_mesh, &nbk);
        int32_t *key = nullptr, *kptr = nullptr;
        ZI_TRY(tmp.alloc(&key, (size_t)n));
        ZI_TRY(tmp.alloc(&kptr, (size_t)nbk + 1));
        ZI_TRY(P.alloc(&sys->perm, (size_t)n));
        ZI_TRY(P.alloc(&sys->iperm, (size_t)n));
        hipLaunchKernelGGL(k_cell_key, dim3(grid_for(n, 256)), dim3(256), 0, s, sys->nodes, n, cg,
                           key);
        ZI_HIP(hipGetLastError());
        ZI_TRY(bucketize(key, n, (int32_t)nbk, kptr, sys->perm, true, tmp, s));
        hipLaunchKernelGGL(k_inverse_perm, dim3(grid_for(n, 256)), dim3(256), 0, s, sys->perm, n,
                           sys->iperm);
        ZI_HIP(hipGetLastError());
    }
    int32_t *splen = nullptr;
    ZI_TRY(tmp.alloc(&splen, (size_t)n));
    ZI_TRY(P.alloc(&sys->sp_ptr, (size_t)n + 1));
    hipLaunchKernelGGL(k_nz_count, dim3(grid_for(n, 256)), dim3(256), 0, s, sys->row_ptr, sys->col,
                       sys->val, sys->diag, sys->perm, n, splen);
    ZI_HIP(hipGetLastError());
    ZI_TRY(scan_exclusive(splen, sys->sp_ptr, n, tmp, s));
    int32_t spnnz = 0;
    ZI_HIP(hipMemcpyAsync(&spnnz, sys->sp_ptr + n, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    ZI_HIP(hipStreamSynchronize(s));
    sys->sp_nnz = spnnz;
    ZI_TRY(P.alloc(&sys->sp_col, (size_t)spnnz));
    ZI_TRY(P.alloc(&sys->sp_val, (size_t)spnnz));
    hipLaunchKernelGGL(k_nz_fill, dim3(grid_for(n, 256)), dim3(256), 0, s, sys->row_ptr, sys->col,
                       sys->val, sys->diag, sys->perm, sys->iperm, n, sys->sp_ptr, sys->sp_col,
                       sys->sp_val);
    ZI_HIP(hipGetLastError());
    ZI_HIP(hipStreamSynchronize(s));
    tmp.release();
    guard.p = nullptr;
    *out = sys;
    return ZI_OK;
}

zi_status zi_point_dipoles_impl(const zi_system *sys, int32_t m, const int32_t *dt, int32_t *cp,
                                int32_t *ri, double *gv, hipStream_t s) {
    Pool tmp;
    int *flags = nullptr;
    ZI_TRY(tmp.alloc(&flags, 1));
    ZI_TRY(fill_i32(flags, 0, 1, s));
    if (m > 0) {
        hipLaunchKernelGGL(k_validate_dipoles, dim3(grid_for(m, 256)), dim3(256), 0, s, dt, m,
                           sys->e, flags);
        ZI_HIP(hipGetLastError());
    }
    int hflags = 0;
    ZI_TRY(read_flags(flags, s, &hflags));
    if (hflags) {
        set_error("dipole tetrahedron index out of range");
        return ZI_EINVAL;
    }
    if (m == 0) return fill_i32(cp, 0, 1, s);
    hipLaunchKernelGGL(k_point_dipoles, dim3(grid_for(m, 128)), dim3(128), 0, s, sys->nodes,
                       sys->tets, dt, m, cp, ri, gv);
    ZI_HIP(hipGetLastError());
    ZI_HIP(hipStreamSynchronize(s));
    return ZI_OK;
}

zi_status zi_eit_columns_impl(const zi_system *sys, const double *U, int32_t P, int32_t ne,
                              const int32_t *elems, int32_t *cp, int32_t *ri, double *gv,
                              hipStream_t s) {
    if (elems) {
        Pool tmp;
        int *flags = nullptr;
        ZI_TRY(tmp.alloc(&flags, 1));
        ZI_TRY(fill_i32(flags, 0, 1, s));
        hipLaunchKernelGGL(k_validate_dipoles, dim3(grid_for(ne, 256)), dim3(256), 0, s, elems,
                           ne, sys->e, flags);
        ZI_HIP(hipGetLastError());
        int hflags = 0;
        ZI_TRY(read_flags(flags, s, &hflags));
        if (hflags) {
            set_error("element index out of range");
            return ZI_EINVAL;
        }
    }
    const size_t cols = (size_t)ne * P;
    hipLaunchKernelGGL(k_eit_columns, dim3(grid_for(cols, 128)), dim3(128), 0, s, sys->nodes,
                       sys->tets, elems, ne, P, U, cp, ri, gv);
    ZI_HIP(hipGetLastError());
    return ZI_OK;
}
