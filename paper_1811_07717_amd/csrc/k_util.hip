// Device utilities: exclusive scan, bucketing (counting sort), fills, the
// device block cache.
#include <map>
#include <mutex>

#include "zi_internal.h"

namespace zi {
namespace {

constexpr int SCAN_THREADS = 256;
constexpr int SCAN_ITEMS = 8;
constexpr int SCAN_TILE = SCAN_THREADS * SCAN_ITEMS;

// Block-local exclusive scan of one tile; writes the tile total to bsum.
__global__ __launch_bounds__(SCAN_THREADS) void k_scan_tile(const int32_t *in, int32_t *out,
                                                            int32_t *bsum, int32_t count) {
    __shared__ int32_t s[SCAN_THREADS];
    const int tid = threadIdx.x;
    const int64_t base = (int64_t)blockIdx.x * SCAN_TILE + (int64_t)tid * SCAN_ITEMS;
    int32_t v[SCAN_ITEMS];
    int32_t sum = 0;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t idx = base + k;
        v[k] = idx < count ? in[idx] : 0;
        sum += v[k];
    }
    s[tid] = sum;
    __syncthreads();
    for (int off = 1; off < SCAN_THREADS; off <<= 1) {
        int32_t t = tid >= off ? s[tid - off] : 0;
        __syncthreads();
        s[tid] += t;
        __syncthreads();
    }
    int32_t run = s[tid] - sum;
#pragma unroll
    for (int k = 0; k < SCAN_ITEMS; ++k) {
        const int64_t idx = base + k;
        if (idx < count) out[idx] = run;
        run += v[k];
    }
    if (tid == SCAN_THREADS - 1) bsum[blockIdx.x] = s[tid];
}

__global__ void k_scan_add(int32_t *out, const int32_t *boff, int32_t count) {
    const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx < count) out[idx] += boff[idx / SCAN_TILE];
}

__global__ void k_copy1(const int32_t *src, int32_t *dst) { *dst = *src; }

__global__ void k_count(const int32_t *keys, int32_t n, int32_t *cnt) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) atomicAdd(&cnt[keys[k]], 1);
}

__global__ void k_place(const int32_t *keys, int32_t n, const int32_t *ptr, int32_t *cursor,
                        int32_t *items) {
    const int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k < n) {
        const int32_t b = keys[k];
        const int32_t pos = atomicAdd(&cursor[b], 1);
        items[ptr[b] + pos] = (int32_t)k;
    }
}

// Insertion sort of every bucket (buckets are short).
__global__ void k_sort_buckets(const int32_t *ptr, int32_t *items, int32_t nb) {
    const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (b >= nb) return;
    const int32_t s = ptr[b], e = ptr[b + 1];
    for (int32_t i = s + 1; i < e; ++i) {
        const int32_t x = items[i];
        int32_t j = i - 1;
        while (j >= s && items[j] > x) {
            items[j + 1] = items[j];
            --j;
        }
        items[j + 1] = x;
    }
}

__global__ void k_fill_i32(int32_t *p, int32_t v, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_f64(double *p, double v, size_t n) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_copy_cols(const double *src, int32_t lds, double *dst, int32_t ldd,
                            int32_t rows, int32_t cols) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)rows * cols) return;
    const size_t r = i / cols, c = i % cols;
    dst[r * ldd + c] = src[r * lds + c];
}

__global__ void k_gather_rows(const double *src, int32_t lds, const int32_t *rows, double *dst,
                              int32_t ldd, int32_t n, int32_t cols) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= (size_t)n * cols) return;
    const size_t r = i / cols, c = i % cols;
    dst[r * ldd + c] = src[(size_t)rows[r] * lds + c];
}

// Plain streaming copy with the 16-byte accesses of the solver kernels, one
// pair per thread (the shape that reaches the highest copy rate on gfx950).
__global__ void k_copy2(const double2 *src, double2 *dst, size_t n2) {
    const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n2) dst[i] = src[i];
}

inline unsigned grid_for(size_t n, int threads) {
    return (unsigned)((n + threads - 1) / threads);
}

zi_status scan_rec(const int32_t *in, int32_t *out, int32_t count, int32_t *total, Pool &pool,
                   hipStream_t s) {
    const int32_t nb = (count + SCAN_TILE - 1) / SCAN_TILE;
    int32_t *bsum = nullptr;
    ZI_TRY(pool.alloc(&bsum, (size_t)nb + 1));
    hipLaunchKernelGGL(k_scan_tile, dim3(nb), dim3(SCAN_THREADS), 0, s, in, out, bsum, count);
    ZI_HIP(hipGetLastError());
    if (nb == 1) {
        hipLaunchKernelGGL(k_copy1, dim3(1), dim3(1), 0, s, bsum, total);
        ZI_HIP(hipGetLastError());
        return ZI_OK;
    }
    int32_t *boff = nullptr;
    ZI_TRY(pool.alloc(&boff, (size_t)nb + 1));
    ZI_TRY(scan_rec(bsum, boff, nb, total, pool, s));
    hipLaunchKernelGGL(k_scan_add, dim3(grid_for(count, 256)), dim3(256), 0, s, out, boff,
                       count);
    ZI_HIP(hipGetLastError());
    return ZI_OK;
}

}  // namespace

namespace {
std::mutex g_cache_mu;
std::multimap<std::pair<int, size_t>, void *> g_cache;   // (device, bytes) -> block
size_t g_cached = 0;
size_t g_cache_cap = 0;   // set on first use: a quarter of the device's memory
}  // namespace

size_t cache_round(size_t bytes) {
    const size_t g = bytes >= (size_t(1) << 20) ? (size_t(2) << 20) : 512;
    return (bytes + g - 1) / g * g;
}

void *cache_take(size_t bytes, int dev) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    auto it = g_cache.find({dev, bytes});
    if (it == g_cache.end()) return nullptr;
    void *p = it->second;
    g_cache.erase(it);
    g_cached -= bytes;
    return p;
}

bool cache_put(void *p, size_t bytes, int dev) {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    if (g_cache_cap == 0) {
        size_t fr = 0, tot = 0;
        if (hipMemGetInfo(&fr, &tot) != hipSuccess) return false;
        g_cache_cap = tot / 4;
    }
    if (g_cached + bytes > g_cache_cap) return false;
    g_cache.emplace(std::make_pair(dev, bytes), p);
    g_cached += bytes;
    return true;
}

zi_status cache_clear() {
    std::lock_guard<std::mutex> lk(g_cache_mu);
    for (auto &kv : g_cache) (void)hipFree(kv.second);
    g_cache.clear();
    g_cached = 0;
    return ZI_OK;
}

zi_status scan_exclusive(const int32_t *in, int32_t *out, int32_t count, Pool &pool,
                         hipStream_t s) {
    if (count == 0) return fill_i32(out, 0, 1, s);
    return scan_rec(in, out, count, out + count, pool, s);
}

zi_status bucketize(const int32_t *keys, int32_t n_items, int32_t n_buckets, int32_t *ptr,
                    int32_t *items, bool sort, Pool &pool, hipStream_t s) {
    int32_t *cnt = nullptr, *cursor = nullptr;
    ZI_TRY(pool.alloc(&cnt, (size_t)n_buckets));
    ZI_TRY(pool.alloc(&cursor, (size_t)n_buckets));
    ZI_TRY(fill_i32(cnt, 0, n_buckets, s));
    ZI_TRY(fill_i32(cursor, 0, n_buckets, s));
    if (n_items > 0) {
        hipLaunchKernelGGL(k_count, dim3(grid_for(n_items, 256)), dim3(256), 0, s, keys,
                           n_items, cnt);
        ZI_HIP(hipGetLastError());
    }
    ZI_TRY(scan_exclusive(cnt, ptr, n_buckets, pool, s));
    if (n_items > 0) {
        hipLaunchKernelGGL(k_place, dim3(grid_for(n_items, 256)), dim3(256), 0, s, keys,
                           n_items, ptr, cursor, items);
        ZI_HIP(hipGetLastError());
        if (sort) {
            hipLaunchKernelGGL(k_sort_buckets, dim3(grid_for(n_buckets, 128)), dim3(128), 0, s,
                               ptr, items, n_buckets);
            ZI_HIP(hipGetLastError());
        }
    }
    return ZI_OK;
}

zi_status fill_i32(int32_t *p, int32_t value, size_t count, hipStream_t s) {
    if (count == 0) return ZI_OK;
    hipLaunchKernelGGL(k_fill_i32, dim3(grid_for(count, 256)), dim3(256), 0, s, p, value,
                       count);
    ZI_HIP(hipGetLastError());
    return ZI_OK;
}

zi_status fill_f64(double *p, double value, size_t count, hipStream_t s) {
    if (count == 0) return ZI_OK;
    hipLaunchKernelGGL(k_fill_f64, dim3(grid_for(count, 256)), dim3(256), 0, s, p, value,
                       count);
    ZI_HIP(hipGetLastError());
    return ZI_OK;
}

zi_status copy_probe(const double *src, double *dst, size_t n, double *ms, hipStream_t s) {
    hipEvent_t e0, e1;
    ZI_HIP(hipEventCreate(&e0));
    ZI_HIP(hipEventCreate(&e1));
    ZI_HIP(hipEventRecord(e0, s));
    if (n / 2 > 0)
        hipLaunchKernelGGL(k_copy2, dim3(grid_for(n / 2, 256)), dim3(256), 0, s,
                           reinterpret_cast<const double2 *>(src), reinterpret_cast<double2 *>(dst),
                           n / 2);
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

zi_status copy_cols(const double *src, int32_t lds, double *dst, int32_t ldd, int32_t rows,
                    int32_t cols, hipStream_t s) {
    const size_t total = (size_t)rows * cols;
    if (total == 0) return ZI_OK;
    hipLaunchKernelGGL(k_copy_cols, dim3(grid_for(total, 256)), dim3(256), 0, s, src, lds, dst,
                       ldd, rows, cols);
    ZI_HIP(hipGetLastError());
    return ZI_OK;
}

zi_status gather_rows(const double *src, int32_t lds, const int32_t *rows, double *dst,
                      int32_t ldd, int32_t n, int32_t cols, hipStream_t s) {
    const size_t total = (size_t)n * cols;
    if (total == 0) return ZI_OK;
    hipLaunchKernelGGL(k_gather_rows, dim3(grid_for(total, 256)), dim3(256), 0, s, src, lds, rows,
                       dst, ldd, n, cols);
    ZI_HIP(hipGetLastError());
    return ZI_OK;
}

}  // namespace zi
