// Error state, device allocation and the exclusive scan used by setup.
#include <cstdarg>
#include <cstdlib>
#include <mutex>
#include <unordered_map>

#include "common.h"

namespace ft {

static thread_local std::string g_last_error;

void set_error(const char* fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    std::vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_last_error = buf;
}

void clear_error() { g_last_error.clear(); }

const char* last_error() { return g_last_error.c_str(); }

// Optional allocation cap (FT_MAX_BYTES) so that the out-of-memory path can
// be exercised without exhausting the device.
static std::mutex g_alloc_mu;
static size_t g_alloc_bytes = 0;
static std::unordered_map<void*, size_t> g_alloc_sizes;

static size_t byte_cap() {
    const char* e = std::getenv("FT_MAX_BYTES");
    if (!e || !*e) return SIZE_MAX;
    return (size_t)std::strtoull(e, nullptr, 10);
}

ft_status dev_alloc(void** p, size_t bytes) {
    *p = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        if (g_alloc_bytes + bytes > byte_cap()) {
            set_error("allocation of %zu bytes exceeds FT_MAX_BYTES", bytes);
            return FT_E_OOM;
        }
        g_alloc_bytes += bytes;
    }
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        g_alloc_bytes -= bytes;
        *p = nullptr;
        set_error("hipMalloc(%zu) failed: %s", bytes, hipGetErrorString(e));
        return e == hipErrorOutOfMemory ? FT_E_OOM : FT_E_DEVICE;
    }
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_alloc_sizes[*p] = bytes;
    return FT_OK;
}

void dev_free(void* p) {
    if (!p) return;
    {
        std::lock_guard<std::mutex> lk(g_alloc_mu);
        auto it = g_alloc_sizes.find(p);
        if (it != g_alloc_sizes.end()) {
            g_alloc_bytes -= it->second;
            g_alloc_sizes.erase(it);
        }
    }
    (void)hipFree(p);
}

// ---------------------------------------------------------------- exclusive scan
// Three phases over chunks of SCAN_CHUNK counts: per-chunk totals, a
// sequential scan of the totals by one block, then a per-chunk rescan with
// the chunk's offset.  Integer arithmetic, so the result is exact.
constexpr int SCAN_BLOCK = 256;
constexpr int SCAN_PER_THREAD = 8;
constexpr int SCAN_CHUNK = SCAN_BLOCK * SCAN_PER_THREAD;

__global__ void k_scan_chunk_totals(const int32_t* __restrict__ counts, int64_t n, int64_t* __restrict__ totals) {
    __shared__ int64_t red[SCAN_BLOCK];
    const int64_t base = int64_t(blockIdx.x) * SCAN_CHUNK + threadIdx.x * SCAN_PER_THREAD;
    int64_t s = 0;
    for (int i = 0; i < SCAN_PER_THREAD; ++i)
        if (base + i < n) s += counts[base + i];
    red[threadIdx.x] = s;
    __syncthreads();
    for (int o = SCAN_BLOCK / 2; o > 0; o >>= 1) {
        if (threadIdx.x < o) red[threadIdx.x] += red[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) totals[blockIdx.x] = red[0];
}

__global__ void k_scan_totals(int64_t* __restrict__ totals, int64_t nchunks, int64_t* __restrict__ grand_out) {
    // one block: sequential passes of SCAN_BLOCK-wide inclusive scans
    __shared__ int64_t buf[SCAN_BLOCK];
    __shared__ int64_t carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int64_t base = 0; base < nchunks; base += SCAN_BLOCK) {
        const int64_t i = base + threadIdx.x;
        const int64_t v = i < nchunks ? totals[i] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < SCAN_BLOCK; o <<= 1) {
            const int64_t add = threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
            __syncthreads();
            buf[threadIdx.x] += add;
            __syncthreads();
        }
        if (i < nchunks) totals[i] = carry + buf[threadIdx.x] - v;   // exclusive
        __syncthreads();
        if (threadIdx.x == 0) carry += buf[SCAN_BLOCK - 1];
        __syncthreads();
    }
    if (threadIdx.x == 0) *grand_out = carry;
}

__global__ void k_scan_apply(const int32_t* __restrict__ counts, int64_t n, const int64_t* __restrict__ chunk_off,
                             int64_t* __restrict__ out) {
    __shared__ int64_t buf[SCAN_BLOCK];
    const int64_t base = int64_t(blockIdx.x) * SCAN_CHUNK + threadIdx.x * SCAN_PER_THREAD;
    int64_t local[SCAN_PER_THREAD];
    int64_t s = 0;
    for (int i = 0; i < SCAN_PER_THREAD; ++i) {
        local[i] = s;
        if (base + i < n) s += counts[base + i];
    }
    buf[threadIdx.x] = s;
    __syncthreads();
    for (int o = 1; o < SCAN_BLOCK; o <<= 1) {
        const int64_t add = threadIdx.x >= o ? buf[threadIdx.x - o] : 0;
        __syncthreads();
        buf[threadIdx.x] += add;
        __syncthreads();
    }
    const int64_t off = chunk_off[blockIdx.x] + buf[threadIdx.x] - s;
    for (int i = 0; i < SCAN_PER_THREAD; ++i)
        if (base + i < n) out[base + i] = off + local[i];
}

int64_t scan_tmp_elems(int64_t n) { return (n + SCAN_CHUNK - 1) / SCAN_CHUNK + 2; }

ft_status exclusive_scan(const int32_t* counts, int64_t* offsets, int64_t n, int64_t* tmp, hipStream_t s) {
    const int64_t nchunks = (n + SCAN_CHUNK - 1) / SCAN_CHUNK;
    if (nchunks == 0) {
        FT_TRY_HIP(hipMemsetAsync(offsets, 0, sizeof(int64_t), s));
        return FT_OK;
    }
    k_scan_chunk_totals<<<(unsigned)nchunks, SCAN_BLOCK, 0, s>>>(counts, n, tmp);
    k_scan_totals<<<1, SCAN_BLOCK, 0, s>>>(tmp, nchunks, offsets + n);
    k_scan_apply<<<(unsigned)nchunks, SCAN_BLOCK, 0, s>>>(counts, n, tmp, offsets);
    FT_TRY_HIP(hipGetLastError());
    return FT_OK;
}

}  // namespace ft
