// Device-wide exclusive scan and stable LSD radix sort of (u64 key, i32 value)
// pairs, written for 64-wide wavefronts.
//
// Sort: 8-bit digits; per pass one histogram kernel and one scatter kernel.
// A block owns a tile of kTile = 8 * 256 consecutive elements and walks it in
// 8 rounds of 256; inside a round, ranks among equal digits come from
// wavefront ballots (8 ballots give each lane the mask of lanes sharing its
// digit) and a per-digit prefix over the 4 wavefronts, so equal keys keep
// their input order (stability).  Ties of the Morton keys are thereby broken
// by the original index, which the values start out as.
#include "sort.h"

namespace fmm {

constexpr int kThreads = 256;
constexpr int kItems = 8;
constexpr int kTile = kThreads * kItems;
constexpr int kWaves = kThreads / 64;

// ---------------- scan ----------------
template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_block_sums(const T *in, int64_t n, T *sums)
{
    __shared__ T sh[kWaves];
    int64_t base = (int64_t)blockIdx.x * kTile;
    T s = 0;
    for (int r = 0; r < kItems; ++r) {
        int64_t i = base + r * kThreads + threadIdx.x;
        if (i < n) s += in[i];
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        T t = 0;
        for (int w = 0; w < kWaves; ++w) t += sh[w];
        sums[blockIdx.x] = t;
    }
}

// one block scans the block sums in place (exclusive), total at sums[nb]
template <typename T>
__device__ inline void k_scan_sums_body(T *sums, int nb)
{
    __shared__ T sh[1024];
    __shared__ T carry;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nb; base += 1024) {
        int i = base + threadIdx.x;
        T v = i < nb ? sums[i] : 0;
        sh[threadIdx.x] = v;
        __syncthreads();
        for (int o = 1; o < 1024; o <<= 1) {
            T t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
            __syncthreads();
            sh[threadIdx.x] += t;
            __syncthreads();
        }
        if (i < nb) sums[i] = carry + sh[threadIdx.x] - v;
        __syncthreads();
        if (threadIdx.x == 1023) carry += sh[1023];
        __syncthreads();
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

template <typename T>
__device__ inline void k_scan_apply_body(const T *in, int64_t n, const T *sums, T *out, int write_total)
{
    __shared__ T sh[kThreads];
    int64_t base = (int64_t)blockIdx.x * kTile;
    T v[kItems];
    T tot = 0;
    for (int r = 0; r < kItems; ++r) {
        int64_t i = base + threadIdx.x * kItems + r;
        v[r] = i < n ? in[i] : 0;
        tot += v[r];
    }
    sh[threadIdx.x] = tot;
    __syncthreads();
    for (int o = 1; o < kThreads; o <<= 1) {
        T t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    T run = sums[blockIdx.x] + sh[threadIdx.x] - tot;
    for (int r = 0; r < kItems; ++r) {
        int64_t i = base + threadIdx.x * kItems + r;
        if (i < n) out[i] = run;
        run += v[r];
    }
    if (write_total && blockIdx.x == gridDim.x - 1 && threadIdx.x == kThreads - 1)
        out[n] = sums[gridDim.x];
}

template <typename T>
__global__ __launch_bounds__(1024) void k_scan_sums(T *sums, int nb)
{
    k_scan_sums_body(sums, nb);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void k_scan_apply(const T *in, int64_t n, const T *sums,
                                                         T *out, int write_total)
{
    k_scan_apply_body(in, n, sums, out, write_total);
}

// Several scans of equal length in one set of launches (blockIdx.y = scan).
struct ScanBatch {
    const int64_t *in[kMaxScanBatch];
    int64_t *out[kMaxScanBatch];
};

__global__ __launch_bounds__(kThreads) void k_scan_block_sums_m(ScanBatch sb, int64_t n, int64_t *sums,
                                                                 int64_t stride)
{
    __shared__ int64_t sh[kWaves];
    const int64_t *in = sb.in[blockIdx.y];
    int64_t base = (int64_t)blockIdx.x * kTile;
    int64_t s = 0;
    for (int r = 0; r < kItems; ++r) {
        int64_t i = base + r * kThreads + threadIdx.x;
        if (i < n) s += in[i];
    }
    for (int o = 32; o > 0; o >>= 1) s += __shfl_down(s, o);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        int64_t t = 0;
        for (int w = 0; w < kWaves; ++w) t += sh[w];
        sums[blockIdx.y * stride + blockIdx.x] = t;
    }
}

__global__ __launch_bounds__(1024) void k_scan_sums_m(int64_t *sums, int nb, int64_t stride)
{
    k_scan_sums_body(sums + blockIdx.x * stride, nb);
}

__global__ __launch_bounds__(kThreads) void k_scan_apply_m(ScanBatch sb, int64_t n, const int64_t *sums,
                                                           int64_t stride)
{
    k_scan_apply_body(sb.in[blockIdx.y], n, sums + blockIdx.y * stride, sb.out[blockIdx.y], 1);
}

size_t scan_multi_scratch_bytes(int64_t n, int count)
{
    return sizeof(int64_t) * (ceil_div(n > 0 ? n : 1, kTile) + 2) * (size_t)count;
}

void scan_exclusive_multi(const int64_t *const *in, int64_t *const *out, int count, int64_t n,
                          int64_t *scratch, hipStream_t s)
{
    ScanBatch sb{};
    for (int i = 0; i < count; ++i) { sb.in[i] = in[i]; sb.out[i] = out[i]; }
    unsigned nb = ceil_div(n > 0 ? n : 1, kTile);
    int64_t stride = nb + 2;
    k_scan_block_sums_m<<<dim3(nb, count), kThreads, 0, s>>>(sb, n, scratch, stride);
    k_scan_sums_m<<<count, 1024, 0, s>>>(scratch, (int)nb, stride);
    k_scan_apply_m<<<dim3(nb, count), kThreads, 0, s>>>(sb, n, scratch, stride);
}

size_t scan_scratch_bytes(int64_t n) { return sizeof(int64_t) * (ceil_div(n > 0 ? n : 1, kTile) + 2); }

void scan_exclusive(const int64_t *in, int64_t *out, int64_t n, int64_t *scratch, hipStream_t s)
{
    unsigned nb = ceil_div(n > 0 ? n : 1, kTile);
    k_scan_block_sums<int64_t><<<nb, kThreads, 0, s>>>(in, n, scratch);
    k_scan_sums<int64_t><<<1, 1024, 0, s>>>(scratch, (int)nb);
    k_scan_apply<int64_t><<<nb, kThreads, 0, s>>>(in, n, scratch, out, 1);
}

// one block, in place, for short arrays (n <= kSmallScan, the digit counts of
// sorts up to 64k elements): 1024 threads own
// runs of n/1024 consecutive elements
constexpr int kSmallScan = 1024 * 8;
__global__ __launch_bounds__(1024) void k_scan_small(int32_t *data, int n)
{
    __shared__ int32_t sh[1024];
    const int per = (n + 1023) / 1024, b = threadIdx.x * per, e = min(b + per, n);
    int32_t tot = 0;
    for (int i = b; i < e; ++i) tot += data[i];
    sh[threadIdx.x] = tot;
    __syncthreads();
    for (int o = 1; o < 1024; o <<= 1) {
        int32_t t = threadIdx.x >= o ? sh[threadIdx.x - o] : 0;
        __syncthreads();
        sh[threadIdx.x] += t;
        __syncthreads();
    }
    int32_t run = sh[threadIdx.x] - tot;
    for (int i = b; i < e; ++i) {
        int32_t v = data[i];
        data[i] = run;
        run += v;
    }
}

static void scan_exclusive_i32(int32_t *data, int64_t n, int32_t *scratch, hipStream_t s)
{
    if (n <= kSmallScan) {
        k_scan_small<<<1, 1024, 0, s>>>(data, (int)n);
        return;
    }
    unsigned nb = ceil_div(n > 0 ? n : 1, kTile);
    k_scan_block_sums<int32_t><<<nb, kThreads, 0, s>>>(data, n, scratch);
    k_scan_sums<int32_t><<<1, 1024, 0, s>>>(scratch, (int)nb);
    k_scan_apply<int32_t><<<nb, kThreads, 0, s>>>(data, n, scratch, data, 0);
}

// ---------------- radix sort ----------------
__global__ __launch_bounds__(kThreads) void k_digit_hist(const uint64_t *keys, int n, int shift,
                                                         int nblocks, int32_t *hist)
{
    __shared__ int32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int base = blockIdx.x * kTile;
    for (int r = 0; r < kItems; ++r) {
        int i = base + r * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255], 1);
    }
    __syncthreads();
    hist[threadIdx.x * nblocks + blockIdx.x] = h[threadIdx.x]; // digit-major
}

__global__ __launch_bounds__(kThreads) void k_digit_scatter(const uint64_t *keys, const int32_t *vals,
                                                            int n, int shift, int nblocks,
                                                            const int32_t *offs, uint64_t *okeys,
                                                            int32_t *ovals)
{
    __shared__ int32_t run[256];        // running count per digit over earlier rounds
    __shared__ int32_t wcnt[kWaves][256];
    __shared__ int32_t wbase[kWaves][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    run[threadIdx.x] = offs[threadIdx.x * nblocks + blockIdx.x];
    int base = blockIdx.x * kTile;
    for (int r = 0; r < kItems; ++r) {
        for (int w = 0; w < kWaves; ++w) wcnt[w][threadIdx.x] = 0;
        __syncthreads();
        int i = base + r * kThreads + threadIdx.x;
        bool valid = i < n;
        uint64_t key = valid ? keys[i] : 0;
        int32_t val = valid ? vals[i] : 0;
        int d = valid ? (int)((key >> shift) & 255) : 0;
        // lanes of this wave holding the same digit
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; ++b) {
            uint64_t m = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? m : ~m;
        }
        uint64_t below = peers & ((1ull << lane) - 1ull);
        int rank = __popcll(below);
        bool leader = valid && below == 0;
        if (leader) wcnt[wave][d] = __popcll(peers);
        __syncthreads();
        { // per digit: offsets of each wave, then advance the running count
            int dd = threadIdx.x;
            int s = run[dd];
            for (int w = 0; w < kWaves; ++w) {
                wbase[w][dd] = s;
                s += wcnt[w][dd];
            }
            run[dd] = s;
        }
        __syncthreads();
        if (valid) {
            int pos = wbase[wave][d] + rank;
            okeys[pos] = key;
            ovals[pos] = val;
        }
        __syncthreads();
    }
}

size_t sort_scratch_bytes(int n)
{
    size_t h = 256 * (size_t)ceil_div(n > 0 ? n : 1, kTile);
    return sizeof(int32_t) * (h + ceil_div((long long)h, kTile) + 2);
}

// Sorts by the low `bits` bits of the keys.  Result ends in (keys, vals);
// (tk, tv) are scratch of the same size.
void radix_sort_pairs(uint64_t *keys, int32_t *vals, uint64_t *tk, int32_t *tv, int n, int bits,
                      int32_t *hist, hipStream_t s)
{
    if (n <= 1 || bits <= 0) return;
    int nb = (int)ceil_div(n, kTile);
    int passes = (bits + 7) / 8;
    uint64_t *ik = keys, *ok = tk;
    int32_t *iv = vals, *ov = tv;
    for (int ps = 0; ps < passes; ++ps) {
        int shift = 8 * ps;
        k_digit_hist<<<nb, kThreads, 0, s>>>(ik, n, shift, nb, hist);
        scan_exclusive_i32(hist, 256LL * nb, hist + 256 * (size_t)nb, s);
        k_digit_scatter<<<nb, kThreads, 0, s>>>(ik, iv, n, shift, nb, hist, ok, ov);
        uint64_t *t = ik; ik = ok; ok = t;
        int32_t *u = iv; iv = ov; ov = u;
    }
    if (ik != keys) {
        hipMemcpyAsync(keys, ik, sizeof(uint64_t) * (size_t)n, hipMemcpyDeviceToDevice, s);
        hipMemcpyAsync(vals, iv, sizeof(int32_t) * (size_t)n, hipMemcpyDeviceToDevice, s);
    }
}

} // namespace fmm
