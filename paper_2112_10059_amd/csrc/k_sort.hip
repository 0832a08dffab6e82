// Morton keys, LSD radix sort of (key, index) pairs, device-wide exclusive scans.
//
// The octree of Sec. 2.4 (leaf cubes holding at most a prescribed number of
// points) is built from points ordered along a 63-bit Morton curve: 21-bit
// quantised coordinates in the root cube, bits interleaved x, y, z from the
// most significant end, so every octree box is a contiguous run of keys.
#include <hip/hip_runtime.h>

#include "k_common.h"

namespace ph {

namespace {

constexpr int kBlock = 256;
constexpr int kItems = 8;                    // keys per thread in the radix passes
constexpr int kTile = kBlock * kItems;       // keys per workgroup tile
constexpr int kScanItems = 16;
constexpr int kScanTile = kBlock * kScanItems;

__device__ __forceinline__ uint64_t spread3(uint32_t v)
{
    uint64_t x = v & 0x1fffffu;
    x = (x | (x << 32)) & 0x001f00000000ffffull;
    x = (x | (x << 16)) & 0x001f0000ff0000ffull;
    x = (x | (x << 8)) & 0x100f00f00f00f00full;
    x = (x | (x << 4)) & 0x10c30c30c30c30c3ull;
    x = (x | (x << 2)) & 0x1249249249249249ull;
    return x;
}

__device__ __forceinline__ uint32_t quantise(double x, double lo, double size)
{
    double f = floor((x - lo) / size * 2097152.0);
    if (f < 0.0) f = 0.0;
    if (f > 2097151.0) f = 2097151.0;
    return (uint32_t)f;
}

__global__ void morton_kernel(const double *__restrict__ xyz, int64_t n, double lo0, double lo1, double lo2,
                              double size, uint64_t *__restrict__ keys, int32_t *__restrict__ idx)
{
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint32_t ix = quantise(xyz[3 * i], lo0, size);
    uint32_t iy = quantise(xyz[3 * i + 1], lo1, size);
    uint32_t iz = quantise(xyz[3 * i + 2], lo2, size);
    keys[i] = (spread3(ix) << 2) | (spread3(iy) << 1) | spread3(iz);
    idx[i] = (int32_t)i;
}

__global__ void gather_sorted_kernel(const double *__restrict__ xyz, const double *__restrict__ w,
                                     const int32_t *__restrict__ perm, int64_t n, double *__restrict__ xyz_s,
                                     double *__restrict__ w_s, int32_t *__restrict__ iperm)
{
    int64_t k = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int32_t o = perm[k];
    xyz_s[3 * k] = xyz[3 * (int64_t)o];
    xyz_s[3 * k + 1] = xyz[3 * (int64_t)o + 1];
    xyz_s[3 * k + 2] = xyz[3 * (int64_t)o + 2];
    if (w) w_s[k] = w[o];
    iperm[o] = (int32_t)k;
}

// ---------------------------------------------------------------- radix sort

// Histogram of one 8-bit digit per tile, stored digit-major: hist[d * nblocks + b].
__global__ void radix_hist_kernel(const uint64_t *__restrict__ keys, int64_t n, int shift,
                                  uint32_t *__restrict__ hist, int nblocks)
{
    __shared__ uint32_t cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kTile;
    for (int it = 0; it < kItems; ++it) {
        int64_t i = base + (int64_t)it * kBlock + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[(size_t)threadIdx.x * nblocks + blockIdx.x] = cnt[threadIdx.x];
}

// Stable scatter.  Wave w of the workgroup owns the contiguous quarter
// [base + w*kTile/4, base + (w+1)*kTile/4) of the tile and walks it 64 keys at
// a time; lanes holding equal digits are ranked by a ballot-built match mask.
__device__ __forceinline__ uint64_t match_digit(uint32_t d, bool valid)
{
    uint64_t m = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
        uint64_t bal = __ballot(valid && ((d >> b) & 1u));
        m &= ((d >> b) & 1u) ? bal : ~bal;
    }
    return m;
}

__global__ void radix_scatter_kernel(const uint64_t *__restrict__ keys, const int32_t *__restrict__ vals,
                                     int64_t n, int shift, const uint32_t *__restrict__ offs, int nblocks,
                                     uint64_t *__restrict__ keys_out, int32_t *__restrict__ vals_out)
{
    __shared__ uint32_t wcnt[4][256];
    __shared__ uint32_t wbase[4][256];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int d = threadIdx.x; d < 256; d += kBlock) {
        wcnt[0][d] = wcnt[1][d] = wcnt[2][d] = wcnt[3][d] = 0;
    }
    __syncthreads();
    const int64_t base = (int64_t)blockIdx.x * kTile + (int64_t)wave * (kTile / 4);
    const uint64_t lt_mask = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    // pass 1: per-wave digit counts
    for (int r = 0; r < kTile / 4 / 64; ++r) {
        int64_t i = base + r * 64 + lane;
        bool valid = i < n;
        uint32_t d = valid ? (uint32_t)((keys[i] >> shift) & 255u) : 0u;
        uint64_t m = match_digit(d, valid);
        if (valid && (m & lt_mask) == 0) wcnt[wave][d] += (uint32_t)__popcll(m);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < 256; d += kBlock) {
        uint32_t g = offs[(size_t)d * nblocks + blockIdx.x];
        uint32_t acc = 0;
        for (int w = 0; w < 4; ++w) {
            wbase[w][d] = g + acc;
            acc += wcnt[w][d];
        }
    }
    __syncthreads();
    // pass 2: rank and scatter in order
    for (int r = 0; r < kTile / 4 / 64; ++r) {
        int64_t i = base + r * 64 + lane;
        bool valid = i < n;
        uint64_t k = valid ? keys[i] : 0ull;
        uint32_t d = (uint32_t)((k >> shift) & 255u);
        uint64_t m = match_digit(d, valid);
        if (valid) {
            uint32_t pos = wbase[wave][d] + (uint32_t)__popcll(m & lt_mask);
            keys_out[pos] = k;
            vals_out[pos] = vals[i];
        }
        // the lowest lane of each digit group advances the running base
        __builtin_amdgcn_wave_barrier();
        if (valid && (m & lt_mask) == 0) wbase[wave][d] += (uint32_t)__popcll(m);
        __builtin_amdgcn_wave_barrier();
    }
}

// ---------------------------------------------------------------- scan
//
// Exclusive scan in three passes over tiles of kScanTile elements (256 threads, 16 per thread):
// tile sums, a scan of the tile sums, and the tile scans.  Inside a tile each wave owns a
// contiguous quarter, read as 16 coalesced strips of 64 and scanned across lanes with shuffles;
// the waves' totals are exchanged once through LDS.  Integer sums: the order does not matter.

constexpr int kWaveSpan = kScanTile / 4;  // elements per wave in a tile

template <class T>
__global__ __launch_bounds__(256) void scan_reduce_kernel(const T *__restrict__ data, int64_t n, T *__restrict__ partial)
{
    __shared__ T wsum[4];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)w * kWaveSpan;
    T acc = 0;
#pragma unroll
    for (int st = 0; st < kWaveSpan / 64; ++st) {
        const int64_t i = base + st * 64 + lane;
        if (i < n) acc += data[i];
    }
    acc = lane_value(wave_inclusive(acc, lane), 63);
    if (lane == 0) wsum[w] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = wsum[0] + wsum[1] + wsum[2] + wsum[3];
}

// one workgroup of 1024 threads: exclusive scan of the nb tile sums, total to *total
template <class T>
__global__ __launch_bounds__(1024) void scan_partials_kernel(T *__restrict__ partial, int64_t nb, T *__restrict__ total)
{
    __shared__ T wtot[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    T carry = 0;
    for (int64_t base = 0; base < nb; base += 1024) {
        const int64_t i = base + threadIdx.x;
        const T v = i < nb ? partial[i] : T(0);
        const T incl = wave_inclusive(v, lane);
        __syncthreads();  // the previous strip's totals have been read
        if (lane == 63) wtot[w] = incl;
        __syncthreads();
        T before = carry;
        for (int q = 0; q < w; ++q) before += wtot[q];
        if (i < nb) partial[i] = before + incl - v;
        for (int q = 0; q < 16; ++q) carry += wtot[q];
    }
    if (threadIdx.x == 0 && total) *total = carry;
}

template <class T>
__global__ __launch_bounds__(256) void scan_apply_kernel(T *__restrict__ data, int64_t n, const T *__restrict__ partial)
{
    __shared__ T wsum[4];
    constexpr int kStrips = kWaveSpan / 64;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)w * kWaveSpan;
    T loc[kStrips];
    T acc = 0;
#pragma unroll
    for (int st = 0; st < kStrips; ++st) {
        const int64_t i = base + st * 64 + lane;
        loc[st] = i < n ? data[i] : T(0);
        acc += loc[st];
    }
    acc = lane_value(wave_inclusive(acc, lane), 63);
    if (lane == 0) wsum[w] = acc;
    __syncthreads();
    T carry = partial[blockIdx.x];
    for (int q = 0; q < w; ++q) carry += wsum[q];
#pragma unroll
    for (int st = 0; st < kStrips; ++st) {
        const T incl = wave_inclusive(loc[st], lane);
        const int64_t i = base + st * 64 + lane;
        if (i < n) data[i] = carry + incl - loc[st];
        carry += lane_value(incl, 63);
    }
}

// Small arrays in one launch: one workgroup of 16 waves, wave w owning a contiguous range of
// kSmallStrips strips of 64 held in registers (loads issued together).
constexpr int kSmallStrips = 40;
constexpr int64_t kSmallScan = 16 * 64 * kSmallStrips;

template <class T>
struct ScanJob {
    T *data;
    T *total;
};

// workgroup j scans array j of up to three (one launch for independent small scans)
template <class T>
__global__ __launch_bounds__(1024) void scan_small_kernel(ScanJob<T> j0, ScanJob<T> j1, ScanJob<T> j2, int64_t n)
{
    const ScanJob<T> job = blockIdx.x == 0 ? j0 : (blockIdx.x == 1 ? j1 : j2);
    T *__restrict__ data = job.data;
    T *__restrict__ total = job.total;
    __shared__ T wsum[16];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t span = ((n + 16 * 64 - 1) / (16 * 64)) * 64;  // elements per wave, a multiple of 64
    const int64_t base = (int64_t)w * span;
    const int strips = (int)(span / 64);
    T loc[sizeof(T) == 4 ? kSmallStrips : 1];
    T acc = 0;
#pragma unroll
    for (int st = 0; st < kSmallStrips; ++st) {
        const int64_t i = base + st * 64 + lane;
        const T v = (st < strips && i < n) ? data[i] : T(0);
        if constexpr (sizeof(T) == 4) loc[st] = v;
        acc += v;
    }
    acc = lane_value(wave_inclusive(acc, lane), 63);
    if (lane == 0) wsum[w] = acc;
    __syncthreads();
    T carry = 0;
    for (int q = 0; q < w; ++q) carry += wsum[q];
    if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int st = 0; st < kSmallStrips; ++st) {
            if (st < strips) {  // a guard, not a break: the strips stay in registers
                const T incl = wave_inclusive(loc[st], lane);
                const int64_t i = base + st * 64 + lane;
                if (i < n) data[i] = carry + incl - loc[st];
                carry += lane_value(incl, 63);
            }
        }
    } else {
        // 64-bit values: read again (from L2) half a span at a time; 40 held would spill
        constexpr int kHalf = kSmallStrips / 2;
        for (int h = 0; h < kSmallStrips; h += kHalf) {
            T v[kHalf];
#pragma unroll
            for (int u = 0; u < kHalf; ++u) {
                const int64_t i = base + (h + u) * 64 + lane;
                v[u] = (h + u < strips && i < n) ? data[i] : T(0);
            }
#pragma unroll
            for (int u = 0; u < kHalf; ++u) {
                if (h + u < strips) {
                    const T incl = wave_inclusive(v[u], lane);
                    const int64_t i = base + (h + u) * 64 + lane;
                    if (i < n) data[i] = carry + incl - v[u];
                    carry += lane_value(incl, 63);
                }
            }
        }
    }
    if (threadIdx.x == 1023 && total) *total = carry;
}

template <class T>
void exclusive_scan(T *data, int64_t n, void *tmp, T *total, hipStream_t s)
{
    if (n <= 0) return;
    if (n <= kSmallScan) {
        const ScanJob<T> j{data, total};
        scan_small_kernel<T><<<1, 1024, 0, s>>>(j, j, j, n);
        return;
    }
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    T *partial = (T *)tmp;
    scan_reduce_kernel<T><<<(unsigned)nb, 256, 0, s>>>(data, n, partial);
    scan_partials_kernel<T><<<1, 1024, 0, s>>>(partial, nb, total);
    scan_apply_kernel<T><<<(unsigned)nb, 256, 0, s>>>(data, n, partial);
}

}  // namespace

void scan_tile_sums_u64(uint64_t *partial, int64_t nb, uint64_t *total, hipStream_t s)
{
    scan_partials_kernel<uint64_t><<<1, 1024, 0, s>>>(partial, nb, total);
}

size_t scan_tmp_bytes(int64_t n, size_t elem)
{
    int64_t nb = (n + kScanTile - 1) / kScanTile;
    return (size_t)(nb + 1) * elem + 256;
}

void exclusive_scan_u32(uint32_t *data, int64_t n, void *tmp, uint32_t *total, hipStream_t s)
{
    exclusive_scan<uint32_t>(data, n, tmp, total, s);
}

void exclusive_scan_u64(uint64_t *data, int64_t n, void *tmp, uint64_t *total, hipStream_t s)
{
    exclusive_scan<uint64_t>(data, n, tmp, total, s);
}


void launch_morton_keys(const double *xyz, int64_t n, double lo0, double lo1, double lo2, double size,
                        uint64_t *keys, int32_t *idx, hipStream_t s)
{
    morton_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(xyz, n, lo0, lo1, lo2, size, keys, idx);
}

void launch_gather_sorted(const double *xyz, const double *w, const int32_t *perm, int64_t n, double *xyz_s,
                          double *w_s, int32_t *iperm, hipStream_t s)
{
    gather_sorted_kernel<<<(unsigned)((n + 255) / 256), 256, 0, s>>>(xyz, w, perm, n, xyz_s, w_s, iperm);
}

size_t radix_sort_tmp_bytes(int64_t n)
{
    int64_t nb = (n + kTile - 1) / kTile;
    return (size_t)256 * nb * 4 + scan_tmp_bytes(256 * nb, 4);
}

void radix_sort_pairs(uint64_t *keys, int32_t *vals, uint64_t *keys_tmp, int32_t *vals_tmp, int64_t n,
                      uint32_t *hist_tmp, size_t, int key_bits, hipStream_t s)
{
    const int nblocks = (int)((n + kTile - 1) / kTile);
    uint32_t *hist = hist_tmp;
    void *scan_tmp = hist_tmp + (size_t)256 * nblocks;
    uint64_t *kin = keys, *kout = keys_tmp;
    int32_t *vin = vals, *vout = vals_tmp;
    int passes = (key_bits + 7) / 8;
    if (passes & 1) passes += 1;  // even number of passes: the result lands back in keys/vals
    for (int p = 0; p < passes; ++p) {
        int shift = 8 * p;
        radix_hist_kernel<<<nblocks, kBlock, 0, s>>>(kin, n, shift, hist, nblocks);
        exclusive_scan<uint32_t>(hist, (int64_t)256 * nblocks, scan_tmp, nullptr, s);
        radix_scatter_kernel<<<nblocks, kBlock, 0, s>>>(kin, vin, n, shift, hist, nblocks, kout, vout);
        std::swap(kin, kout);
        std::swap(vin, vout);
    }
}

}  // namespace ph
