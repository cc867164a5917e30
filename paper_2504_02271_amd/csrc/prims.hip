// Device-wide primitives for gfx950: exclusive scan and a stable LSD radix
// sort (8-bit digits, wave64 ballot ranking).  Used by the CSR builder, the
// hyperwedge builder and the closure scheduler.
#include "internal.hpp"

namespace htri {

namespace {

constexpr int kScanBlock = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanBlock * kScanItems;

__device__ __forceinline__ int lane_id() { return (int)__lane_id(); }

template <typename T>
__device__ __forceinline__ T wave_incl_scan(T v) {
    const int lane = lane_id();
#pragma unroll
    for (int o = 1; o < kWave; o <<= 1) {
        T u = __shfl_up(v, o, kWave);
        if (lane >= o) v += u;
    }
    return v;
}

// Block-wide exclusive scan of one value per thread; returns the prefix and
// writes the block total to *total (all threads).
template <typename T>
__device__ __forceinline__ T block_excl_scan(T v, T *smem /*[kScanBlock/kWave + 1]*/, T *total) {
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    const int nwaves = blockDim.x / kWave;
    T incl = wave_incl_scan(v);
    if (lane == kWave - 1) smem[wave] = incl;
    __syncthreads();
    if (threadIdx.x == 0) {
        T run = 0;
        for (int w = 0; w < nwaves; w++) {
            T c = smem[w];
            smem[w] = run;
            run += c;
        }
        smem[nwaves] = run;
    }
    __syncthreads();
    T res = smem[wave] + incl - v;
    *total = smem[nwaves];
    __syncthreads();
    return res;
}

template <typename T>
__global__ __launch_bounds__(kScanBlock) void k_scan_reduce(const T *in, int64_t n, T *partials) {
    __shared__ T smem[kScanBlock / kWave + 1];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T sum = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; q++) {
        int64_t i = base + q;
        if (i < n) sum += in[i];
    }
    T total;
    (void)block_excl_scan<T>(sum, smem, &total);
    if (threadIdx.x == 0) partials[blockIdx.x] = total;
}

template <typename T>
__global__ __launch_bounds__(kScanBlock) void k_scan_down(const T *in, T *out, int64_t n,
                                                          const T *offsets, T *total_out) {
    __shared__ T smem[kScanBlock / kWave + 1];
    int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    T vals[kScanItems];
    T sum = 0;
#pragma unroll
    for (int q = 0; q < kScanItems; q++) {
        int64_t i = base + q;
        vals[q] = i < n ? in[i] : T(0);
        sum += vals[q];
    }
    T total;
    T pre = block_excl_scan<T>(sum, smem, &total);
    T run = (offsets ? offsets[blockIdx.x] : T(0)) + pre;
#pragma unroll
    for (int q = 0; q < kScanItems; q++) {
        int64_t i = base + q;
        if (i < n) out[i] = run;
        run += vals[q];
    }
    if (total_out && blockIdx.x == gridDim.x - 1 && threadIdx.x == blockDim.x - 1)
        *total_out = run;
}

// total of an empty scan: a kernel rather than a memset node, so that a
// captured launch sequence holds no memset
template <typename T>
__global__ void k_zero_one(T *p) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *p = T(0);
}

template <typename T>
void scan_exclusive(Allocator &a, const T *in, T *out, int64_t n, T *total, hipStream_t s) {
    if (n <= 0) {
        if (total) {
            hipLaunchKernelGGL(k_zero_one<T>, dim3(1), dim3(64), 0, s, total);
            HTRI_LAUNCH_CHECK();
        }
        return;
    }
    int64_t tiles = (n + kScanTile - 1) / kScanTile;
    if (tiles == 1) {
        hipLaunchKernelGGL(k_scan_down<T>, dim3(1), dim3(kScanBlock), 0, s, in, out, n, nullptr, total);
        HTRI_LAUNCH_CHECK();
        return;
    }
    DBuf<T> part(a, tiles);
    hipLaunchKernelGGL(k_scan_reduce<T>, dim3((unsigned)tiles), dim3(kScanBlock), 0, s, in, n, part.p);
    HTRI_LAUNCH_CHECK();
    scan_exclusive<T>(a, part.p, part.p, tiles, nullptr, s);
    hipLaunchKernelGGL(k_scan_down<T>, dim3((unsigned)tiles), dim3(kScanBlock), 0, s, in, out, n, part.p,
                       total);
    HTRI_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- radix sort

constexpr int kSortBlock = 256;
constexpr int kSortWaves = kSortBlock / kWave;
constexpr int kSortItems = 16;
constexpr int kSortTile = kSortBlock * kSortItems;
constexpr int kRadix = 256;

// Per-tile digit histogram, digit-major: hist[d * ntiles + tile].
__global__ __launch_bounds__(kSortBlock) void k_rs_hist(const uint64_t *keys, int64_t n, int shift,
                                                        uint32_t *hist, int64_t ntiles) {
    __shared__ uint32_t h[kSortWaves][kRadix];
    const int wave = threadIdx.x / kWave;
    for (int t = threadIdx.x; t < kSortWaves * kRadix; t += kSortBlock) (&h[0][0])[t] = 0;
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
#pragma unroll 4
    for (int q = 0; q < kSortItems; q++) {
        int64_t i = base + (int64_t)q * kSortBlock + threadIdx.x;
        if (i < n) atomicAdd(&h[wave][(keys[i] >> shift) & 0xFF], 1u);
    }
    __syncthreads();
    for (int d = threadIdx.x; d < kRadix; d += kSortBlock) {
        uint32_t c = 0;
        for (int w = 0; w < kSortWaves; w++) c += h[w][d];
        hist[(int64_t)d * ntiles + blockIdx.x] = c;
    }
}

// Stable scatter: element order inside a tile is (round, thread); each round
// ranks its 256 elements with per-wave digit match masks.
template <bool V>
__global__ __launch_bounds__(kSortBlock) void k_rs_scatter(const uint64_t *kin, const uint32_t *vin,
                                                           int64_t n, int shift, const uint32_t *offs,
                                                           int64_t ntiles, uint64_t *kout,
                                                           uint32_t *vout) {
    __shared__ uint32_t run[kRadix];              // next output slot per digit
    __shared__ uint32_t wcnt[kSortWaves][kRadix]; // per-wave counts of a round
    const int lane = lane_id();
    const int wave = threadIdx.x / kWave;
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (kWave - lane));
    for (int d = threadIdx.x; d < kRadix; d += kSortBlock) {
        run[d] = offs[(int64_t)d * ntiles + blockIdx.x];
        for (int w = 0; w < kSortWaves; w++) wcnt[w][d] = 0;
    }
    __syncthreads();
    int64_t base = (int64_t)blockIdx.x * kSortTile;
    for (int q = 0; q < kSortItems; q++) {
        int64_t i = base + (int64_t)q * kSortBlock + threadIdx.x;
        bool valid = i < n;
        uint64_t key = valid ? kin[i] : 0;
        uint32_t val = (V && valid) ? vin[i] : 0;
        uint32_t d = (uint32_t)(key >> shift) & 0xFF;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int b = 0; b < 8; b++) {
            uint64_t bal = __ballot((d >> b) & 1);
            peers &= ((d >> b) & 1) ? bal : ~bal;
        }
        uint32_t rank = (uint32_t)__popcll(peers & lt);
        bool last = valid && ((peers >> lane) == 1ull);
        if (last) wcnt[wave][d] = rank + 1;
        __syncthreads();
        for (int dd = threadIdx.x; dd < kRadix; dd += kSortBlock) {
            uint32_t r = run[dd];
            for (int w = 0; w < kSortWaves; w++) {
                uint32_t c = wcnt[w][dd];
                wcnt[w][dd] = r;
                r += c;
            }
            run[dd] = r;
        }
        __syncthreads();
        if (valid) {
            uint32_t pos = wcnt[wave][d] + rank;
            kout[pos] = key;
            if (V) vout[pos] = val;
        }
        __syncthreads();
        // reset the per-wave counts for the next round
        for (int dd = threadIdx.x; dd < kRadix; dd += kSortBlock)
            for (int w = 0; w < kSortWaves; w++) wcnt[w][dd] = 0;
        __syncthreads();
    }
}

template <typename T>
__global__ void k_fill(T *p, int64_t n, T v) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        p[i] = v;
}

}  // namespace

void scan_exclusive_i64(Allocator &a, const int64_t *in, int64_t *out, int64_t n, int64_t *total,
                        hipStream_t s) {
    scan_exclusive<int64_t>(a, in, out, n, total, s);
}

void scan_exclusive_u32(Allocator &a, const uint32_t *in, uint32_t *out, int64_t n, uint32_t *total,
                        hipStream_t s) {
    scan_exclusive<uint32_t>(a, in, out, n, total, s);
}

// inclusive scan of doubles in a fixed summation order (exclusive scan, then add)
namespace {
__global__ void k_add_self(const double *in, double *out, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        out[i] += in[i];
}
}  // namespace

void scan_inclusive_f64(Allocator &a, const double *in, double *out, int64_t n, hipStream_t s) {
    if (n <= 0) return;
    scan_exclusive<double>(a, in, out, n, nullptr, s);
    hipLaunchKernelGGL(k_add_self, dim3(grid_for(n, 256, 8192)), dim3(256), 0, s, in, out, n);
    HTRI_LAUNCH_CHECK();
}

void radix_sort_u64(Allocator &a, uint64_t *keys, uint32_t *vals, int64_t n, int key_bits,
                    hipStream_t s) {
    if (n <= 1 || key_bits <= 0) return;
    if (n >= (int64_t)UINT32_MAX) fail(HTRI_E_UNSUPPORTED, "radix sort beyond 2^32 elements");
    int64_t ntiles = (n + kSortTile - 1) / kSortTile;
    DBuf<uint64_t> k2(a, n);
    DBuf<uint32_t> v2;
    if (vals) v2.alloc(a, n);
    DBuf<uint32_t> hist(a, (size_t)kRadix * ntiles);
    uint64_t *kin = keys, *kout = k2.p;
    uint32_t *vin = vals, *vout = v2.p;
    int passes = 0;
    for (int shift = 0; shift < key_bits; shift += 8) {
        hipLaunchKernelGGL(k_rs_hist, dim3((unsigned)ntiles), dim3(kSortBlock), 0, s, kin, n, shift,
                           hist.p, ntiles);
        HTRI_LAUNCH_CHECK();
        scan_exclusive<uint32_t>(a, hist.p, hist.p, (int64_t)kRadix * ntiles, nullptr, s);
        if (vals)
            hipLaunchKernelGGL(k_rs_scatter<true>, dim3((unsigned)ntiles), dim3(kSortBlock), 0, s, kin,
                               vin, n, shift, hist.p, ntiles, kout, vout);
        else
            hipLaunchKernelGGL(k_rs_scatter<false>, dim3((unsigned)ntiles), dim3(kSortBlock), 0, s, kin,
                               vin, n, shift, hist.p, ntiles, kout, vout);
        HTRI_LAUNCH_CHECK();
        std::swap(kin, kout);
        std::swap(vin, vout);
        passes++;
    }
    if (passes & 1) {
        HTRI_HIP(hipMemcpyAsync(keys, kin, sizeof(uint64_t) * n, hipMemcpyDeviceToDevice, s));
        if (vals) HTRI_HIP(hipMemcpyAsync(vals, vin, sizeof(uint32_t) * n, hipMemcpyDeviceToDevice, s));
    }
    // the temporaries are released when this returns; keep the stream ordered
    stream_sync(s);
}

void fill_u32(uint32_t *p, int64_t n, uint32_t v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<uint32_t>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
    HTRI_LAUNCH_CHECK();
}

void fill_u64(uint64_t *p, int64_t n, uint64_t v, hipStream_t s) {
    if (n <= 0) return;
    hipLaunchKernelGGL(k_fill<uint64_t>, dim3(grid_for(n, 256, 4096)), dim3(256), 0, s, p, n, v);
    HTRI_LAUNCH_CHECK();
}

thread_local Replay *tl_replay = nullptr;

int device_cu_count() {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess) return 256;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
    return cus > 0 ? cus : 256;
}

}  // namespace htri
