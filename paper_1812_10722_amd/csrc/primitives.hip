// Device primitives used by the geometry set-up: exclusive scan and a stable LSD radix sort
// of 64-bit keys carrying 32-bit values.  Both are hand-written for 64-wide wavefronts.
#include "primitives.hpp"

namespace lspr {

namespace {

constexpr int SCAN_THREADS = 1024;

// Single-workgroup exclusive scan of n int64 counts (setup-time sizes, up to a few million).
// out[i] = sum_{k < i} in[k]; out[n] = total.  in and out may alias: each thread reads its
// SCAN_ITEMS consecutive elements of a chunk into registers and writes only those.  Per chunk,
// the thread sums are scanned in LDS, one wave's 64 by one thread, then the 16 wave sums by
// thread 0, which carries the running total from chunk to chunk (four barriers per chunk).
constexpr int SCAN_ITEMS = 8;
__global__ void __launch_bounds__(SCAN_THREADS) k_scan_excl(const int64_t* in, int64_t* out,
                                                             int64_t n) {
    constexpr int NW = SCAN_THREADS / 64, CH = SCAN_THREADS * SCAN_ITEMS;
    __shared__ int64_t tsum[SCAN_THREADS];
    __shared__ int64_t wsum[NW];
    int64_t carry = 0;  // thread 0 only
    const int tid = threadIdx.x;
    for (int64_t base = 0; base < n; base += CH) {
        const int64_t first = base + static_cast<int64_t>(tid) * SCAN_ITEMS;
        int64_t v[SCAN_ITEMS], sum = 0;
#pragma unroll
        for (int e = 0; e < SCAN_ITEMS; ++e) {
            v[e] = first + e < n ? in[first + e] : 0;
            sum += v[e];
        }
        tsum[tid] = sum;
        __syncthreads();
        if (tid < NW) {
            int64_t a = 0;
            for (int l = 0; l < 64; ++l) {
                const int64_t t = tsum[64 * tid + l];
                tsum[64 * tid + l] = a;
                a += t;
            }
            wsum[tid] = a;
        }
        __syncthreads();
        if (tid == 0) {
            for (int w = 0; w < NW; ++w) {
                const int64_t t = wsum[w];
                wsum[w] = carry;
                carry += t;
            }
        }
        __syncthreads();
        int64_t pre = wsum[tid >> 6] + tsum[tid];
#pragma unroll
        for (int e = 0; e < SCAN_ITEMS; ++e) {
            if (first + e < n) out[first + e] = pre;
            pre += v[e];
        }
        __syncthreads();
    }
    if (tid == 0) out[n] = carry;
}

constexpr int RS_THREADS = 256;               // 4 wavefronts
constexpr int RS_ROUNDS = 16;                 // keys per thread per tile
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;
constexpr int RS_BINS = 256;                  // 8-bit digits

// Per-tile digit histogram, stored digit-major: hist[d * n_tiles + tile].
__global__ void __launch_bounds__(RS_THREADS) k_rs_hist(const uint64_t* keys, int64_t n,
                                                        int shift, int64_t* hist, int n_tiles) {
    __shared__ int h[RS_BINS];
    for (int b = threadIdx.x; b < RS_BINS; b += RS_THREADS) h[b] = 0;
    __syncthreads();
    const int64_t base = static_cast<int64_t>(blockIdx.x) * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const int64_t i = base + r * RS_THREADS + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & (RS_BINS - 1)], 1);
    }
    __syncthreads();
    for (int b = threadIdx.x; b < RS_BINS; b += RS_THREADS)
        hist[static_cast<int64_t>(b) * n_tiles + blockIdx.x] = h[b];
}

// Stable scatter.  Within a tile keys are visited round by round (key r*256 + t in round r),
// so rank order is round, then wavefront, then lane: the original order.  Lanes of a
// wavefront holding the same digit are found with one ballot per digit bit.
__global__ void __launch_bounds__(RS_THREADS) k_rs_scatter(const uint64_t* keys_in,
                                                           const int32_t* vals_in,
                                                           uint64_t* keys_out,
                                                           int32_t* vals_out, int64_t n,
                                                           int shift, const int64_t* offs,
                                                           int n_tiles) {
    constexpr int WAVES = RS_THREADS / 64;
    __shared__ int64_t base_digit[RS_BINS];   // global start of each digit for this tile so far
    __shared__ int wave_cnt[WAVES][RS_BINS];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int b = threadIdx.x; b < RS_BINS; b += RS_THREADS)
        base_digit[b] = offs[static_cast<int64_t>(b) * n_tiles + blockIdx.x];
    const uint64_t below = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    const int64_t tile0 = static_cast<int64_t>(blockIdx.x) * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        for (int b = threadIdx.x; b < WAVES * RS_BINS; b += RS_THREADS)
            (&wave_cnt[0][0])[b] = 0;
        __syncthreads();
        const int64_t i = tile0 + r * RS_THREADS + threadIdx.x;
        const bool valid = i < n;
        const uint64_t key = valid ? keys_in[i] : 0;
        const int digit = static_cast<int>((key >> shift) & (RS_BINS - 1));
        uint64_t peers = __ballot(valid);
        for (int bit = 0; bit < 8; ++bit) {
            const uint64_t ones = __ballot(valid && ((digit >> bit) & 1));
            peers &= ((digit >> bit) & 1) ? ones : ~ones;
        }
        const int rank = __popcll(peers & below);
        if (valid && rank == 0) wave_cnt[wave][digit] = __popcll(peers);
        __syncthreads();
        // exclusive prefix over wavefronts for the digit of this key
        int64_t pos = 0;
        if (valid) {
            int before = 0;
            for (int w = 0; w < wave; ++w) before += wave_cnt[w][digit];
            pos = base_digit[digit] + before + rank;
        }
        __syncthreads();
        if (valid) {
            keys_out[pos] = key;
            vals_out[pos] = vals_in[i];
        }
        // advance the per-digit base by this round's totals
        for (int b = threadIdx.x; b < RS_BINS; b += RS_THREADS) {
            int tot = 0;
            for (int w = 0; w < WAVES; ++w) tot += wave_cnt[w][b];
            base_digit[b] += tot;
        }
        __syncthreads();
    }
}

}  // namespace

void scan_exclusive(const int64_t* in, int64_t* out, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_scan_excl, dim3(1), dim3(SCAN_THREADS), 0, s, in, out, n);
    LSPR_HIP(hipGetLastError());
}

void radix_sort_pairs(uint64_t* keys, int32_t* vals, int64_t n, int key_bits, hipStream_t s) {
    if (n <= 1) return;
    const int n_tiles = static_cast<int>((n + RS_TILE - 1) / RS_TILE);
    DevBuf<uint64_t> k2(n);
    DevBuf<int32_t> v2(n);
    DevBuf<int64_t> hist(static_cast<size_t>(RS_BINS) * n_tiles + 1);
    uint64_t* ka = keys;
    int32_t* va = vals;
    uint64_t* kb = k2.p;
    int32_t* vb = v2.p;
    const int passes = (key_bits + 7) / 8;
    for (int pass = 0; pass < passes; ++pass) {
        const int shift = 8 * pass;
        hipLaunchKernelGGL(k_rs_hist, dim3(n_tiles), dim3(RS_THREADS), 0, s, ka, n, shift,
                           hist.p, n_tiles);
        LSPR_HIP(hipGetLastError());
        scan_exclusive(hist.p, hist.p, static_cast<int64_t>(RS_BINS) * n_tiles, s);
        hipLaunchKernelGGL(k_rs_scatter, dim3(n_tiles), dim3(RS_THREADS), 0, s, ka, va, kb,
                           vb, n, shift, hist.p, n_tiles);
        LSPR_HIP(hipGetLastError());
        std::swap(ka, kb);
        std::swap(va, vb);
    }
    if (ka != keys) {
        LSPR_HIP(hipMemcpyAsync(keys, ka, n * sizeof(uint64_t), hipMemcpyDeviceToDevice, s));
        LSPR_HIP(hipMemcpyAsync(vals, va, n * sizeof(int32_t), hipMemcpyDeviceToDevice, s));
    }
    LSPR_HIP(hipStreamSynchronize(s));  // temporaries are freed on return
}

}  // namespace lspr
