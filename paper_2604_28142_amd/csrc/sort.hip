// Device-wide building blocks: exclusive scan and stable LSD radix sort.
//
// The radix sort groups token vectors by token id (the per-token subproblems of
// Sect. 2.1) and orders rows by assigned centroid for the deterministic update
// sums.  It is the classic three-step counting sort per 8-bit digit:
// per-tile digit histograms, a digit-major exclusive scan over tiles, and a
// stable scatter in which each 64-wide wavefront ranks equal digits with eight
// ballots (lanes whose digits agree on every bit are peers).
#include "tac_internal.h"

namespace tac {

namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 8;
constexpr int kScanTile = kScanThreads * kScanItems;

constexpr int kSortThreads = 256;
constexpr int kSortWaves = kSortThreads / 64;
constexpr int kSortRounds = 16;  // 64-key rounds per wave
constexpr int kSortTile = kSortThreads * kSortRounds;

__device__ inline int64_t block_exclusive_scan(int64_t v, int64_t* lds, int64_t* total) {
    const int t = threadIdx.x;
    lds[t] = v;
    __syncthreads();
    for (int off = 1; off < kScanThreads; off <<= 1) {
        int64_t add = t >= off ? lds[t - off] : 0;
        __syncthreads();
        lds[t] += add;
        __syncthreads();
    }
    int64_t incl = lds[t];
    *total = lds[kScanThreads - 1];
    __syncthreads();
    return incl - v;
}

__global__ void __launch_bounds__(kScanThreads) scan_tile_sums(const int64_t* __restrict__ in, int64_t n,
                                                               int64_t* __restrict__ sums) {
    __shared__ int64_t lds[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t s = 0;
    for (int i = 0; i < kScanItems; ++i)
        if (base + i < n) s += in[base + i];
    int64_t total;
    block_exclusive_scan(s, lds, &total);
    if (threadIdx.x == 0) sums[blockIdx.x] = total;
}

// One block: exclusive scan of sums[0..nb) in place, sums[nb] = total.
__global__ void __launch_bounds__(kScanThreads) scan_partials(int64_t* __restrict__ sums, int64_t nb) {
    __shared__ int64_t lds[kScanThreads];
    int64_t carry = 0;
    for (int64_t base = 0; base < nb; base += kScanThreads) {
        const int64_t i = base + threadIdx.x;
        int64_t v = i < nb ? sums[i] : 0;
        int64_t total;
        int64_t ex = block_exclusive_scan(v, lds, &total);
        if (i < nb) sums[i] = carry + ex;
        carry += total;
    }
    if (threadIdx.x == 0) sums[nb] = carry;
}

__global__ void __launch_bounds__(kScanThreads) scan_tiles(const int64_t* in, int64_t* out, int64_t n,
                                                           const int64_t* __restrict__ sums, int64_t nb) {
    __shared__ int64_t lds[kScanThreads];
    const int64_t base = (int64_t)blockIdx.x * kScanTile + (int64_t)threadIdx.x * kScanItems;
    int64_t v[kScanItems];
    int64_t s = 0;
    for (int i = 0; i < kScanItems; ++i) {
        v[i] = base + i < n ? in[base + i] : 0;
        s += v[i];
    }
    int64_t total;
    int64_t run = sums[blockIdx.x] + block_exclusive_scan(s, lds, &total);
    for (int i = 0; i < kScanItems; ++i) {
        if (base + i < n) out[base + i] = run;
        run += v[i];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) out[n] = sums[nb];
}

__global__ void __launch_bounds__(kSortThreads) radix_hist(const uint32_t* __restrict__ keys, int64_t n, int shift,
                                                           int64_t* __restrict__ hist, int64_t nb) {
    __shared__ int cnt[256];
    cnt[threadIdx.x] = 0;
    __syncthreads();
    const int64_t tile = (int64_t)blockIdx.x * kSortTile;
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = tile + (int64_t)r * kSortThreads + threadIdx.x;
        if (i < n) atomicAdd(&cnt[(keys[i] >> shift) & 0xFFu], 1);
    }
    __syncthreads();
    hist[(int64_t)threadIdx.x * nb + blockIdx.x] = cnt[threadIdx.x];
}

// Lanes of the wavefront whose digit equals this lane's digit (among `valid` lanes).
__device__ inline uint64_t match_digit(uint32_t digit, bool valid) {
    uint64_t peers = __ballot(valid);
    for (int b = 0; b < 8; ++b) {
        const bool bit = (digit >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
    }
    return peers;
}

__global__ void __launch_bounds__(kSortThreads) radix_scatter(const uint32_t* __restrict__ kin,
                                                              const int32_t* __restrict__ vin, int64_t n, int shift,
                                                              const int64_t* __restrict__ off, int64_t nb,
                                                              uint32_t* __restrict__ kout,
                                                              int32_t* __restrict__ vout) {
    __shared__ int64_t wbase[kSortWaves][256];
    __shared__ int wcnt[kSortWaves][256];
    const int lane = threadIdx.x & 63;
    const int wave = threadIdx.x >> 6;
    for (int i = threadIdx.x; i < kSortWaves * 256; i += kSortThreads) (&wcnt[0][0])[i] = 0;
    __syncthreads();

    const int64_t base = (int64_t)blockIdx.x * kSortTile + (int64_t)wave * (kSortRounds * 64);
    const uint64_t lt = (1ull << lane) - 1ull;
    uint32_t key[kSortRounds];
    int32_t val[kSortRounds];
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = base + (int64_t)r * 64 + lane;
        const bool valid = i < n;
        key[r] = valid ? kin[i] : 0u;
        val[r] = valid ? (vin ? vin[i] : (int32_t)i) : 0;
        const uint32_t d = (key[r] >> shift) & 0xFFu;
        const uint64_t peers = match_digit(d, valid);
        if (valid && (peers & lt) == 0) wcnt[wave][d] += __popcll(peers);
    }
    __syncthreads();
    {
        const int d = threadIdx.x;  // one digit per thread
        int64_t run = off[(int64_t)d * nb + blockIdx.x];
        for (int w = 0; w < kSortWaves; ++w) {
            wbase[w][d] = run;
            run += wcnt[w][d];
        }
    }
    __syncthreads();
    for (int r = 0; r < kSortRounds; ++r) {
        const int64_t i = base + (int64_t)r * 64 + lane;
        const bool valid = i < n;
        const uint32_t d = (key[r] >> shift) & 0xFFu;
        const uint64_t peers = match_digit(d, valid);
        if (valid) {
            const int64_t pos = wbase[wave][d] + __popcll(peers & lt);
            kout[pos] = key[r];
            vout[pos] = val[r];
        }
        __builtin_amdgcn_wave_barrier();
        if (valid && (peers & lt) == 0) wbase[wave][d] += __popcll(peers);
        __builtin_amdgcn_wave_barrier();
    }
}

}  // namespace

size_t scan_scratch_bytes(int64_t n) {
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    return (size_t)(nb + 1) * sizeof(int64_t);
}

tac_status exclusive_scan_i64(hipStream_t s, const int64_t* in, int64_t* out, int64_t n, void* scratch) {
    int64_t* sums = static_cast<int64_t*>(scratch);
    const int64_t nb = (n + kScanTile - 1) / kScanTile;
    if (nb > 0) {
        scan_tile_sums<<<dim3((unsigned)nb), dim3(kScanThreads), 0, s>>>(in, n, sums);
        TAC_LAUNCH_CHECK("scan_tile_sums");
    }
    scan_partials<<<1, kScanThreads, 0, s>>>(sums, nb);
    TAC_LAUNCH_CHECK("scan_partials");
    scan_tiles<<<dim3((unsigned)(nb > 0 ? nb : 1)), dim3(kScanThreads), 0, s>>>(in, out, n, sums, nb);
    TAC_LAUNCH_CHECK("scan_tiles");
    return TAC_OK;
}

size_t radix_sort_scratch_bytes(int64_t n) {
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    const int64_t hist = 256 * nb;
    return ((size_t)(hist + 1) * sizeof(int64_t) + 255) / 256 * 256 + scan_scratch_bytes(hist);
}

tac_status radix_sort(hipStream_t s, int64_t n, int bits, uint32_t* k0, int32_t* v0, uint32_t* k1, int32_t* v1,
                      const int32_t* vals_in, void* scratch, int* result_in_1) {
    *result_in_1 = 0;
    if (n <= 0) return TAC_OK;
    const int64_t nb = (n + kSortTile - 1) / kSortTile;
    int64_t* hist = static_cast<int64_t*>(scratch);
    // hist holds 256 * nb counts plus the total the scan writes after them
    void* scan_scr = static_cast<char*>(scratch) + ((size_t)(256 * nb + 1) * sizeof(int64_t) + 255) / 256 * 256;
    const int passes = bits <= 0 ? 1 : (bits + 7) / 8;
    const uint32_t* kin = k0;
    const int32_t* vin = vals_in;
    int cur = 0;
    for (int p = 0; p < passes; ++p) {
        uint32_t* kout = cur == 0 ? k1 : k0;
        int32_t* vout = cur == 0 ? v1 : v0;
        radix_hist<<<dim3((unsigned)nb), dim3(kSortThreads), 0, s>>>(kin, n, 8 * p, hist, nb);
        TAC_LAUNCH_CHECK("radix_hist");
        tac_status st = exclusive_scan_i64(s, hist, hist, 256 * nb, scan_scr);
        if (st != TAC_OK) return st;
        radix_scatter<<<dim3((unsigned)nb), dim3(kSortThreads), 0, s>>>(kin, vin, n, 8 * p, hist, nb, kout, vout);
        TAC_LAUNCH_CHECK("radix_scatter");
        kin = kout;
        vin = vout;
        cur ^= 1;
    }
    *result_in_1 = cur;
    return TAC_OK;
}

}  // namespace tac
