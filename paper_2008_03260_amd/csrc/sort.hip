// Device LSD radix sort (key-value, uint32) and exclusive scan.
//
// Each pass: (1) every tile of 8192 keys counts its digits in LDS, counts are
// stored digit-major; (2) an exclusive scan of the counts gives every
// (digit, tile) its output offset; (3) every tile ranks its keys stably (a
// wave ranks 64 keys at once by matching digits with ballots; waves own
// consecutive sub-tiles), stages them in LDS in digit order and writes each
// digit's run contiguously.  No global atomics, so the output is
// deterministic.  The scatter visits tiles in XCD-contiguous order so that
// the short runs that neighbouring tiles write for one digit meet in one L2.
#include "slash_internal.h"

namespace slash {

namespace {

constexpr int kThreads = 512;
constexpr int kWaves = kThreads / SL_WAVE;
constexpr int kItems = 16;                 // per thread
constexpr int kTile = kThreads * kItems;   // 8192
constexpr int kSubTile = kTile / kWaves;   // 1024 per wave
constexpr int kRounds = kSubTile / SL_WAVE;
constexpr int kUpRounds = 1;  // digits counted with one atomic per wave before the per-lane atomics

__device__ __forceinline__ uint32_t wave_incl_scan(uint32_t v) {
  const uint32_t lane = lane_id();
#pragma unroll
  for (int o = 1; o < SL_WAVE; o <<= 1) {
    uint32_t y = __shfl_up(v, o, SL_WAVE);
    if (lane >= (uint32_t)o) v += y;
  }
  return v;
}

// Exclusive scan across the block of one value per thread; *total = sum.
__device__ __forceinline__ uint32_t block_excl_scan(uint32_t v, uint32_t* sh, uint32_t* total) {
  const uint32_t wave = threadIdx.x / SL_WAVE, lane = lane_id();
  uint32_t inc = wave_incl_scan(v);
  if (lane == SL_WAVE - 1) sh[wave] = inc;
  __syncthreads();
  uint32_t off = 0, tot = 0;
  for (int w = 0; w < kWaves; ++w) {
    uint32_t x = sh[w];
    if ((uint32_t)w < wave) off += x;
    tot += x;
  }
  __syncthreads();
  *total = tot;
  return off + inc - v;
}

// Keys (and values) of one wave's sub-tile: every load is issued before any
// is used, unpredicated when the tile is full.
template <bool WITH_VALS>
__device__ __forceinline__ void load_subtile(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin,
                                             uint64_t sbase, uint64_t n, bool full, uint32_t (&key)[kRounds],
                                             uint32_t (&val)[kRounds]) {
  const uint32_t lane = lane_id();
  if (full) {
#pragma unroll
    for (int r = 0; r < kRounds; ++r) key[r] = kin[sbase + (uint64_t)r * SL_WAVE + lane];
    if (WITH_VALS) {
#pragma unroll
      for (int r = 0; r < kRounds; ++r) val[r] = vin[sbase + (uint64_t)r * SL_WAVE + lane];
    }
  } else {
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const uint64_t i = sbase + (uint64_t)r * SL_WAVE + lane;
      key[r] = i < n ? kin[i] : 0u;
      if (WITH_VALS) val[r] = i < n ? vin[i] : 0u;
    }
  }
  if (!WITH_VALS) {
#pragma unroll
    for (int r = 0; r < kRounds; ++r) val[r] = (uint32_t)(sbase + (uint64_t)r * SL_WAVE + lane);
  }
}

template <int BITS>
__global__ void __launch_bounds__(kThreads)
    k_upsweep(const uint32_t* __restrict__ keys, uint64_t n, int shift, uint32_t* __restrict__ hist,
              uint32_t n_tiles) {
  __shared__ uint32_t cnt[256];
  constexpr uint32_t nd = 1u << BITS, dmask = nd - 1;
  for (uint32_t d = threadIdx.x; d < nd; d += kThreads) cnt[d] = 0;
  __syncthreads();
  const uint64_t base = (uint64_t)blockIdx.x * kTile;
  const uint32_t lane = lane_id();
  const bool full = base + kTile <= n;
  uint32_t k[kItems];
  if (full) {
#pragma unroll
    for (int j = 0; j < kItems; ++j) k[j] = keys[base + (uint64_t)j * kThreads + threadIdx.x];
  } else {
#pragma unroll
    for (int j = 0; j < kItems; ++j) {
      const uint64_t i = base + (uint64_t)j * kThreads + threadIdx.x;
      k[j] = i < n ? keys[i] : 0u;
    }
  }
  // Counts need no ranks: each key adds one with an LDS atomic.  Skewed
  // buckets make many lanes of a wave share a digit, and LDS atomics to one
  // address serialise, so the lanes sharing the digits of the first
  // kUpRounds remaining lanes add them with one atomic per digit first.
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    const bool v = full || base + (uint64_t)j * kThreads + threadIdx.x < n;
    const uint32_t d = (k[j] >> shift) & dmask;
    uint64_t rest = ballot64(v);
#pragma unroll
    for (int round = 0; round < kUpRounds; ++round) {
      if (rest == 0) break;
      const uint32_t first = (uint32_t)__builtin_ctzll(rest);
      const uint32_t d0 = __builtin_amdgcn_readlane(d, first);
      const uint64_t m = ballot64(((rest >> lane) & 1) && d == d0);
      if (lane == first) atomicAdd(&cnt[d0], (uint32_t)__builtin_popcountll(m));
      rest &= ~m;
    }
    if ((rest >> lane) & 1) atomicAdd(&cnt[d], 1u);
  }
  __syncthreads();
  for (uint32_t d = threadIdx.x; d < nd; d += kThreads) hist[(uint64_t)d * n_tiles + blockIdx.x] = cnt[d];
}

template <int BITS>
__global__ void __launch_bounds__(kThreads)
    k_downsweep(const uint32_t* __restrict__ kin, const uint32_t* __restrict__ vin, uint64_t n, int shift,
                const uint32_t* __restrict__ offs, uint32_t n_tiles, uint32_t* __restrict__ kout,
                uint32_t* __restrict__ vout) {
  __shared__ uint32_t wcnt[kWaves][256];
  __shared__ uint32_t tile_off[256];
  __shared__ uint32_t goff[256];  // output offset of the digit's run, minus its tile offset
  __shared__ uint32_t scan_sh[kWaves];
  __shared__ uint32_t sk[kTile];
  __shared__ uint32_t sv[kTile];
  constexpr uint32_t nd = 1u << BITS, dmask = nd - 1;
  const uint32_t wave = threadIdx.x / SL_WAVE, lane = lane_id();
  const uint32_t tile = xcd_tile(blockIdx.x, n_tiles);
  const uint64_t tbase = (uint64_t)tile * kTile;
  const uint64_t sbase = tbase + (uint64_t)wave * kSubTile;
  const bool full = tbase + kTile <= n;
  uint32_t key[kRounds], val[kRounds], loc[kRounds];
  if (vin)
    load_subtile<true>(kin, vin, sbase, n, full, key, val);
  else
    load_subtile<false>(kin, vin, sbase, n, full, key, val);
  for (uint32_t e = threadIdx.x; e < kWaves * 256; e += kThreads) (&wcnt[0][0])[e] = 0;
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    const bool v = full || sbase + (uint64_t)r * SL_WAVE + lane < n;
    uint32_t d = (key[r] >> shift) & dmask;
    uint64_t peers = match_digit(d, BITS, ballot64(v));
    uint32_t before = (uint32_t)__builtin_popcountll(peers & lanemask_lt());
    uint32_t b0 = v ? wcnt[wave][d] : 0u;
    wave_sync();
    if (v && lane == (uint32_t)__builtin_ctzll(peers)) wcnt[wave][d] = b0 + (uint32_t)__builtin_popcountll(peers);
    wave_sync();
    loc[r] = b0 + before;
  }
  __syncthreads();
  // per digit: prefix over waves, tile total, then tile offsets
  uint32_t tot_d = 0;
  if (threadIdx.x < 256) {
    uint32_t d = threadIdx.x;
    uint32_t acc = 0;
    for (int w = 0; w < kWaves; ++w) {
      uint32_t x = d < nd ? wcnt[w][d] : 0u;
      if (d < nd) wcnt[w][d] = acc;
      acc += x;
    }
    tot_d = acc;
  }
  uint32_t total;
  uint32_t off = block_excl_scan(tot_d, scan_sh, &total);
  if (threadIdx.x < nd) {
    tile_off[threadIdx.x] = off;
    goff[threadIdx.x] = offs[(uint64_t)threadIdx.x * n_tiles + tile] - off;
  }
  __syncthreads();
#pragma unroll
  for (int r = 0; r < kRounds; ++r) {
    if (full || sbase + (uint64_t)r * SL_WAVE + lane < n) {
      uint32_t d = (key[r] >> shift) & dmask;
      uint32_t p = tile_off[d] + wcnt[wave][d] + loc[r];
      sk[p] = key[r];
      sv[p] = val[r];
    }
  }
  __syncthreads();
  const uint32_t tn = (uint32_t)min((uint64_t)kTile, n - tbase);
  for (uint32_t p = threadIdx.x; p < tn; p += kThreads) {
    uint32_t k = sk[p];
    uint32_t d = (k >> shift) & dmask;
    uint32_t g = goff[d] + p;
    kout[g] = k;
    vout[g] = sv[p];
  }
}

// ----------------------------------------------------------------- scan

__global__ void __launch_bounds__(kThreads) k_scan_reduce(const uint32_t* __restrict__ d, uint64_t n,
                                                          uint32_t* __restrict__ part) {
  __shared__ uint32_t sh[kWaves];
  const uint64_t base = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kItems;
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j)
    if (base + j < n) s += d[base + j];
  uint32_t tot;
  block_excl_scan(s, sh, &tot);
  if (threadIdx.x == 0) part[blockIdx.x] = tot;
}

__global__ void __launch_bounds__(kThreads) k_scan_partials(uint32_t* part, uint32_t np) {
  __shared__ uint32_t sh[kWaves];
  uint32_t carry = 0;
  for (uint32_t b = 0; b < np; b += kThreads) {
    uint32_t i = b + threadIdx.x;
    uint32_t v = i < np ? part[i] : 0u;
    uint32_t tot;
    uint32_t ex = block_excl_scan(v, sh, &tot);
    if (i < np) part[i] = carry + ex;
    carry += tot;
  }
}

__global__ void __launch_bounds__(kThreads) k_scan_down(uint32_t* __restrict__ d, uint64_t n,
                                                        const uint32_t* __restrict__ part) {
  __shared__ uint32_t sh[kWaves];
  const uint64_t base = (uint64_t)blockIdx.x * kTile + (uint64_t)threadIdx.x * kItems;
  uint32_t v[kItems];
  uint32_t s = 0;
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    v[j] = base + j < n ? d[base + j] : 0u;
    s += v[j];
  }
  uint32_t tot;
  uint32_t ex = block_excl_scan(s, sh, &tot) + part[blockIdx.x];
#pragma unroll
  for (int j = 0; j < kItems; ++j) {
    if (base + j < n) d[base + j] = ex;
    ex += v[j];
  }
}

typedef void (*UpFn)(const uint32_t*, uint64_t, int, uint32_t*, uint32_t);
typedef void (*DownFn)(const uint32_t*, const uint32_t*, uint64_t, int, const uint32_t*, uint32_t, uint32_t*,
                       uint32_t*);

UpFn upsweep_fn(int bits) {
  switch (bits) {
    case 1: return k_upsweep<1>;
    case 2: return k_upsweep<2>;
    case 3: return k_upsweep<3>;
    case 4: return k_upsweep<4>;
    case 5: return k_upsweep<5>;
    case 6: return k_upsweep<6>;
    case 7: return k_upsweep<7>;
    default: return k_upsweep<8>;
  }
}

DownFn downsweep_fn(int bits) {
  switch (bits) {
    case 1: return k_downsweep<1>;
    case 2: return k_downsweep<2>;
    case 3: return k_downsweep<3>;
    case 4: return k_downsweep<4>;
    case 5: return k_downsweep<5>;
    case 6: return k_downsweep<6>;
    case 7: return k_downsweep<7>;
    default: return k_downsweep<8>;
  }
}

}  // namespace

size_t sort_hist_entries(uint64_t n) { return (size_t)256 * ((n + kTile - 1) / kTile) + 1; }
size_t sort_part_entries(uint64_t n) { return (size_t)((n + kTile - 1) / kTile) + 1; }

hipError_t exclusive_scan(uint32_t* data, uint64_t n, uint32_t* part, hipStream_t st) {
  if (n == 0) return hipSuccess;
  uint32_t nb = (uint32_t)((n + kTile - 1) / kTile);
  hipLaunchKernelGGL(k_scan_reduce, dim3(nb), dim3(kThreads), 0, st, data, n, part);
  hipLaunchKernelGGL(k_scan_partials, dim3(1), dim3(kThreads), 0, st, part, nb);
  hipLaunchKernelGGL(k_scan_down, dim3(nb), dim3(kThreads), 0, st, data, n, part);
  return hipGetLastError();
}

hipError_t radix_sort(const uint32_t* keys_in, const uint32_t* vals_in, uint64_t n, int nbits, SortBuffers& b,
                      uint32_t** keys_out, uint32_t** vals_out, hipStream_t st, PhaseTimer* timer) {
  const uint32_t* sk = keys_in;
  const uint32_t* sv = vals_in;
  if (nbits < 1) nbits = 1;
  const int passes = (nbits + 7) / 8;
  const uint32_t n_tiles = (uint32_t)((n + kTile - 1) / kTile);
  uint32_t *dk = b.k0, *dv = b.v0;
  for (int p = 0; p < passes; ++p) {
    int shift = p * 8;
    int bits = min(8, nbits - shift);
    dk = (p & 1) ? b.k1 : b.k0;
    dv = (p & 1) ? b.v1 : b.v0;
    if (n > 0) {
      if (timer) timer->begin(PH_UPSWEEP, st);
      hipLaunchKernelGGL(upsweep_fn(bits), dim3(n_tiles), dim3(kThreads), 0, st, sk, n, shift, b.hist, n_tiles);
      if (timer) timer->end(PH_UPSWEEP, st);
      if (timer) timer->begin(PH_SCAN, st);
      hipError_t e = exclusive_scan(b.hist, (uint64_t)n_tiles << bits, b.part, st);
      if (timer) timer->end(PH_SCAN, st);
      if (e != hipSuccess) return e;
      if (timer) timer->begin(PH_DOWNSWEEP, st);
      hipLaunchKernelGGL(downsweep_fn(bits), dim3(n_tiles), dim3(kThreads), 0, st, sk, sv, n, shift, b.hist, n_tiles,
                         dk, dv);
      if (timer) timer->end(PH_DOWNSWEEP, st);
    }
    sk = dk;
    sv = dv;
  }
  *keys_out = dk;
  *vals_out = dv;
  return hipGetLastError();
}

}  // namespace slash
