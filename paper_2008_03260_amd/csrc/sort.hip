// Device LSD radix sort and exclusive scan.
//
// Each pass: (1) every tile of 8192 keys counts its digits in LDS, counts are
// stored digit-major; (2) an exclusive scan of the counts gives every
// (digit, tile) its output offset; (3) every tile ranks its keys stably (a
// wave ranks 64 keys at once by matching digits with ballots; waves own
// consecutive sub-tiles), stages them in LDS in digit order and writes each
// digit's run contiguously.  The scatter visits tiles in XCD-contiguous order
// so that the short runs that neighbouring tiles write for one digit meet in
// one L2.
//
// Two item forms.  The general form moves a uint32 key and a uint32 value
// (no global atomics: the output is deterministic).  The build's packed form
// (ids below 2^28, keys below 2^20) moves 6 bytes per item: the key's low 16
// bits in a uint16 array and a uint32 word holding key bits 16-19 above a
// 28-bit id; its first pass reads the hash keys with the ids implicit, and its
// last pass writes the ids alone plus each key's [start, end) run (a key
// changes between neighbours inside a tile's digit run: a plain store; at the
// edges of a run it may continue in another tile, so the edge items' keys are
// written to a side array and a small pass over the (digit, tile) runs
// compares each run's first and last key with its global neighbours), so no
// sorted keys are written and no pass over all items finds the runs.  No
// atomics: a Zipf head bucket spans thousands of tiles, and device-wide
// atomics on its two words serialised the pass.
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

// Input and output item forms of a scatter pass.
enum { IN_KV = 0, IN_KEYS = 1, IN_PACKED = 2 };    // key+value, keys (values = positions), packed
enum { OUT_KV = 0, OUT_PACKED = 1, OUT_IDS = 2 };  // key+value, packed, ids + key runs
constexpr uint32_t kIdBits = 28, kIdMask = (1u << kIdBits) - 1;

struct ScatterIO {
  const uint32_t* kin;  // IN_KV, IN_KEYS: keys
  const uint32_t* vin;  // IN_KV: values
  const uint16_t* lin;  // IN_PACKED: low key halves
  const uint32_t* win;  // IN_PACKED: words
  uint32_t* kout;       // OUT_KV: keys
  uint32_t* vout;       // OUT_KV: values; OUT_IDS: ids
  uint16_t* lout;       // OUT_PACKED: low key halves
  uint32_t* wout;       // OUT_PACKED: words
  uint32_t* start;      // OUT_IDS: first position of each key whose run starts inside a tile's digit run
  uint32_t* end;        // OUT_IDS: one past its last position, likewise
  uint32_t* edge;       // OUT_IDS: keys at the first and last position of every (digit, tile) run
};

__device__ __forceinline__ uint32_t packed_key(uint16_t lo, uint32_t w) { return (uint32_t)lo | ((w >> kIdBits) << 16); }

// Keys and values of one wave's sub-tile: every load is issued before any is
// used, unpredicated when the tile is full.
template <int IN>
__device__ __forceinline__ void load_subtile(const ScatterIO& io, uint64_t sbase, uint64_t n, bool full,
                                             uint32_t (&key)[kRounds], uint32_t (&val)[kRounds]) {
  const uint32_t lane = lane_id();
  if (IN == IN_PACKED) {
    uint16_t lo[kRounds];
    uint32_t w[kRounds];
    if (full) {
#pragma unroll
      for (int r = 0; r < kRounds; ++r) lo[r] = io.lin[sbase + (uint64_t)r * SL_WAVE + lane];
#pragma unroll
      for (int r = 0; r < kRounds; ++r) w[r] = io.win[sbase + (uint64_t)r * SL_WAVE + lane];
    } else {
#pragma unroll
      for (int r = 0; r < kRounds; ++r) {
        const uint64_t i = sbase + (uint64_t)r * SL_WAVE + lane;
        lo[r] = i < n ? io.lin[i] : (uint16_t)0;
        w[r] = i < n ? io.win[i] : 0u;
      }
    }
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      key[r] = packed_key(lo[r], w[r]);
      val[r] = w[r] & kIdMask;
    }
    return;
  }
  if (full) {
#pragma unroll
    for (int r = 0; r < kRounds; ++r) key[r] = io.kin[sbase + (uint64_t)r * SL_WAVE + lane];
    if (IN == IN_KV) {
#pragma unroll
      for (int r = 0; r < kRounds; ++r) val[r] = io.vin[sbase + (uint64_t)r * SL_WAVE + lane];
    }
  } else {
#pragma unroll
    for (int r = 0; r < kRounds; ++r) {
      const uint64_t i = sbase + (uint64_t)r * SL_WAVE + lane;
      key[r] = i < n ? io.kin[i] : 0u;
      if (IN == IN_KV) val[r] = i < n ? io.vin[i] : 0u;
    }
  }
  if (IN == IN_KEYS) {
#pragma unroll
    for (int r = 0; r < kRounds; ++r) val[r] = (uint32_t)(sbase + (uint64_t)r * SL_WAVE + lane);
  }
}

// Digit counts of one tile.  T = uint32_t: keys (HI: packed words, whose
// key bits 16-19 sit above the id); T = uint16_t: packed low key halves.
template <int BITS, typename T, bool HI>
__global__ void __launch_bounds__(kThreads)
    k_upsweep(const T* __restrict__ keys, uint64_t n, int shift, uint32_t* __restrict__ hist, uint32_t n_tiles) {
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
      k[j] = i < n ? (uint32_t)keys[i] : 0u;
    }
  }
  if (HI) {
#pragma unroll
    for (int j = 0; j < kItems; ++j) k[j] = (k[j] >> kIdBits) << 16;
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

template <int BITS, int IN, int OUT>
__global__ void __launch_bounds__(kThreads)
    k_downsweep(ScatterIO io, uint64_t n, int shift, const uint32_t* __restrict__ offs, uint32_t n_tiles) {
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
  load_subtile<IN>(io, sbase, n, full, key, val);
  // the tile's output offset per digit, in flight while the keys are ranked
  const uint32_t my_off = threadIdx.x < nd ? offs[(uint64_t)threadIdx.x * n_tiles + tile] : 0u;
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
    goff[threadIdx.x] = my_off - off;
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
    const uint32_t k = sk[p];
    const uint32_t d = (k >> shift) & dmask;
    const uint32_t g = goff[d] + p;
    if (OUT == OUT_KV) {
      io.kout[g] = k;
      io.vout[g] = sv[p];
    } else if (OUT == OUT_PACKED) {
      io.lout[g] = (uint16_t)k;
      io.wout[g] = ((k >> 16) << kIdBits) | sv[p];
    } else {
      io.vout[g] = sv[p];
      // inside the tile's run of digit d the key's neighbours are its global
      // neighbours; at the run's edges they lie in other tiles
      const bool first = p == 0 || ((sk[p - 1] >> shift) & dmask) != d;
      const bool last = p + 1 == tn || ((sk[p + 1] >> shift) & dmask) != d;
      if (first || last) io.edge[g] = k;
      if (!first && sk[p - 1] != k) io.start[k] = g;
      if (!last && sk[p + 1] != k) io.end[k] = g + 1;
    }
  }
}

// After the last scatter: every (digit, tile) run's first and last item
// decide their key's start and end when the item on their other side (the
// neighbouring run's edge item, or nothing) holds another key.  `offs` are
// the pass's scanned digit-major counts, so a run is [offs[e], offs[e + 1]).
__global__ void __launch_bounds__(256)
    k_run_edges(const uint32_t* __restrict__ offs, uint64_t n_runs, uint64_t n, const uint32_t* __restrict__ edge,
                uint32_t* __restrict__ start, uint32_t* __restrict__ end) {
  for (uint64_t e = blockIdx.x * (uint64_t)blockDim.x + threadIdx.x; e < n_runs;
       e += (uint64_t)gridDim.x * blockDim.x) {
    const uint32_t o = offs[e], o1 = e + 1 < n_runs ? offs[e + 1] : (uint32_t)n;
    if (o1 == o) continue;
    const uint32_t kf = edge[o], kl = edge[o1 - 1];
    if (o == 0 || edge[o - 1] != kf) start[kf] = o;
    if (o1 == n || edge[o1] != kl) end[kl] = o1;
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

template <typename T, bool HI>
const void* upsweep_fn(int bits) {
  switch (bits) {
    case 1: return (const void*)k_upsweep<1, T, HI>;
    case 2: return (const void*)k_upsweep<2, T, HI>;
    case 3: return (const void*)k_upsweep<3, T, HI>;
    case 4: return (const void*)k_upsweep<4, T, HI>;
    case 5: return (const void*)k_upsweep<5, T, HI>;
    case 6: return (const void*)k_upsweep<6, T, HI>;
    case 7: return (const void*)k_upsweep<7, T, HI>;
    default: return (const void*)k_upsweep<8, T, HI>;
  }
}

template <int IN, int OUT>
const void* downsweep_fn(int bits) {
  switch (bits) {
    case 1: return (const void*)k_downsweep<1, IN, OUT>;
    case 2: return (const void*)k_downsweep<2, IN, OUT>;
    case 3: return (const void*)k_downsweep<3, IN, OUT>;
    case 4: return (const void*)k_downsweep<4, IN, OUT>;
    case 5: return (const void*)k_downsweep<5, IN, OUT>;
    case 6: return (const void*)k_downsweep<6, IN, OUT>;
    case 7: return (const void*)k_downsweep<7, IN, OUT>;
    default: return (const void*)k_downsweep<8, IN, OUT>;
  }
}

// One pass: digit counts, their scan, the scatter.
template <typename T, bool HI>
hipError_t sort_pass(const T* ukeys, const void* down, const ScatterIO& io, uint64_t n, int shift, int bits,
                     uint32_t n_tiles, SortBuffers& b, hipStream_t st, PhaseTimer* timer) {
  typedef void (*UpFn)(const T*, uint64_t, int, uint32_t*, uint32_t);
  typedef void (*DownFn)(ScatterIO, uint64_t, int, const uint32_t*, uint32_t);
  const UpFn up = (UpFn)upsweep_fn<T, HI>(bits);
  const DownFn dn = (DownFn)down;
  if (timer) timer->begin(PH_UPSWEEP, st);
  hipLaunchKernelGGL(up, dim3(n_tiles), dim3(kThreads), 0, st, ukeys, n, shift, b.hist, n_tiles);
  if (timer) timer->end(PH_UPSWEEP, st);
  if (timer) timer->begin(PH_SCAN, st);
  hipError_t e = exclusive_scan(b.hist, (uint64_t)n_tiles << bits, b.part, st);
  if (timer) timer->end(PH_SCAN, st);
  if (e != hipSuccess) return e;
  if (timer) timer->begin(PH_DOWNSWEEP, st);
  hipLaunchKernelGGL(dn, dim3(n_tiles), dim3(kThreads), 0, st, io, n, shift, (const uint32_t*)b.hist, n_tiles);
  if (timer) timer->end(PH_DOWNSWEEP, st);
  return hipGetLastError();
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
      ScatterIO io{};
      io.kin = sk;
      io.vin = sv;
      io.kout = dk;
      io.vout = dv;
      const void* down = sv ? downsweep_fn<IN_KV, OUT_KV>(bits) : downsweep_fn<IN_KEYS, OUT_KV>(bits);
      hipError_t e = sort_pass<uint32_t, false>(sk, down, io, n, shift, bits, n_tiles, b, st, timer);
      if (e != hipSuccess) return e;
    }
    sk = dk;
    sv = dv;
  }
  *keys_out = dk;
  *vals_out = dv;
  return hipGetLastError();
}

bool packed_sort_ok(uint64_t n, int nbits) { return n <= (1ull << kIdBits) && nbits >= 1 && nbits <= 20; }

hipError_t radix_sort_runs(const uint32_t* keys_in, uint64_t n, int nbits, SortBuffers& b, uint32_t* start,
                           uint32_t* end, uint32_t** ids_out, hipStream_t st, PhaseTimer* timer) {
  if (!packed_sort_ok(n, nbits)) return hipErrorInvalidValue;
  const int passes = (nbits + 7) / 8;
  const uint32_t n_tiles = (uint32_t)((n + kTile - 1) / kTile);
  uint16_t* lo[2] = {(uint16_t*)b.k0, (uint16_t*)b.k1};
  uint32_t* w[2] = {b.v0, b.v1};
  // the last pass writes the ids over the low halves of its own parity and
  // the run-edge keys over its words, neither of which is its input
  uint32_t* ids = ((passes - 1) & 1) ? b.k1 : b.k0;
  uint32_t* edge = w[(passes - 1) & 1];
  if (n > 0) {
    for (int p = 0; p < passes; ++p) {
      const int shift = p * 8, bits = min(8, nbits - shift);
      const bool first = p == 0, last = p + 1 == passes;
      ScatterIO io{};
      io.kin = keys_in;
      io.lin = lo[(p + 1) & 1];
      io.win = w[(p + 1) & 1];
      io.lout = lo[p & 1];
      io.wout = w[p & 1];
      io.vout = ids;
      io.start = start;
      io.end = end;
      io.edge = edge;
      const void* down = first ? (last ? downsweep_fn<IN_KEYS, OUT_IDS>(bits) : downsweep_fn<IN_KEYS, OUT_PACKED>(bits))
                               : (last ? downsweep_fn<IN_PACKED, OUT_IDS>(bits) : downsweep_fn<IN_PACKED, OUT_PACKED>(bits));
      hipError_t e;
      if (first)
        e = sort_pass<uint32_t, false>(keys_in, down, io, n, shift, bits, n_tiles, b, st, timer);
      else if (shift + bits <= 16)
        e = sort_pass<uint16_t, false>(io.lin, down, io, n, shift, bits, n_tiles, b, st, timer);
      else
        e = sort_pass<uint32_t, true>(io.win, down, io, n, shift, bits, n_tiles, b, st, timer);
      if (e != hipSuccess) return e;
    }
    const int last_bits = nbits - 8 * (passes - 1);
    const uint64_t n_runs = (uint64_t)n_tiles << last_bits;
    if (timer) timer->begin(PH_BOUNDS, st);
    hipLaunchKernelGGL(k_run_edges, dim3((uint32_t)std::min<uint64_t>((n_runs + 255) / 256, 65536)), dim3(256), 0, st,
                       (const uint32_t*)b.hist, n_runs, n, (const uint32_t*)edge, start, end);
    if (timer) timer->end(PH_BOUNDS, st);
  }
  *ids_out = ids;
  return hipGetLastError();
}

}  // namespace slash
