// Device-wide primitives of the MPI build: single-pass exclusive scans, a stable LSD radix
// sort of (u32 key, u32 value) pairs, and a fill kernel.  Every launch has a host-fixed grid;
// data dependent lengths are read from device memory, so nothing here waits on the host.
#include "sort_internal.h"
#include "lds_sync.h"

namespace lf {
namespace {

// ---------------------------------------------------------------------------------------
// Look-back status words: a flag in the top two bits, a count below.  They are read and
// written with device-scope atomics, so every XCD sees one coherent value; a flag and its
// count travel in one word, which is why relaxed ordering suffices.
// ---------------------------------------------------------------------------------------
constexpr uint64_t kStAgg = 1ull << 62;   // the work-group's own aggregate
constexpr uint64_t kStPre = 2ull << 62;   // inclusive prefix through the work-group
constexpr uint64_t kStVal = kStAgg - 1;
constexpr int kSpinLimit = 1 << 18;       // polls before a wait gives up (about 0.1-0.3 s)

// Exclusive scan of one u32 per thread over a work-group of NW waves: wave scans by
// shuffles, then the wave totals (LDS scratch `wt`).  *total = the work-group's sum.
template <int NW>
__device__ __forceinline__ uint32_t block_scan_u32(uint32_t v, uint32_t* wt, uint32_t* total) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  uint32_t x = v;
#pragma unroll
  for (int off = 1; off < 64; off <<= 1) {
    const uint32_t y = __shfl_up(x, off, 64);
    if (lane >= off) x += y;
  }
  if (lane == 63) wt[wave] = x;
  lds_barrier();
  uint32_t before = 0, sum = 0;
#pragma unroll
  for (int w = 0; w < NW; ++w) {
    const uint32_t t = wt[w];
    before += w < wave ? t : 0u;
    sum += t;
  }
  *total = sum;
  lds_barrier();                                           // wt is free again
  return before + x - v;
}

__device__ __forceinline__ uint64_t load_status(const uint64_t* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_status(uint64_t* p, uint64_t v) {
  __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Wait for a predecessor's status.  On the bound: *err is raised and an empty prefix is
// returned, which ends the walk (the results are then wrong, but each stays at or below
// its true value, so every index derived from them stays in range).
__device__ uint64_t wait_status(const uint64_t* p, uint32_t* err) {
  for (int i = 0; i < kSpinLimit; ++i) {
    const uint64_t v = load_status(p);
    if (v & (kStAgg | kStPre)) return v;
    __builtin_amdgcn_s_sleep(2);
  }
  atomicOr(err, 1u);
  return kStPre;
}

// h[d] += 1 for each active lane.  When the whole wave holds one digit (long runs of equal
// high digits are common) one lane adds the count: same-address LDS atomics serialise.
__device__ __forceinline__ void count_digit(uint32_t* h, uint32_t d) {
  const uint64_t act = __ballot(true);
  const uint32_t d0 = __builtin_amdgcn_readfirstlane(d);
  if (__ballot(d == d0) == act) {
    if ((threadIdx.x & 63) == __builtin_ctzll(act)) atomicAdd(&h[d0], (uint32_t)__popcll(act));
  } else {
    atomicAdd(&h[d], 1u);
  }
}

// Exclusive prefix of one (work-group j, digit d) over the work-groups before j, from
// status words status[k * stride + d].  G consecutive lanes share the digit and each holds
// U predecessors of a window of G U (lane g: k - g U - u), so one step covers G U
// work-groups: the walk stops at the nearest published inclusive prefix.
template <int G, int U>
__device__ uint64_t look_back(const uint64_t* status, int64_t stride, int64_t j, int d, int g, uint32_t* err) {
  uint64_t excl = 0;
  for (int64_t k = j - 1;; k -= G * U) {
    uint64_t w[U];
#pragma unroll
    for (int u = 0; u < U; ++u) {
      const int64_t q = k - (int64_t)g * U - u;
      w[u] = q >= 0 ? load_status(status + q * stride + d) : kStPre;
    }
    int near = G * U;                 // window position of the nearest inclusive prefix
#pragma unroll
    for (int u = U - 1; u >= 0; --u) {
      if (!(w[u] & (kStAgg | kStPre))) w[u] = wait_status(status + (k - (int64_t)g * U - u) * stride + d, err);
      if (w[u] & kStPre) near = g * U + u;
    }
#pragma unroll
    for (int off = 1; off < G; off <<= 1) near = min(near, __shfl_xor(near, off, 64));
    uint64_t x = 0;
#pragma unroll
    for (int u = 0; u < U; ++u)
      if (g * U + u <= near) x += w[u] & kStVal;
#pragma unroll
    for (int off = 1; off < G; off <<= 1) x += __shfl_xor(x, off, 64);
    excl += x;
    if (near < G * U) return excl;
  }
}

// ---------------------------------------------------------------------------------------
// Scans
// ---------------------------------------------------------------------------------------
constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanChunk = kScanThreads * kScanItems;   // elements per work-group

// Exclusive scan of one value per thread (Hillis-Steele in LDS); *total = the block sum.
template <typename T>
__device__ T block_exclusive_scan(T v, T* sh, T* total) {
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    const T add = tid >= off ? sh[tid - off] : T(0);
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  const T incl = sh[tid];
  *total = sh[kScanThreads - 1];
  __syncthreads();
  return incl - v;
}

// Work-group j scans [j kScanChunk, (j + 1) kScanChunk).  PAIR scans two u32 arrays at once
// as a[i] | b[i] << 32 (no carry crosses bit 32 while a's total < 2^32).  state[1 + j] is
// the status of work-group j (state[0] is unused).
template <bool PAIR>
__global__ __launch_bounds__(kScanThreads) void scan_onepass(const uint64_t* in, uint64_t* out, const uint32_t* a,
                                                             uint32_t* oa, const uint32_t* b, uint32_t* ob,
                                                             int64_t n, uint64_t* state, uint32_t* err,
                                                             uint32_t* heads, int64_t n_heads, int head_shift) {
  __shared__ uint64_t sh[kScanThreads];
  __shared__ uint64_t s_excl;
  const int tid = threadIdx.x;
  const int64_t j = blockIdx.x;
  uint64_t* st = state + 1;
  const int64_t base = j * kScanChunk + (int64_t)tid * kScanItems;
  uint64_t v[kScanItems];
  uint64_t sum = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t e = base + i;
    if (PAIR) v[i] = e < n ? ((uint64_t)a[e] | ((uint64_t)b[e] << 32)) : 0ull;
    else v[i] = e < n ? in[e] : 0ull;
    sum += v[i];
  }
  uint64_t total;
  uint64_t run = block_exclusive_scan<uint64_t>(sum, sh, &total);
  if (tid < 64) {
    // wave 0 publishes and looks back 64 predecessors at a time (lane i: work-group k - i)
    uint64_t excl = 0;
    if (j > 0) {
      if (tid == 0) store_status(st + j, kStAgg | total);
      for (int64_t k = j - 1;; k -= 64) {
        const int64_t q = k - tid;
        const uint64_t w = q >= 0 ? wait_status(st + q, err) : kStPre;
        const uint64_t pm = __ballot((w & kStPre) != 0);
        const int stop = pm ? __builtin_ctzll(pm) : 63;     // nearest published prefix
        uint64_t x = tid <= stop ? (w & kStVal) : 0ull;
        for (int off = 32; off > 0; off >>= 1) x += __shfl_xor(x, off, 64);
        excl += x;
        if (pm) break;
      }
    }
    if (tid == 0) {
      store_status(st + j, kStPre | (excl + total));
      s_excl = excl;
    }
  }
  __syncthreads();
  run += s_excl;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t e = base + i;
    if (e < n) {
      if (PAIR) {
        oa[e] = (uint32_t)run;
        ob[e] = (uint32_t)(run >> 32);
      } else {
        out[e] = run;
        if (heads && v[i] > 0) {
          // the element holds the outputs [run, run + v): it heads every multiple of
          // 2^head_shift among them
          const uint64_t end = run + v[i];
          for (uint64_t h = (run + ((1ull << head_shift) - 1)) >> head_shift;
               (h << head_shift) < end && (int64_t)h < n_heads; ++h)
            heads[h] = (uint32_t)e;
        }
      }
    }
    run += v[i];
  }
  if (j == (int64_t)gridDim.x - 1 && tid == 0) {
    const uint64_t grand = s_excl + total;
    if (PAIR) {
      oa[n] = (uint32_t)grand;
      ob[n] = (uint32_t)(grand >> 32);
    } else {
      out[n] = grand;
    }
  }
}

// ---------------------------------------------------------------------------------------
// Radix sort.  One histogram launch counts the digits of every pass; then each pass is one
// launch: work-group j sorts the span [j span, (j + 1) span) of the current
// order, span = ceil(n / (P 256)) 256 with n read from device memory.  The output position
// of an element = (elements of smaller digits) + (elements of its digit in earlier spans,
// from the look-back over per-(span, digit) status words) + (its rank in its own span).
// ---------------------------------------------------------------------------------------
constexpr int kRadixThreads = 512;
constexpr int kWaves = kRadixThreads / 64;
constexpr int kMaxPasses = 8;
constexpr int kHistPerBlock = 4096;
constexpr int kItems = 8;                           // elements per thread loaded together
constexpr int kChunk = kItems * kRadixThreads;
constexpr int kHistBlocksMax = 256;

__device__ __forceinline__ int64_t sort_len(const int64_t* n_dev, int64_t cap) {
  const int64_t n = n_dev ? *n_dev : cap;
  return n < 0 ? 0 : (n < cap ? n : cap);
}

__device__ __forceinline__ int64_t block_span(int64_t n, int64_t blocks) {
  const int64_t per = (n + blocks * kRadixThreads - 1) / (blocks * kRadixThreads);
  return per * kRadixThreads;
}

// Digit totals of every pass (ghist[p R + d] += count), and zeroing of the passes' status
// words (`clear`, nclear u64) for the launches that follow.
template <int BITS>
__global__ __launch_bounds__(kRadixThreads) void radix_histogram(const uint32_t* keys, const int64_t* n_dev,
                                                                 int64_t cap, int lo_bit, int bits, uint32_t* ghist,
                                                                 uint64_t* clear, int64_t nclear) {
  constexpr int R = 1 << BITS;
  constexpr int NP = (32 + BITS - 1) / BITS;
  __shared__ uint32_t h[NP * R];
  const int npass = (bits + BITS - 1) / BITS;
  const int tid = threadIdx.x;
  for (int i = tid; i < npass * R; i += kRadixThreads) h[i] = 0;
  for (int64_t i = (int64_t)blockIdx.x * kRadixThreads + tid; i < nclear; i += (int64_t)gridDim.x * kRadixThreads)
    clear[i] = 0ull;
  __syncthreads();
  const int64_t n = sort_len(n_dev, cap);
  const int64_t span = block_span(n, gridDim.x);
  const int64_t b0 = min(n, (int64_t)blockIdx.x * span);
  const int64_t b1 = min(n, b0 + span);
  for (int64_t c0 = b0; c0 < b1; c0 += kChunk) {
    uint32_t kk[kItems];
#pragma unroll
    for (int i = 0; i < kItems; ++i) {     // every load of the chunk in flight at once
      const int64_t e = c0 + i * kRadixThreads + tid;
      kk[i] = e < b1 ? keys[e] : 0u;
    }
#pragma unroll
    for (int i = 0; i < kItems; ++i) {
      if (c0 + i * kRadixThreads + tid >= b1) break;
      for (int p = 0; p < npass; ++p) {
        const int sh = lo_bit + p * BITS;
        const int w = min(BITS, lo_bit + bits - sh);
        count_digit(h + p * R, (kk[i] >> sh) & ((1u << w) - 1u));
      }
    }
  }
  __syncthreads();
  for (int i = tid; i < npass * R; i += kRadixThreads)
    if (h[i]) atomicAdd(&ghist[i], h[i]);
}

template <int BITS>
__global__ __launch_bounds__(kRadixThreads) void radix_onesweep(const uint32_t* keys_in, const uint32_t* vals_in,
                                                                uint32_t* keys_out, uint32_t* vals_out,
                                                                const int64_t* n_dev, int64_t cap, int shift,
                                                                uint32_t mask, const uint32_t* ghist,
                                                                uint64_t* status, uint32_t* err) {
  constexpr int R = 1 << BITS;
  constexpr int PER = R >= kRadixThreads ? R / kRadixThreads : 1;
  // elements per thread and per chunk: wide digits get longer chunks, so that each digit's
  // run of a chunk (about CH / R elements) still fills part of a cache line
  constexpr int IT = BITS >= 10 ? 2 * kItems : kItems;
  constexpr int CH = IT * kRadixThreads;
  __shared__ uint32_t hist[R];            // this span's digit counts
  __shared__ uint32_t running[R];         // output position of the next element of each digit
  __shared__ uint32_t wcount[kWaves][R];  // per-wave digit counts of a chunk, then offsets
  __shared__ uint32_t lstart[R + 1];      // digit starts inside the chunk's LDS copy
  __shared__ uint32_t s_key[CH];
  __shared__ uint32_t s_val[CH];
  __shared__ uint32_t wt[kWaves];
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  for (int d = tid; d < R; d += kRadixThreads) {
    hist[d] = 0;
    for (int w = 0; w < kWaves; ++w) wcount[w][d] = 0;
  }
  __syncthreads();
  const int64_t j = blockIdx.x;
  const int64_t n = sort_len(n_dev, cap);
  const int64_t span = block_span(n, gridDim.x);
  const int64_t b0 = min(n, j * span);
  const int64_t b1 = min(n, b0 + span);
  // Spans are filled in order, so an empty span has only empty successors, and no
  // one waits on it.
  if (b0 >= b1) return;
  for (int64_t c0 = b0; c0 < b1; c0 += CH) {
    uint32_t kk[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int64_t e = c0 + i * kRadixThreads + tid;
      kk[i] = e < b1 ? keys_in[e] : 0u;
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      if (c0 + i * kRadixThreads + tid >= b1) break;
      count_digit(hist, (kk[i] >> shift) & mask);
    }
  }
  // digit starts: exclusive scan of the pass's digit totals, PER digits per thread (the
  // scan's barriers also close the counting)
  {
    uint32_t loc[PER];
    uint32_t s = 0;
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int d = tid * PER + i;
      loc[i] = d < R ? ghist[d] : 0u;
      s += loc[i];
    }
    uint32_t total;
    uint32_t run = block_scan_u32<kWaves>(s, wt, &total);
#pragma unroll
    for (int i = 0; i < PER; ++i) {
      const int d = tid * PER + i;
      if (d < R) running[d] = run;
      run += loc[i];
    }
  }
  lds_barrier();   // (for R > 256 the loop below gives a digit to another thread)
  // publish this span's digit counts, then add up the earlier spans' counts: G threads per
  // digit (R <= 256), or digits in rounds of 256 with one thread each
  constexpr int G = R >= kRadixThreads ? 1 : kRadixThreads / R;
  constexpr int U = G >= 2 ? 8 : 16;
  for (int d0 = 0; d0 < R; d0 += kRadixThreads / G) {
    const int d = d0 + tid / G, g = tid % G;
    const uint32_t c = hist[d];
    uint64_t* mine = status + (size_t)j * R + d;
    if (g == 0) store_status(mine, (j == 0 ? kStPre : kStAgg) | c);
    const uint64_t excl = j == 0 ? 0ull : look_back<G, U>(status, R, j, d, g, err);
    if (g == 0) {
      if (j > 0) store_status(mine, kStPre | (excl + c));
      running[d] += (uint32_t)excl;
    }
  }
  lds_barrier();
  // Scatter, a chunk of CH elements at a time.  Wave w takes the chunk's w-th quarter
  // (contiguous, so waves in order and items in order within a wave is element order:
  // stable) and ranks its items one after another against its own digit counters (one
  // wave's LDS operations complete in order: no barrier between items).  The chunk is then
  // reordered by digit in LDS, so the global writes of each digit's run are contiguous.
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int64_t c0 = b0; c0 < b1; c0 += CH) {
    const int clen = (int)min((int64_t)CH, b1 - c0);
    const int64_t wb = c0 + (int64_t)wave * (IT * 64) + lane;
    uint32_t kk[IT], vv[IT], rk[IT];
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const int64_t e = wb + i * 64;
      kk[i] = e < b1 ? keys_in[e] : 0u;
      vv[i] = e < b1 ? vals_in[e] : 0u;
    }
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      const bool valid = wb + i * 64 < b1;
      const uint32_t d = valid ? (kk[i] >> shift) & mask : 0u;
      // lanes of this wave holding the same digit
      uint64_t peers = __ballot(valid);
#pragma unroll
      for (int b = 0; b < BITS; ++b) {
        const bool bit = (d >> b) & 1u;
        const uint64_t m = __ballot(bit);
        peers &= bit ? m : ~m;
      }
      const uint32_t before = wcount[wave][d];
      const uint32_t rank = __popcll(peers & lt);
      rk[i] = before + rank;
      if (valid && rank == 0) wcount[wave][d] = before + (uint32_t)__popcll(peers);
    }
    lds_barrier();
    {
      // per digit: the waves' counts become offsets; the chunk's digit starts by a scan
      uint32_t cnt[PER];
      uint32_t s = 0;
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int d = tid * PER + q;
        uint32_t c = 0;
        if (d < R) {
#pragma unroll
          for (int w = 0; w < kWaves; ++w) {
            const uint32_t t = wcount[w][d];
            wcount[w][d] = c;
            c += t;
          }
        }
        cnt[q] = c;
        s += c;
      }
      uint32_t tot;
      uint32_t run = block_scan_u32<kWaves>(s, wt, &tot);
#pragma unroll
      for (int q = 0; q < PER; ++q) {
        const int d = tid * PER + q;
        if (d < R) lstart[d] = run;
        run += cnt[q];
      }
      if (tid == 0) lstart[R] = tot;
    }
    lds_barrier();
#pragma unroll
    for (int i = 0; i < IT; ++i) {
      if (wb + i * 64 < b1) {
        const uint32_t d = (kk[i] >> shift) & mask;
        const uint32_t lp = lstart[d] + wcount[wave][d] + rk[i];
        s_key[lp] = kk[i];
        s_val[lp] = vv[i];
      }
    }
    lds_barrier();
    for (int idx = tid; idx < clen; idx += kRadixThreads) {
      const uint32_t key = s_key[idx];
      const uint32_t d = (key >> shift) & mask;
      const uint32_t pos = running[d] + ((uint32_t)idx - lstart[d]);
      keys_out[pos] = key;
      vals_out[pos] = s_val[idx];
    }
    lds_barrier();
    for (int d = tid; d < R; d += kRadixThreads) {
      running[d] += lstart[d + 1] - lstart[d];
#pragma unroll
      for (int w = 0; w < kWaves; ++w) wcount[w][d] = 0;
    }
    lds_barrier();
  }
}

__global__ void fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

// ---- scans ----------------------------------------------------------------------------
size_t scan_state_words(int64_t n) { return (size_t)((n + kScanChunk - 1) / kScanChunk) + 1; }

static hipError_t scan_launch(bool pair, const uint64_t* in, uint64_t* out, const uint32_t* a, uint32_t* oa,
                              const uint32_t* b, uint32_t* ob, int64_t n, uint64_t* state, uint32_t* err,
                              uint32_t* heads, int64_t n_heads, int head_shift, hipStream_t s) {
  if (n < 0 || !state || !err) return hipErrorInvalidValue;
  if (n == 0) {
    // totals only
    if (pair) {
      hipLaunchKernelGGL(fill_u32, dim3(1), dim3(1), 0, s, oa, (int64_t)1, 0u);
      hipLaunchKernelGGL(fill_u32, dim3(1), dim3(1), 0, s, ob, (int64_t)1, 0u);
    } else {
      hipLaunchKernelGGL(fill_u32, dim3(1), dim3(2), 0, s, reinterpret_cast<uint32_t*>(out), (int64_t)2, 0u);
    }
    return hipGetLastError();
  }
  const int64_t nb = (n + kScanChunk - 1) / kScanChunk;
  if (nb > (1LL << 31)) return hipErrorInvalidValue;
  if (pair)
    hipLaunchKernelGGL(scan_onepass<true>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, nullptr, nullptr, a, oa, b,
                       ob, n, state, err, nullptr, (int64_t)0, 0);
  else
    hipLaunchKernelGGL(scan_onepass<false>, dim3((unsigned)nb), dim3(kScanThreads), 0, s, in, out, nullptr, nullptr,
                       nullptr, nullptr, n, state, err, heads, n_heads, head_shift);
  return hipGetLastError();
}

hipError_t exclusive_scan_u64(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* state, uint32_t* err,
                              hipStream_t s, uint32_t* heads, int64_t n_heads, int head_shift) {
  if (heads && (head_shift < 0 || head_shift > 40)) return hipErrorInvalidValue;
  return scan_launch(false, in, out, nullptr, nullptr, nullptr, nullptr, n, state, err, heads, n_heads, head_shift, s);
}

hipError_t exclusive_scan_pair_u32(const uint32_t* a, uint32_t* oa, const uint32_t* b, uint32_t* ob, int64_t n,
                                   uint64_t* state, uint32_t* err, hipStream_t s) {
  return scan_launch(true, nullptr, nullptr, a, oa, b, ob, n, state, err, nullptr, 0, 0, s);
}

// ---- radix sort -----------------------------------------------------------------------
// About 4096 elements per work-group and at most 512 work-groups, so the look-back
// traffic (digits x predecessors visited) stays small; the status words of one pass
// (2^digit_bits * work-groups) are kept to 2^18.
constexpr int64_t kMaxStatus = 1 << 18;
constexpr int64_t kSpanTarget = 4096;
constexpr int64_t kMaxRadixBlocks = 512;
constexpr int kMinDigitBits = 4, kMaxDigitBits = 11;

int radix_blocks(int64_t cap, int digit_bits) {
  int64_t b = (cap + kSpanTarget - 1) / kSpanTarget;
  int64_t lim = kMaxStatus >> digit_bits;
  if (lim > kMaxRadixBlocks) lim = kMaxRadixBlocks;
  if (b > lim) b = lim;
  return (int)(b < 1 ? 1 : b);
}

int radix_passes(int bits, int max_digit_bits) { return bits < 1 ? 0 : (bits + max_digit_bits - 1) / max_digit_bits; }

int radix_digit_bits(int bits, int max_digit_bits) {
  const int np = radix_passes(bits, max_digit_bits);
  return np ? (bits + np - 1) / np : 0;
}

int radix_hist_words(int bits, int max_digit_bits) {
  return radix_passes(bits, max_digit_bits) << radix_digit_bits(bits, max_digit_bits);
}

size_t radix_tmp_u32(int64_t cap) {
  // the status words of every pass, for the widest layout any digit width needs
  int64_t most = 0;
  for (int d = kMinDigitBits; d <= kMaxDigitBits; ++d) {
    const int64_t w = (int64_t)radix_passes(32, d) * radix_blocks(cap, d) * ((int64_t)1 << d);
    if (w > most) most = w;
  }
  return (size_t)(2 * most);
}

hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, int64_t cap,
                            const int64_t* n_dev, int lo_bit, int bits, uint32_t* tmp, uint32_t* ghist,
                            uint32_t* err, int* result_in_alt, hipStream_t s, int max_digit_bits) {
  if (bits < 1 || lo_bit < 0 || lo_bit + bits > 32) return hipErrorInvalidValue;
  if (max_digit_bits < kMinDigitBits || max_digit_bits > kMaxDigitBits) return hipErrorInvalidValue;
  if (cap < 0 || cap >= (1LL << 31) || !tmp || !ghist || !err) return hipErrorInvalidValue;
  const int npass = radix_passes(bits, max_digit_bits);
  const int dbits = radix_digit_bits(bits, max_digit_bits);
  if (npass > kMaxPasses) return hipErrorInvalidValue;
  const int P = radix_blocks(cap, dbits);
  const int64_t R = 1LL << dbits;
  uint64_t* status = reinterpret_cast<uint64_t*>(tmp);
  const int64_t nclear = (int64_t)npass * P * R;
  const int64_t hb = (cap + kHistPerBlock - 1) / kHistPerBlock;
  const unsigned H = (unsigned)(hb < 1 ? 1 : (hb > kHistBlocksMax ? kHistBlocksMax : hb));
  switch (dbits) {
#define LF_RADIX_HIST(B) case B: hipLaunchKernelGGL(radix_histogram<B>, dim3(H), dim3(kRadixThreads), 0, s, keys, n_dev, cap, lo_bit, bits, ghist, status, nclear); break;
    LF_RADIX_HIST(4) LF_RADIX_HIST(5) LF_RADIX_HIST(6) LF_RADIX_HIST(7) LF_RADIX_HIST(8) LF_RADIX_HIST(9)
    LF_RADIX_HIST(10) default: LF_RADIX_HIST(11)
#undef LF_RADIX_HIST
  }
  uint32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
  for (int p = 0; p < npass; ++p) {
    const int shift = lo_bit + p * dbits;
    const int w = lo_bit + bits - shift < dbits ? lo_bit + bits - shift : dbits;
    const uint32_t mask = (1u << w) - 1u;   // the last pass may be narrower
    const uint32_t* gh = ghist + p * R;
    uint64_t* st = status + (int64_t)p * P * R;
    switch (dbits) {
#define LF_RADIX_PASS(B) case B: hipLaunchKernelGGL(radix_onesweep<B>, dim3(P), dim3(kRadixThreads), 0, s, ki, vi, ko, vo, n_dev, cap, shift, mask, gh, st, err); break;
      LF_RADIX_PASS(4) LF_RADIX_PASS(5) LF_RADIX_PASS(6) LF_RADIX_PASS(7) LF_RADIX_PASS(8) LF_RADIX_PASS(9)
      LF_RADIX_PASS(10) default: LF_RADIX_PASS(11)
#undef LF_RADIX_PASS
    }
    uint32_t* t = ki; ki = ko; ko = t;
    t = vi; vi = vo; vo = t;
  }
  *result_in_alt = npass & 1;
  return hipGetLastError();
}

hipError_t fill(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace lf
