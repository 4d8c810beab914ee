// Device-wide primitives of the MPI build: exclusive scans, a stable LSD radix sort of
// (u32 key, u32 value) pairs, and a fill kernel.  Every launch has a host-fixed grid; data
// dependent lengths are read from device memory, so nothing here waits on the host.
#include "sort_internal.h"

namespace lf {
namespace {

constexpr int kScanThreads = 256;
constexpr int kScanItems = 16;
constexpr int kScanChunk = kScanThreads * kScanItems;   // elements per scan block

template <typename T>
__device__ T block_exclusive_scan(T v, T* sh, T* total) {
  // Hillis-Steele inclusive scan over kScanThreads values in LDS.
  const int tid = threadIdx.x;
  sh[tid] = v;
  __syncthreads();
  for (int off = 1; off < kScanThreads; off <<= 1) {
    T add = tid >= off ? sh[tid - off] : T(0);
    __syncthreads();
    sh[tid] += add;
    __syncthreads();
  }
  const T incl = sh[tid];
  *total = sh[kScanThreads - 1];
  __syncthreads();
  return incl - v;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_reduce(const T* in, int64_t n, T* block_sums) {
  __shared__ T sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk;
  T s = 0;
  for (int i = 0; i < kScanItems; ++i) {
    const int64_t e = base + (int64_t)i * kScanThreads + threadIdx.x;
    if (e < n) s += in[e];
  }
  T total;
  block_exclusive_scan<T>(s, sh, &total);
  if (threadIdx.x == 0) block_sums[blockIdx.x] = total;
}

// One block scans the block sums (nb <= kScanChunk) in place; writes the grand total too.
template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_top(T* block_sums, int nb, T* total_out) {
  __shared__ T sh[kScanThreads];
  const int per = (nb + kScanThreads - 1) / kScanThreads;
  const int b0 = threadIdx.x * per;
  T s = 0;
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) s += block_sums[b0 + i];
  T total;
  T run = block_exclusive_scan<T>(s, sh, &total);
  for (int i = 0; i < per; ++i)
    if (b0 + i < nb) {
      const T v = block_sums[b0 + i];
      block_sums[b0 + i] = run;
      run += v;
    }
  if (threadIdx.x == 0) *total_out = total;
}

template <typename T>
__global__ __launch_bounds__(kScanThreads) void scan_down(const T* in, T* out, int64_t n, const T* block_sums) {
  __shared__ T sh[kScanThreads];
  const int64_t base = (int64_t)blockIdx.x * kScanChunk + (int64_t)threadIdx.x * kScanItems;
  T v[kScanItems];
  T s = 0;
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    v[i] = base + i < n ? in[base + i] : T(0);
    s += v[i];
  }
  T total;
  T run = block_exclusive_scan<T>(s, sh, &total) + block_sums[blockIdx.x];
#pragma unroll
  for (int i = 0; i < kScanItems; ++i) {
    if (base + i < n) out[base + i] = run;
    run += v[i];
  }
}

// ---------------------------------------------------------------------------------------
// Radix sort.  P blocks; block b sorts the elements [b*span, min(n, (b+1)*span)) where
// span = ceil(n / (P*256)) * 256 and n is read from device memory.
// ---------------------------------------------------------------------------------------
constexpr int kRadixThreads = 256;
constexpr int kWaves = kRadixThreads / 64;

__device__ __forceinline__ int64_t sort_len(const int64_t* n_dev, int64_t n_host, int64_t cap) {
  int64_t n = n_dev ? *n_dev : n_host;
  return n < cap ? n : cap;
}

__device__ __forceinline__ int64_t block_span(int64_t n) {
  const int64_t per = (n + (int64_t)gridDim.x * kRadixThreads - 1) / ((int64_t)gridDim.x * kRadixThreads);
  return per * kRadixThreads;
}

template <int BITS>
__global__ __launch_bounds__(kRadixThreads) void radix_upsweep(const uint32_t* keys, const int64_t* n_dev,
                                                               int64_t n_host, int64_t cap, int shift,
                                                               uint32_t mask, uint32_t* counts) {
  constexpr int R = 1 << BITS;
  __shared__ uint32_t hist[R];
  const int64_t n = sort_len(n_dev, n_host, cap);
  const int64_t span = block_span(n);
  const int64_t b0 = (int64_t)blockIdx.x * span;
  const int64_t b1 = min(n, b0 + span);
  for (int d = threadIdx.x; d < R; d += kRadixThreads) hist[d] = 0;
  __syncthreads();
  for (int64_t e = b0 + threadIdx.x; e < b1; e += kRadixThreads) atomicAdd(&hist[(keys[e] >> shift) & mask], 1u);
  __syncthreads();
  for (int d = threadIdx.x; d < R; d += kRadixThreads) counts[(int64_t)d * gridDim.x + blockIdx.x] = hist[d];
}

template <int BITS>
__global__ __launch_bounds__(kRadixThreads) void radix_downsweep(const uint32_t* keys_in, const uint32_t* vals_in,
                                                                 uint32_t* keys_out, uint32_t* vals_out,
                                                                 const int64_t* n_dev, int64_t n_host, int64_t cap,
                                                                 int shift, uint32_t mask, const uint32_t* offsets) {
  constexpr int R = 1 << BITS;
  __shared__ uint32_t running[R];
  __shared__ uint32_t wcount[kWaves][R];
  const int64_t n = sort_len(n_dev, n_host, cap);
  const int64_t span = block_span(n);
  const int64_t b0 = (int64_t)blockIdx.x * span;
  const int64_t b1 = min(n, b0 + span);
  const int tid = threadIdx.x;
  const int lane = tid & 63;
  const int wave = tid >> 6;
  for (int d = tid; d < R; d += kRadixThreads) {
    running[d] = offsets[(int64_t)d * gridDim.x + blockIdx.x];
    for (int w = 0; w < kWaves; ++w) wcount[w][d] = 0;
  }
  __syncthreads();
  const uint64_t lt = lane ? (~0ull >> (64 - lane)) : 0ull;
  for (int64_t r0 = b0; r0 < b1; r0 += kRadixThreads) {
    const int64_t e = r0 + tid;
    const bool valid = e < b1;
    uint32_t key = 0, val = 0, d = 0;
    if (valid) {
      key = keys_in[e];
      val = vals_in[e];
      d = (key >> shift) & mask;
    }
    // lanes of this wave holding the same digit
    uint64_t peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < BITS; ++b) {
      const bool bit = (d >> b) & 1u;
      const uint64_t m = __ballot(bit);
      peers &= bit ? m : ~m;
    }
    const uint32_t rank = __popcll(peers & lt);
    const uint32_t cnt = __popcll(peers);
    const bool leader = valid && rank == 0;
    if (leader) wcount[wave][d] = cnt;
    __syncthreads();
    if (valid) {
      uint32_t pos = running[d] + rank;
      for (int w = 0; w < wave; ++w) pos += wcount[w][d];
      keys_out[pos] = key;
      vals_out[pos] = val;
    }
    __syncthreads();
    // Only the digits present in this round change: each wave's leader for a digit advances
    // the running offset and clears its count.  The next round reads both only after its
    // first barrier, which every wave reaches after these updates.
    if (leader) {
      atomicAdd(&running[d], cnt);
      wcount[wave][d] = 0;
    }
  }
}

__global__ void fill_u32(uint32_t* p, int64_t n, uint32_t v) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = v;
}

}  // namespace

size_t scan_tmp_elems(int64_t n) { return (size_t)((n + kScanChunk - 1) / kScanChunk) + 1; }

template <typename T>
hipError_t exclusive_scan(const T* in, T* out, int64_t n, T* tmp, hipStream_t s) {
  // out[0..n) = exclusive prefix sums, out[n] = total.  tmp holds scan_tmp_elems(n) values.
  const int nb = (int)((n + kScanChunk - 1) / kScanChunk);
  if (nb == 0) {
    hipLaunchKernelGGL(fill_u32, dim3(1), dim3(1), 0, s, reinterpret_cast<uint32_t*>(out), (int64_t)(sizeof(T) / 4), 0u);
    return hipGetLastError();
  }
  if (nb > kScanChunk) return hipErrorInvalidValue;
  hipLaunchKernelGGL((scan_reduce<T>), dim3(nb), dim3(kScanThreads), 0, s, in, n, tmp);
  hipLaunchKernelGGL((scan_top<T>), dim3(1), dim3(kScanThreads), 0, s, tmp, nb, out + n);
  hipLaunchKernelGGL((scan_down<T>), dim3(nb), dim3(kScanThreads), 0, s, in, out, n, tmp);
  return hipGetLastError();
}

template hipError_t exclusive_scan<uint32_t>(const uint32_t*, uint32_t*, int64_t, uint32_t*, hipStream_t);
template hipError_t exclusive_scan<uint64_t>(const uint64_t*, uint64_t*, int64_t, uint64_t*, hipStream_t);

// Blocks of the radix grid: about 1024 elements per block, so small sorts still spread
// over the CUs, with the per-block digit counts (2^digit_bits * blocks) kept to 2^18.
constexpr int64_t kMaxCounts = 1 << 18;

int radix_blocks(int64_t cap, int digit_bits) {
  int64_t b = (cap + 1023) / 1024;
  const int64_t lim = kMaxCounts >> digit_bits;
  if (b > lim) b = lim;
  return (int)(b < 1 ? 1 : b);
}

constexpr int kMaxDigitBits = 11;

size_t radix_tmp_u32(int64_t cap) {
  (void)cap;
  return (size_t)(2 * kMaxCounts + scan_tmp_elems(kMaxCounts) + 1);
}

hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, int64_t cap,
                            const int64_t* n_dev, int lo_bit, int bits, uint32_t* tmp, int* result_in_alt,
                            hipStream_t s, int max_digit_bits) {
  if (bits < 1 || lo_bit < 0 || lo_bit + bits > 32) return hipErrorInvalidValue;
  if (max_digit_bits < 1 || max_digit_bits > kMaxDigitBits) return hipErrorInvalidValue;
  // passes of at most max_digit_bits bits, as even as possible (32 bits at 11: 11 + 11 + 10)
  const int npass = (bits + max_digit_bits - 1) / max_digit_bits;
  const int dbits = (bits + npass - 1) / npass;
  const int P = radix_blocks(cap, dbits);
  const int64_t nc = (1LL << dbits) * P;
  uint32_t* counts = tmp;
  uint32_t* offs = tmp + nc;
  uint32_t* stmp = tmp + 2 * nc + 1;       // offs holds nc + 1 values (the scan writes the total)
  uint32_t *ki = keys, *vi = vals, *ko = keys_alt, *vo = vals_alt;
  int passes = 0;
  for (int shift = lo_bit; shift < lo_bit + bits; shift += dbits) {
    const int w = lo_bit + bits - shift < dbits ? lo_bit + bits - shift : dbits;
    const uint32_t mask = (1u << w) - 1u;   // the last pass may be narrower
    switch (dbits) {
#define LF_RADIX_UP(B) case B: hipLaunchKernelGGL(radix_upsweep<B>, dim3(P), dim3(kRadixThreads), 0, s, ki, n_dev, cap, cap, shift, mask, counts); break;
      LF_RADIX_UP(1) LF_RADIX_UP(2) LF_RADIX_UP(3) LF_RADIX_UP(4) LF_RADIX_UP(5) LF_RADIX_UP(6)
      LF_RADIX_UP(7) LF_RADIX_UP(8) LF_RADIX_UP(9) LF_RADIX_UP(10) default: LF_RADIX_UP(11)
#undef LF_RADIX_UP
    }
    hipError_t e = exclusive_scan<uint32_t>(counts, offs, nc, stmp, s);
    if (e != hipSuccess) return e;
    switch (dbits) {
#define LF_RADIX_DOWN(B) case B: hipLaunchKernelGGL(radix_downsweep<B>, dim3(P), dim3(kRadixThreads), 0, s, ki, vi, ko, vo, n_dev, cap, cap, shift, mask, offs); break;
      LF_RADIX_DOWN(1) LF_RADIX_DOWN(2) LF_RADIX_DOWN(3) LF_RADIX_DOWN(4) LF_RADIX_DOWN(5) LF_RADIX_DOWN(6)
      LF_RADIX_DOWN(7) LF_RADIX_DOWN(8) LF_RADIX_DOWN(9) LF_RADIX_DOWN(10) default: LF_RADIX_DOWN(11)
#undef LF_RADIX_DOWN
    }
    uint32_t* t = ki; ki = ko; ko = t;
    t = vi; vi = vo; vo = t;
    ++passes;
  }
  *result_in_alt = passes & 1;
  return hipGetLastError();
}

int radix_passes(int bits, int max_digit_bits) { return bits < 1 ? 0 : (bits + max_digit_bits - 1) / max_digit_bits; }

hipError_t fill(uint32_t* p, int64_t n, uint32_t v, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(fill_u32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n, v);
  return hipGetLastError();
}

}  // namespace lf
