// Device-wide scan / radix-sort primitives used by the MPI build.
//
// Both are single-pass over the data with decoupled look-back (Merrill & Garland, "Single-pass
// Parallel Prefix Scan with Decoupled Look-back", 2016; the radix passes follow Adinets &
// Merrill, "Onesweep", 2022): work-group j publishes its local aggregate, then walks back
// over the published aggregates / inclusive prefixes of work-groups j - 1, j - 2, ...  The
// chain follows launch order, the order in which work-groups are dispatched, so a
// work-group only waits on ones already running or done.  Every wait is bounded besides:
// on the bound it gives up, sets *err, and the results are wrong but every index stays in
// range.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lf {

// ---- scans ----------------------------------------------------------------------------
// u64 words of zero-initialised state a single-pass scan of n values needs.
size_t scan_state_words(int64_t n);

// out[0..n) = exclusive prefix sums of in[0..n), out[n] = total.  out holds n + 1 values;
// `state` (scan_state_words(n) u64) must be zero on entry and is not reusable afterwards.
// Sums must stay below 2^62.  With `heads`, in[] are taken as lengths of consecutive
// output segments, and heads[h] (h < n_heads, h 2^head_shift < total) receives the index
// of the segment holding output h 2^head_shift (the one with a non-zero length).
hipError_t exclusive_scan_u64(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* state, uint32_t* err,
                              hipStream_t s, uint32_t* heads = nullptr, int64_t n_heads = 0, int head_shift = 0);

// Two u32 scans in one pass (oa from a, ob from b, each with its total at [n]); the totals
// of a must stay below 2^32 and those of b below 2^30.
hipError_t exclusive_scan_pair_u32(const uint32_t* a, uint32_t* oa, const uint32_t* b, uint32_t* ob, int64_t n,
                                   uint64_t* state, uint32_t* err, hipStream_t s);

// ---- radix sort -----------------------------------------------------------------------
// Digit width of a sort of `bits` key bits with digits of at most max_digit_bits (4..11)
// bits, its number of passes, and the u32 words of zero-initialised digit totals (`ghist`)
// it needs.
int radix_digit_bits(int bits, int max_digit_bits);
int radix_passes(int bits, int max_digit_bits);
int radix_hist_words(int bits, int max_digit_bits);
constexpr int kRadixHistWordsMax = 6144;   // over every (bits <= 32, digit width 4..11)

// Work-groups of the fixed radix grid for up to `cap` elements, and the u32 scratch of a
// sort (cap < 2^31).
int radix_blocks(int64_t cap, int digit_bits);
size_t radix_tmp_u32(int64_t cap);

// Stable LSD sort of (key, value) pairs by the key bits [lo_bit, lo_bit + bits) (keys are
// moved whole).  The length is min(*n_dev, cap) (n_dev may be NULL: length = cap).  On
// return the sorted pairs are in (keys_alt, vals_alt) if *result_in_alt, else in (keys, vals).
// `ghist` (radix_hist_words u32) must be zero on entry; `tmp` needs no initialisation.
hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, int64_t cap,
                            const int64_t* n_dev, int lo_bit, int bits, uint32_t* tmp, uint32_t* ghist,
                            uint32_t* err, int* result_in_alt, hipStream_t s, int max_digit_bits = 8);

hipError_t fill(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);

}  // namespace lf
