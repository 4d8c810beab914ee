// Device-wide scan / radix-sort primitives used by the MPI build.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace lf {

// Elements of scratch an exclusive scan of n values needs.
size_t scan_tmp_elems(int64_t n);

// out[0..n) = exclusive prefix sums of in[0..n), out[n] = total (n is host-known).  out holds
// n + 1 values; tmp (scan_tmp_elems(n) values) must not overlap out.
template <typename T>
hipError_t exclusive_scan(const T* in, T* out, int64_t n, T* tmp, hipStream_t s);

// Blocks of the fixed radix-sort grid for up to `cap` elements with digit_bits-bit digits,
// and the scratch size (u32) of any sort.
int radix_blocks(int64_t cap, int digit_bits);
size_t radix_tmp_u32(int64_t cap);

// Stable LSD sort of (key, value) pairs by the key bits [lo_bit, lo_bit + bits) (keys are
// moved whole).  The length is min(*n_dev, cap) (n_dev may be NULL: length = cap).  On
// return the sorted pairs are in (keys_alt, vals_alt) if *result_in_alt, else in (keys, vals).
// Digits of at most max_digit_bits (<= 11) bits per pass: wide digits mean fewer passes,
// narrow ones longer runs of equal digits per work-group round and so more coalesced writes.
hipError_t radix_sort_pairs(uint32_t* keys, uint32_t* vals, uint32_t* keys_alt, uint32_t* vals_alt, int64_t cap,
                            const int64_t* n_dev, int lo_bit, int bits, uint32_t* tmp, int* result_in_alt,
                            hipStream_t s, int max_digit_bits = 11);

hipError_t fill(uint32_t* p, int64_t n, uint32_t v, hipStream_t s);

// Number of passes radix_sort_pairs makes over `bits` key bits (odd: result in the alt arrays).
int radix_passes(int bits, int max_digit_bits = 11);

}  // namespace lf
