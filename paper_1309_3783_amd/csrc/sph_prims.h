// Device-wide primitives (scan, radix sort, fill) used by the cell build.
#pragma once
#include "sph_internal.h"

namespace sph {

// Words of uint32 scratch an exclusive scan of n elements needs.
size_t scan_tmp_words(int64_t n);
// out[i] = sum_{k<i} in[k] (in may equal out); *total (device, nullable) = sum.
hipError_t exclusive_scan(const uint32_t* in, uint32_t* out, int64_t n, uint32_t* tmp, uint32_t* total,
                          hipStream_t st);

// Words of uint32 scratch a radix sort of n elements needs.
size_t radix_tmp_words(int64_t n);
// Stable LSD sort of key[0..n) on bits [lo_bit, lo_bit + nbits) (8 bits per
// pass), moving val along (val may be null); keys equal on those bits keep
// their input order.  Ping-pongs with key_alt/val_alt; on return
// *result_in_alt tells which buffer holds the sorted data.
hipError_t radix_sort(uint64_t* key, uint32_t* val, uint64_t* key_alt, uint32_t* val_alt, int64_t n,
                      int nbits, uint32_t* tmp, hipStream_t st, bool* result_in_alt, int lo_bit = 0);

hipError_t fill_u32(uint32_t* p, int64_t n, uint32_t v, hipStream_t st);

}  // namespace sph
