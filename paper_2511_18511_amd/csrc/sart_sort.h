// Sort of W's entries by column: the transpose that SART's back-projection
// pass streams (Sec. 3.1).  Internal to librtx.
#pragma once
#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

// One entry of W's transpose: the row (ray) it belongs to and its weight.
template <class R>
struct CscEnt {
    int32_t row;
    R val;
};

// Stable sort of n (key, entry) pairs by the key bits [0, end_bit) on stream s
// (rocPRIM's LSD radix sort: entries with equal keys keep their input order).
// With tmp == nullptr only stores the scratch size that n pairs need in
// tmp_bytes.  The four arrays are distinct device buffers.
template <class R>
hipError_t csc_sort(void *tmp, size_t &tmp_bytes, const uint32_t *key_in, uint32_t *key_out,
                    const CscEnt<R> *ent_in, CscEnt<R> *ent_out, size_t n, unsigned end_bit, hipStream_t s);
