// The column sort of SART's transpose, in a translation unit of its own so
// that rocPRIM's templates are compiled once and apart from the tracer.
#include "sart_sort.h"

#include <rocprim/device/device_radix_sort.hpp>

template <class R>
hipError_t csc_sort(void *tmp, size_t &tmp_bytes, const uint32_t *key_in, uint32_t *key_out,
                    const CscEnt<R> *ent_in, CscEnt<R> *ent_out, size_t n, unsigned end_bit, hipStream_t s)
{
    return rocprim::radix_sort_pairs(tmp, tmp_bytes, key_in, key_out, ent_in, ent_out, n, 0u, end_bit, s);
}

template hipError_t csc_sort<float>(void *, size_t &, const uint32_t *, uint32_t *, const CscEnt<float> *,
                                    CscEnt<float> *, size_t, unsigned, hipStream_t);
template hipError_t csc_sort<double>(void *, size_t &, const uint32_t *, uint32_t *, const CscEnt<double> *,
                                     CscEnt<double> *, size_t, unsigned, hipStream_t);
