// Radix sort of (64-bit key, int32 value) pairs on the context stream
// (rocPRIM device primitive: stable, deterministic).
#include <cstring>
#include <hip/hip_runtime.h>

#include <rocprim/rocprim.hpp>

#include "lss_internal.h"

namespace lss {

size_t sort_pairs_u64_tmp_bytes(int64_t n) {
    size_t bytes = 0;
    LSS_HIP(rocprim::radix_sort_pairs(nullptr, bytes, (const uint64_t *)nullptr, (uint64_t *)nullptr,
                                      (const int32_t *)nullptr, (int32_t *)nullptr, (size_t)n, 0, 64,
                                      (hipStream_t)0));
    return bytes + 256;
}

void sort_pairs_u64(void *tmp, size_t tmp_bytes, const uint64_t *kin, uint64_t *kout, const int32_t *vin,
                    int32_t *vout, int64_t n, int begin_bit, int end_bit, hipStream_t s) {
    if (n <= 0) return;
    LSS_HIP(rocprim::radix_sort_pairs(tmp, tmp_bytes, kin, kout, vin, vout, (size_t)n, (unsigned)begin_bit,
                                      (unsigned)end_bit, s));
}

void sort_pairs(Ctx &c, const uint64_t *kin, uint64_t *kout, const int32_t *vin, int32_t *vout, int64_t n,
                int end_bit) {
    if (n <= 0) return;
    size_t tb = sort_pairs_u64_tmp_bytes(n);
    c.sort_tmp.ensure(tb);
    sort_pairs_u64(c.sort_tmp.p, tb, kin, kout, vin, vout, n, 0, end_bit, c.stream);
}

}  // namespace lss
