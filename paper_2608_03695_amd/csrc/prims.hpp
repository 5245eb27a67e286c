// Device-wide primitives between the method's kernels, written for gfx950 (prims.hip): stable
// LSD radix sorts of key/value pairs over the key bits in use, exclusive scans and
// reduce-by-key over sorted keys.  All work runs on the given stream; temporary storage comes
// from the callback (one request per call).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stddef.h>

namespace mslm {

// Temporary-storage callback: returns a device pointer of at least `bytes`.
struct TempAlloc {
  void *(*get)(void *ctx, size_t bytes);
  void *ctx;
};

hipError_t sort_pairs_u32_u32(const uint32_t *kin, uint32_t *kout, const uint32_t *vin,
                              uint32_t *vout, int64_t n, int end_bit, hipStream_t st, TempAlloc ta);
hipError_t sort_pairs_u64_i64(const uint64_t *kin, uint64_t *kout, const int64_t *vin,
                              int64_t *vout, int64_t n, int end_bit, hipStream_t st, TempAlloc ta);
hipError_t sort_pairs_u64_i32(const uint64_t *kin, uint64_t *kout, const int32_t *vin,
                              int32_t *vout, int64_t n, int end_bit, hipStream_t st, TempAlloc ta);
hipError_t reduce_by_key_u64_i64(const uint64_t *kin, uint64_t *kout, const int64_t *vin,
                                 int64_t *vout, int64_t *nout, int64_t n, hipStream_t st,
                                 TempAlloc ta);
hipError_t reduce_by_key_u64_i32(const uint64_t *kin, uint64_t *kout, const int32_t *vin,
                                 int32_t *vout, int64_t *nout, int64_t n, hipStream_t st,
                                 TempAlloc ta);
hipError_t exclusive_sum_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t st,
                             TempAlloc ta);
hipError_t exclusive_sum_u8_i64(const uint8_t *in, int64_t *out, int64_t n, hipStream_t st,
                                TempAlloc ta);
hipError_t exclusive_sum_u32_i64(const uint32_t *in, int64_t *out, int64_t n, hipStream_t st,
                                 TempAlloc ta);

}  // namespace mslm
