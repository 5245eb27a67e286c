#include "prims.hpp"

#include <hipcub/hipcub.hpp>

namespace mslm {

namespace {
struct SumI64 {
  __host__ __device__ int64_t operator()(int64_t a, int64_t b) const { return a + b; }
};
struct SumI32 {
  __host__ __device__ int32_t operator()(int32_t a, int32_t b) const { return a + b; }
};
struct U8ToI64 {
  __host__ __device__ int64_t operator()(uint8_t x) const { return (int64_t)x; }
};
struct U32ToI64 {
  __host__ __device__ int64_t operator()(uint32_t x) const { return (int64_t)x; }
};

template <class F>
hipError_t two_phase(F f, TempAlloc ta) {
  size_t bytes = 0;
  hipError_t e = f(nullptr, bytes);
  if (e != hipSuccess) return e;
  void *p = ta.get(ta.ctx, bytes ? bytes : 1);
  if (!p) return hipErrorOutOfMemory;
  return f(p, bytes);
}
}  // namespace

hipError_t sort_pairs_u32_u32(const uint32_t *kin, uint32_t *kout, const uint32_t *vin,
                              uint32_t *vout, int64_t n, int end_bit, hipStream_t st,
                              TempAlloc ta) {
  if (n == 0) return hipSuccess;
  return two_phase([&](void *p, size_t &b) {
    return hipcub::DeviceRadixSort::SortPairs(p, b, kin, kout, vin, vout, n, 0, end_bit, st);
  }, ta);
}

hipError_t sort_pairs_u64_i64(const uint64_t *kin, uint64_t *kout, const int64_t *vin,
                              int64_t *vout, int64_t n, int end_bit, hipStream_t st,
                              TempAlloc ta) {
  if (n == 0) return hipSuccess;
  return two_phase([&](void *p, size_t &b) {
    return hipcub::DeviceRadixSort::SortPairs(p, b, kin, kout, vin, vout, n, 0, end_bit, st);
  }, ta);
}

hipError_t sort_pairs_u64_i32(const uint64_t *kin, uint64_t *kout, const int32_t *vin,
                              int32_t *vout, int64_t n, int end_bit, hipStream_t st,
                              TempAlloc ta) {
  if (n == 0) return hipSuccess;
  return two_phase([&](void *p, size_t &b) {
    return hipcub::DeviceRadixSort::SortPairs(p, b, kin, kout, vin, vout, n, 0, end_bit, st);
  }, ta);
}

hipError_t reduce_by_key_u64_i64(const uint64_t *kin, uint64_t *kout, const int64_t *vin,
                                 int64_t *vout, int64_t *nout, int64_t n, hipStream_t st,
                                 TempAlloc ta) {
  if (n == 0) return hipMemsetAsync(nout, 0, sizeof(int64_t), st);
  return two_phase([&](void *p, size_t &b) {
    return hipcub::DeviceReduce::ReduceByKey(p, b, kin, kout, vin, vout, nout, SumI64(), n, st);
  }, ta);
}

hipError_t reduce_by_key_u64_i32(const uint64_t *kin, uint64_t *kout, const int32_t *vin,
                                 int32_t *vout, int64_t *nout, int64_t n, hipStream_t st,
                                 TempAlloc ta) {
  if (n == 0) return hipMemsetAsync(nout, 0, sizeof(int64_t), st);
  return two_phase([&](void *p, size_t &b) {
    return hipcub::DeviceReduce::ReduceByKey(p, b, kin, kout, vin, vout, nout, SumI32(), n, st);
  }, ta);
}

hipError_t exclusive_sum_i64(const int64_t *in, int64_t *out, int64_t n, hipStream_t st,
                             TempAlloc ta) {
  if (n == 0) return hipSuccess;
  return two_phase([&](void *p, size_t &b) {
    return hipcub::DeviceScan::ExclusiveSum(p, b, in, out, n, st);
  }, ta);
}

hipError_t exclusive_sum_u8_i64(const uint8_t *in, int64_t *out, int64_t n, hipStream_t st,
                                TempAlloc ta) {
  if (n == 0) return hipSuccess;
  hipcub::TransformInputIterator<int64_t, U8ToI64, const uint8_t *> it(in, U8ToI64());
  return two_phase([&](void *p, size_t &b) {
    return hipcub::DeviceScan::ExclusiveSum(p, b, it, out, n, st);
  }, ta);
}

hipError_t exclusive_sum_u32_i64(const uint32_t *in, int64_t *out, int64_t n, hipStream_t st,
                                 TempAlloc ta) {
  if (n == 0) return hipSuccess;
  hipcub::TransformInputIterator<int64_t, U32ToI64, const uint32_t *> it(in, U32ToI64());
  return two_phase([&](void *p, size_t &b) {
    return hipcub::DeviceScan::ExclusiveSum(p, b, it, out, n, st);
  }, ta);
}

}  // namespace mslm
