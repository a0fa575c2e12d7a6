// Read+write stream kernel for gfx950, used by the benchmark to measure the
// practical HBM ceiling of a kernel that reads every byte of one buffer once
// and writes every byte of another once (the traffic pattern of one worm-LBM
// step: each population read once and written once).  Not part of the
// worm-LBM library; built as its own shared object.
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

namespace {

constexpr int kThreads = 256;
// four floats moved by one 16-byte load or store
typedef float v4f __attribute__((ext_vector_type(4)));

// Each thread copies U 16-byte values, U * kThreads apart, so that a wave's
// loads and stores cover whole 1 KiB runs and U loads are in flight before
// the first store.  NT: stores carry the non-temporal hint, as the worm-LBM
// step kernels' population stores do.
template <int U, bool NT>
__global__ __launch_bounds__(kThreads) void k_copy(const v4f* __restrict__ src,
                                                  v4f* __restrict__ dst, size_t n4) {
  const size_t base = size_t(blockIdx.x) * kThreads * U + threadIdx.x;
  v4f v[U];
#pragma unroll
  for (int j = 0; j < U; ++j) {
    const size_t i = base + size_t(j) * kThreads;
    if (i < n4) v[j] = src[i];
  }
#pragma unroll
  for (int j = 0; j < U; ++j) {
    const size_t i = base + size_t(j) * kThreads;
    if (i < n4) {
      if constexpr (NT)
        __builtin_nontemporal_store(v[j], dst + i);
      else
        dst[i] = v[j];
    }
  }
}

// The same with 4-byte values (one float per lane per access, as the step
// kernels' population loads and stores): U floats per thread, U * kThreads
// apart.
template <int U, bool NT>
__global__ __launch_bounds__(kThreads) void k_copy_f32(const float* __restrict__ src,
                                                      float* __restrict__ dst, size_t n) {
  const size_t base = size_t(blockIdx.x) * kThreads * U + threadIdx.x;
  float v[U];
#pragma unroll
  for (int j = 0; j < U; ++j) {
    const size_t i = base + size_t(j) * kThreads;
    if (i < n) v[j] = src[i];
  }
#pragma unroll
  for (int j = 0; j < U; ++j) {
    const size_t i = base + size_t(j) * kThreads;
    if (i < n) {
      if constexpr (NT)
        __builtin_nontemporal_store(v[j], dst + i);
      else
        dst[i] = v[j];
    }
  }
}

template <int U, bool NT>
hipError_t launch_f32(const float* s, float* d, size_t n, hipStream_t st) {
  const size_t per = size_t(kThreads) * U;
  const size_t blocks = (n + per - 1) / per;
  if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_copy_f32<U, NT>), dim3(unsigned(blocks)), dim3(kThreads), 0, st, s, d, n);
  return hipGetLastError();
}

template <int U, bool NT>
hipError_t launch(const v4f* s, v4f* d, size_t n4, hipStream_t st) {
  const size_t per = size_t(kThreads) * U;
  const size_t blocks = (n4 + per - 1) / per;
  if (blocks > 0x7fffffffu) return hipErrorInvalidValue;
  hipLaunchKernelGGL((k_copy<U, NT>), dim3(unsigned(blocks)), dim3(kThreads), 0, st, s, d, n4);
  return hipGetLastError();
}

}  // namespace

extern "C" __attribute__((visibility("default"))) int wlbm_probe_copy(const void* src, void* dst,
                                                                      size_t bytes, int unroll,
                                                                      int nontemporal,
                                                                      void* stream) {
  // bytes: a multiple of 16 (whole 16-byte values); src and dst 16-byte aligned
  if (bytes % 16 || reinterpret_cast<uintptr_t>(src) % 16 || reinterpret_cast<uintptr_t>(dst) % 16)
    return int(hipErrorInvalidValue);
  const size_t n4 = bytes / 16;
  const auto* s = static_cast<const v4f*>(src);
  auto* d = static_cast<v4f*>(dst);
  auto st = static_cast<hipStream_t>(stream);
  hipError_t e;
  switch (unroll * 2 + (nontemporal ? 1 : 0)) {
    case 2: e = launch<1, false>(s, d, n4, st); break;
    case 3: e = launch<1, true>(s, d, n4, st); break;
    case 4: e = launch<2, false>(s, d, n4, st); break;
    case 5: e = launch<2, true>(s, d, n4, st); break;
    case 8: e = launch<4, false>(s, d, n4, st); break;
    case 9: e = launch<4, true>(s, d, n4, st); break;
    default: e = hipErrorInvalidValue;
  }
  return int(e);
}

// The 4-byte variant: unroll 4, 8 or 16 floats per thread.
extern "C" __attribute__((visibility("default"))) int wlbm_probe_copy_f32(const void* src,
                                                                          void* dst,
                                                                          size_t bytes,
                                                                          int unroll,
                                                                          int nontemporal,
                                                                          void* stream) {
  if (bytes % 4 || reinterpret_cast<uintptr_t>(src) % 4 || reinterpret_cast<uintptr_t>(dst) % 4)
    return int(hipErrorInvalidValue);
  const size_t n = bytes / 4;
  const auto* s = static_cast<const float*>(src);
  auto* d = static_cast<float*>(dst);
  auto st = static_cast<hipStream_t>(stream);
  hipError_t e;
  switch (unroll * 2 + (nontemporal ? 1 : 0)) {
    case 8: e = launch_f32<4, false>(s, d, n, st); break;
    case 9: e = launch_f32<4, true>(s, d, n, st); break;
    case 16: e = launch_f32<8, false>(s, d, n, st); break;
    case 17: e = launch_f32<8, true>(s, d, n, st); break;
    case 32: e = launch_f32<16, false>(s, d, n, st); break;
    case 33: e = launch_f32<16, true>(s, d, n, st); break;
    default: e = hipErrorInvalidValue;
  }
  return int(e);
}
