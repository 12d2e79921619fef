// The controller search's selection step on the device: every candidate's
// fitness from its rollout (or plain-step) end state, then the best n_top
// candidates in order. The search runs one candidate controller per robot,
// scores it by how far the robot walked along its start heading with a
// penalty for the motors' effort, and re-simulates only the best few with the
// plain step (the surrogate screen of the controller experiments, Sec. V).
#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include <cmath>
#include <cstdint>

#include "npx.h"
#include "npx_internal.h"

using npx::fail;

namespace {

// f = (p1 - p0) . h - w tau / n_calls; -inf for a flagged candidate or a
// non-finite value. The sort key maps f to an unsigned integer that orders
// like -f (best first): the float's bits with the sign bit set for f >= 0
// and all bits flipped for f < 0 order like f; their complement like -f.
__global__ void fitness_kernel(const float* __restrict__ s0, const float* __restrict__ s1,
                               int64_t lds, const float* __restrict__ heading,
                               const float* __restrict__ tau, float inv_calls, float wt,
                               const int32_t* __restrict__ flags, int64_t n, float* fitness,
                               uint32_t* key, int32_t* idx) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const float dx = s1[i * lds] - s0[i * lds], dy = s1[i * lds + 1] - s0[i * lds + 1];
  const float dist = dx * heading[2 * i] + dy * heading[2 * i + 1];
  float f = dist - wt * (tau[i] * inv_calls);
  if ((flags && flags[i] != 0) || !isfinite(f)) f = -INFINITY;
  if (f == 0.f) f = 0.f;  // -0 ranks as +0
  fitness[i] = f;
  if (key) {
    const uint32_t b = __float_as_uint(f);
    const uint32_t up = (b & 0x80000000u) ? ~b : (b | 0x80000000u);
    key[i] = ~up;
    idx[i] = (int32_t)i;
  }
}

}  // namespace

extern "C" {

npx_status npx_sur_screen_select(const float* s0, const float* s1, int64_t lds,
                                 const float* heading, const float* tau, int32_t n_calls,
                                 float torque_weight, const int32_t* flags, int64_t n,
                                 int32_t n_top, float* fitness, int32_t* top, void* stream) {
  if (n < 0 || n > INT32_MAX || n_top < 0 || n_top > n)
    return fail(NPX_EINVAL, "need 0 <= n_top <= n <= 2^31 - 1 (n %lld, n_top %d)",
                (long long)n, n_top);
  if (n_calls < 1 || lds < 2) return fail(NPX_EINVAL, "need n_calls >= 1 and lds >= 2");
  if (n > 0 && (!s0 || !s1 || !heading || !tau || !fitness))
    return fail(NPX_EINVAL, "null input or output");
  if (n_top > 0 && !top) return fail(NPX_EINVAL, "null top output");
  if (n == 0) return NPX_OK;
  hipStream_t st = (hipStream_t)stream;
  const unsigned blocks = (unsigned)((n + 255) / 256);
  if (n_top == 0) {
    hipLaunchKernelGGL(fitness_kernel, dim3(blocks), dim3(256), 0, st, s0, s1, lds, heading, tau,
                       1.0f / (float)n_calls, torque_weight, flags, n, fitness, nullptr, nullptr);
    const hipError_t e = hipGetLastError();
    return e == hipSuccess ? NPX_OK : fail(NPX_EHIP, "fitness launch: %s", hipGetErrorString(e));
  }
  // keys and indices in, sorted keys and indices out, then the sort's own
  // temporary storage: one stream-ordered allocation, freed on the stream
  const int ni = (int)n;
  size_t tmp = 0;
  if (hipcub::DeviceRadixSort::SortPairs(nullptr, tmp, (const uint32_t*)nullptr,
                                         (uint32_t*)nullptr, (const int32_t*)nullptr,
                                         (int32_t*)nullptr, ni, 0, 32, st) != hipSuccess)
    return fail(NPX_EHIP, "sort size query failed");
  const size_t arr = ((size_t)n * 4 + 255) / 256 * 256;
  char* buf = nullptr;
  if (hipMallocAsync(reinterpret_cast<void**>(&buf), 4 * arr + tmp, st) != hipSuccess)
    return fail(NPX_ENOMEM, "screen selection: %zu bytes of scratch", 4 * arr + tmp);
  uint32_t* k_in = reinterpret_cast<uint32_t*>(buf);
  uint32_t* k_out = reinterpret_cast<uint32_t*>(buf + arr);
  int32_t* i_in = reinterpret_cast<int32_t*>(buf + 2 * arr);
  int32_t* i_out = reinterpret_cast<int32_t*>(buf + 3 * arr);
  hipLaunchKernelGGL(fitness_kernel, dim3(blocks), dim3(256), 0, st, s0, s1, lds, heading, tau,
                     1.0f / (float)n_calls, torque_weight, flags, n, fitness, k_in, i_in);
  hipError_t e = hipGetLastError();
  // radix sort is stable: equal fitness keeps the lower index first
  if (e == hipSuccess)
    e = hipcub::DeviceRadixSort::SortPairs(buf + 4 * arr, tmp, k_in, k_out, i_in, i_out, ni, 0,
                                           32, st);
  if (e == hipSuccess)
    e = hipMemcpyAsync(top, i_out, (size_t)n_top * sizeof(int32_t), hipMemcpyDeviceToDevice, st);
  const hipError_t ef = hipFreeAsync(buf, st);
  if (e != hipSuccess) return fail(NPX_EHIP, "screen selection: %s", hipGetErrorString(e));
  if (ef != hipSuccess) return fail(NPX_EHIP, "screen scratch free: %s", hipGetErrorString(ef));
  return NPX_OK;
}

}  // extern "C"
