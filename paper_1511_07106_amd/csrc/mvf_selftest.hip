// Self-test of the hardware square-root estimate that the integration
// kernel's square-root filter relies on (not part of the libmvf ABI; built
// as libmvf_selftest.so for the GPU tests).
//
// For every binary32 x with bit pattern in [first, first + count) (positive
// values), compares the estimate (v_sqrt_f32) with the correctly rounded
// root: the largest distance in units in the last place for x >= 2^-96, and
// the largest absolute difference for x < 2^-96.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <string.h>

namespace {

__global__ __launch_bounds__(256) void sqrt_check_kernel(uint32_t first, uint32_t count, unsigned int* out)
{
    unsigned int max_ulp = 0;
    float max_abs = 0.0f;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t j = blockIdx.x * blockDim.x + threadIdx.x; j < count; j += stride) {
        const float x = __uint_as_float(first + j);
        const float e = __builtin_amdgcn_sqrtf(x);
        const float r = sqrtf(x);
        if (x >= 0x1p-96f) {
            const int d = (int)__float_as_uint(e) - (int)__float_as_uint(r);
            max_ulp = max(max_ulp, (unsigned int)(d < 0 ? -d : d));
        } else {
            max_abs = fmaxf(max_abs, fabsf(e - r));
        }
    }
    for (int o = 32; o >= 1; o >>= 1) {
        max_ulp = max(max_ulp, (unsigned int)__shfl_xor((int)max_ulp, o));
        max_abs = fmaxf(max_abs, __shfl_xor(max_abs, o));
    }
    if ((threadIdx.x & 63) == 0) {
        atomicMax(&out[0], max_ulp);
        atomicMax(&out[1], __float_as_uint(max_abs));  // non-negative floats order like their bits
    }
}

}  // namespace

// Returns 0 on success.  max_ulp: largest ulp distance for x >= 2^-96;
// max_abs: largest absolute difference for x < 2^-96.  Synchronous.
extern "C" int mvf_selftest_sqrt(uint32_t first, uint32_t count, uint32_t* max_ulp, float* max_abs)
{
    if (!max_ulp || !max_abs || first >= 0x7f800000u || count > 0x7f800000u - first) return 1;
    unsigned int* d = nullptr;
    if (hipMalloc((void**)&d, 2 * sizeof(unsigned int)) != hipSuccess) return 2;
    unsigned int h[2] = {0, 0};
    int rc = 0;
    if (hipMemcpy(d, h, sizeof(h), hipMemcpyHostToDevice) != hipSuccess) rc = 3;
    if (!rc && count) {
        hipLaunchKernelGGL(sqrt_check_kernel, dim3(4096), dim3(256), 0, nullptr, first, count, d);
        if (hipGetLastError() != hipSuccess) rc = 4;
    }
    if (!rc && hipMemcpy(h, d, sizeof(h), hipMemcpyDeviceToHost) != hipSuccess) rc = 5;
    (void)hipFree(d);
    *max_ulp = h[0];
    memcpy(max_abs, &h[1], sizeof(float));
    return rc;
}
