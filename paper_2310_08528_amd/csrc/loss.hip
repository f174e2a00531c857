// Photometric L1 loss of Eq. 9 (its image term): L = mean |I_hat - I| over
// the 3 x H x W values, and dL/dI_hat = sign(I_hat - I) / count (0 where the
// two are equal).  One pass: each 1024-thread block reduces its partial sum
// in LDS and adds it to the scalar with one atomic; the grid is held to 64
// blocks, since atomics on one word serialise (~2048 of them cost ~30 us,
// 256 ~13 us) while 64 wide blocks still stream the image at HBM rate.
#include "g4d_internal.h"

namespace g4d {
namespace {

__global__ __launch_bounds__(1024) void k_l1(const float *__restrict__ img, const float *__restrict__ target,
                                            size_t count, float inv_count, float *__restrict__ loss,
                                            float *__restrict__ grad) {
    __shared__ float s_part[16];
    float acc = 0.0f;
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    const size_t first = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    auto sgn = [&](float d) { return d > 0.0f ? inv_count : (d < 0.0f ? -inv_count : 0.0f); };
    // four values per load where the arrays allow it (16-byte aligned)
    const bool vec = ((reinterpret_cast<uintptr_t>(img) | reinterpret_cast<uintptr_t>(target) |
                       reinterpret_cast<uintptr_t>(grad)) & 15) == 0;
    const size_t n4 = vec ? count / 4 : 0;
    for (size_t i = first; i < n4; i += stride) {
        const float4 a = reinterpret_cast<const float4 *>(img)[i];
        const float4 b = reinterpret_cast<const float4 *>(target)[i];
        const float4 d = make_float4(a.x - b.x, a.y - b.y, a.z - b.z, a.w - b.w);
        acc += (fabsf(d.x) + fabsf(d.y)) + (fabsf(d.z) + fabsf(d.w));
        if (grad) reinterpret_cast<float4 *>(grad)[i] = make_float4(sgn(d.x), sgn(d.y), sgn(d.z), sgn(d.w));
    }
    for (size_t i = 4 * n4 + first; i < count; i += stride) {
        const float d = img[i] - target[i];
        acc += fabsf(d);
        if (grad) grad[i] = sgn(d);
    }
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0 && loss) {
        float sum = 0.0f;
        for (int w = 0; w < (int)(blockDim.x >> 6); ++w) sum += s_part[w];
        atomicAdd(loss, sum * inv_count);
    }
}

__global__ void k_zero1(float *p) { *p = 0.0f; }

}  // namespace
}  // namespace g4d

extern "C" g4d_status g4d_l1_loss(const float *image, const float *target, int64_t count, float *loss, float *grad,
                                  void *stream) {
    if (!image || !target || count < 1 || (!loss && !grad)) return G4D_EINVAL;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (loss) hipLaunchKernelGGL(g4d::k_zero1, dim3(1), dim3(1), 0, s, loss);
    const int blocks = (int)std::min<int64_t>((count + 1023) / 1024, 64);
    hipLaunchKernelGGL(g4d::k_l1, dim3(blocks), dim3(1024), 0, s, image, target, (size_t)count, 1.0f / (float)count,
                       loss, grad);
    G4D_HIP_CHECK(hipGetLastError());
    return G4D_OK;
}
