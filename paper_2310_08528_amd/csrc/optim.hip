// The rest of a training iteration: the grid total-variation term of Eq. 9
// on the HexPlane cells, and an Adam update of every trainable tensor.
//
// TV: for each plane [n_b][n_a][F] of each scale, the mean squared difference
// of neighbouring cells along a plus that along b,
//   tv = sum_planes ( mean (R[i, j+1] - R[i, j])^2 + mean (R[i+1, j] - R[i, j])^2 ),
// loss += weight * tv, and dtv/dR[i, j] = 2/N_a (2 R[i,j] - R[i,j-1] -
// R[i,j+1]) + 2/N_b (...) with the missing neighbours left out at the edges
// (N_a = n_b (n_a - 1) F, N_b = (n_b - 1) n_a F differences).  32-bit
// indices (a plane holds at most 2^31 values; F = 16 or 32 is a shift); each
// block reduces its loss terms and adds them with one atomic.
//
// Adam (Kingma & Ba): m <- b1 m + (1 - b1) g, v <- b2 v + (1 - b2) g^2,
// p <- p - lr (m / (1 - b1^t)) / (sqrt(v / (1 - b2^t)) + eps); up to 64
// tensors per launch, one grid-stride pass each.
#include "g4d_internal.h"

namespace g4d {
namespace {

struct TvPlanes {
    const float *plane[18];
    float *grad[18];
    int na[18], nb[18];
    int n_planes, feat;
    float weight;
};

// The loss terms and gradient of one value, given its four neighbours'
// differences (each present or not).
__device__ __forceinline__ float tv_one(float r, float rr, float rl, float rd, float ru, bool has_r, bool has_l,
                                        bool has_d, bool has_u, float ia, float ib, float &acc) {
    float g = 0.0f;
    if (has_r) {
        const float d = rr - r;
        acc += d * d * ia;
        g -= 2.0f * d * ia;
    }
    if (has_l) g += 2.0f * (r - rl) * ia;
    if (has_d) {
        const float d = rd - r;
        acc += d * d * ib;
        g -= 2.0f * d * ib;
    }
    if (has_u) g += 2.0f * (r - ru) * ib;
    return g;
}

__device__ __forceinline__ void tv_block_loss(float acc, float weight, float *__restrict__ loss) {
    __shared__ float s_part[4];
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) acc += __shfl_xor(acc, o, 64);
    if ((threadIdx.x & 63) == 0) s_part[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0 && loss) atomicAdd(loss, weight * ((s_part[0] + s_part[1]) + (s_part[2] + s_part[3])));
}

// Vector form (every plane and gradient 16-byte aligned): a thread takes
// four consecutive channels of a cell (16-byte loads and stores), kTvSteps
// such groups 256 apart, all independent; a block whose range starts past
// its plane leaves at once (no loss term, no atomic).
constexpr int kTvSteps = 4;

__global__ __launch_bounds__(256) void k_tv4(TvPlanes P, float *__restrict__ loss) {
    const int p = blockIdx.y;
    const int na = P.na[p], nb = P.nb[p], F = P.feat;
    const int lq = F == 32 ? 3 : 2;   // log2 of the 4-channel groups per cell
    const uint32_t quads = (uint32_t)(na * nb) << lq;
    const uint32_t q0 = blockIdx.x * (256u * kTvSteps);
    if (q0 >= quads) return;
    const float4 *R = reinterpret_cast<const float4 *>(P.plane[p]);
    float4 *G = reinterpret_cast<float4 *>(P.grad[p]);
    const uint32_t f4 = 1u << lq, row4 = (uint32_t)na << lq;
    const float ia = 1.0f / (float)((size_t)nb * (na - 1) * F);
    const float ib = 1.0f / (float)((size_t)(nb - 1) * na * F);
    float acc = 0.0f;
#pragma unroll
    for (int k = 0; k < kTvSteps; ++k) {
        const uint32_t q = q0 + k * 256u + threadIdx.x;
        if (q < quads) {
            const uint32_t cell = q >> lq;
            const uint32_t i = cell / (uint32_t)na, j = cell - i * (uint32_t)na;
            const bool hr = j + 1 < (uint32_t)na, hl = j > 0, hd = i + 1 < (uint32_t)nb, hu = i > 0;
            const float4 r = R[q];
            const float4 z = make_float4(0.f, 0.f, 0.f, 0.f);
            const float4 rr = hr ? R[q + f4] : z, rl = hl ? R[q - f4] : z;
            const float4 rd = hd ? R[q + row4] : z, ru = hu ? R[q - row4] : z;
            const float gx = tv_one(r.x, rr.x, rl.x, rd.x, ru.x, hr, hl, hd, hu, ia, ib, acc);
            const float gy = tv_one(r.y, rr.y, rl.y, rd.y, ru.y, hr, hl, hd, hu, ia, ib, acc);
            const float gz = tv_one(r.z, rr.z, rl.z, rd.z, ru.z, hr, hl, hd, hu, ia, ib, acc);
            const float gw = tv_one(r.w, rr.w, rl.w, rd.w, ru.w, hr, hl, hd, hu, ia, ib, acc);
            if (G) {
                float4 o = G[q];
                o.x += P.weight * gx;
                o.y += P.weight * gy;
                o.z += P.weight * gz;
                o.w += P.weight * gw;
                G[q] = o;
            }
        }
    }
    tv_block_loss(acc, P.weight, loss);
}

// Scalar form (any alignment): one value per thread, grid-stride.
__global__ __launch_bounds__(256) void k_tv(TvPlanes P, float *__restrict__ loss) {
    const int p = blockIdx.y;
    const int na = P.na[p], nb = P.nb[p], F = P.feat;
    const int lf = F == 32 ? 5 : 4;
    const float *R = P.plane[p];
    float *G = P.grad[p];
    const uint32_t cells = (uint32_t)(na * nb) << lf, row = (uint32_t)na << lf;
    const float ia = 1.0f / (float)((size_t)nb * (na - 1) * F);
    const float ib = 1.0f / (float)((size_t)(nb - 1) * na * F);
    float acc = 0.0f;
    for (uint32_t c = blockIdx.x * blockDim.x + threadIdx.x; c < cells; c += gridDim.x * blockDim.x) {
        const uint32_t cell = c >> lf;
        const uint32_t i = cell / (uint32_t)na, j = cell - i * (uint32_t)na;
        const bool hr = j + 1 < (uint32_t)na, hl = j > 0, hd = i + 1 < (uint32_t)nb, hu = i > 0;
        const float g = tv_one(R[c], hr ? R[c + F] : 0.0f, hl ? R[c - F] : 0.0f, hd ? R[c + row] : 0.0f,
                               hu ? R[c - row] : 0.0f, hr, hl, hd, hu, ia, ib, acc);
        if (G) G[c] += P.weight * g;
    }
    tv_block_loss(acc, P.weight, loss);
}

struct AdamList {
    float *param[64];
    const float *grad[64];
    float *m[64], *v[64];
    uint32_t count[64];
    float lr[64];
    int n;
    float b1, b2, eps, c1, c2;   // c1 = 1 / (1 - b1^t), c2 = 1 / (1 - b2^t)
};

__device__ __forceinline__ void adam_one(const AdamList &A, float lr, float &p, float &m, float &v, float g) {
    const float mi = A.b1 * m + (1.0f - A.b1) * g;
    const float vi = A.b2 * v + (1.0f - A.b2) * g * g;
    m = mi;
    v = vi;
    p -= lr * (mi * A.c1) / (sqrtf(vi * A.c2) + A.eps);
}

// Four consecutive values per thread (16-byte accesses) when all four arrays
// of the tensor are 16-byte aligned, the remainder (and unaligned tensors)
// one value per thread.
__global__ __launch_bounds__(256) void k_adam(AdamList A) {
    const int a = blockIdx.y;
    if (a >= A.n) return;
    float *p = A.param[a], *m = A.m[a], *v = A.v[a];
    const float *g = A.grad[a];
    const float lr = A.lr[a];
    const uint32_t count = A.count[a];
    const bool vec = ((reinterpret_cast<uintptr_t>(p) | reinterpret_cast<uintptr_t>(m) |
                       reinterpret_cast<uintptr_t>(v) | reinterpret_cast<uintptr_t>(g)) & 15u) == 0;
    const uint32_t n4 = vec ? count / 4 : 0;
    const uint32_t stride = gridDim.x * blockDim.x;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < n4; i += stride) {
        float4 pp = reinterpret_cast<float4 *>(p)[i], mm = reinterpret_cast<float4 *>(m)[i];
        float4 vv = reinterpret_cast<float4 *>(v)[i];
        const float4 gg = reinterpret_cast<const float4 *>(g)[i];
        adam_one(A, lr, pp.x, mm.x, vv.x, gg.x);
        adam_one(A, lr, pp.y, mm.y, vv.y, gg.y);
        adam_one(A, lr, pp.z, mm.z, vv.z, gg.z);
        adam_one(A, lr, pp.w, mm.w, vv.w, gg.w);
        reinterpret_cast<float4 *>(p)[i] = pp;
        reinterpret_cast<float4 *>(m)[i] = mm;
        reinterpret_cast<float4 *>(v)[i] = vv;
    }
    for (uint32_t i = 4 * n4 + blockIdx.x * blockDim.x + threadIdx.x; i < count; i += stride)
        adam_one(A, lr, p[i], m[i], v[i], g[i]);
}

__global__ void k_zero_scalar(float *p) { *p = 0.0f; }

}  // namespace
}  // namespace g4d

extern "C" g4d_status g4d_tv_loss(const g4d_planes *P, float weight, float *loss, g4d_deform_grad *grad,
                                  void *stream) {
    if (!P || P->n_scales < 1 || P->n_scales > 3 || (P->feat != 16 && P->feat != 32)) return G4D_EINVAL;
    if (!loss && !grad) return G4D_EINVAL;
    static const int ax[6][2] = {{0, 1}, {0, 2}, {1, 2}, {0, 3}, {1, 3}, {2, 3}};
    g4d::TvPlanes T{};
    size_t max_cells = 0;
    for (int l = 0; l < P->n_scales; ++l)
        for (int p = 0; p < 6; ++p) {
            const int q = l * 6 + p;
            if (!P->plane[l][p] || (grad && !grad->plane[l][p])) return G4D_EINVAL;
            T.plane[q] = P->plane[l][p];
            T.grad[q] = grad ? grad->plane[l][p] : nullptr;
            T.na[q] = P->res[l][ax[p][0]];
            T.nb[q] = P->res[l][ax[p][1]];
            if (T.na[q] < 2 || T.nb[q] < 2 || (size_t)T.na[q] * T.nb[q] * P->feat > 0x7fffffffu) return G4D_EINVAL;
            max_cells = std::max(max_cells, (size_t)T.na[q] * T.nb[q] * P->feat);
        }
    T.n_planes = P->n_scales * 6;
    T.feat = P->feat;
    T.weight = weight;
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    if (loss) hipLaunchKernelGGL(g4d::k_zero_scalar, dim3(1), dim3(1), 0, s, loss);
    bool aligned = true;
    for (int q = 0; q < T.n_planes; ++q)
        aligned = aligned && ((reinterpret_cast<uintptr_t>(T.plane[q]) | reinterpret_cast<uintptr_t>(T.grad[q])) & 15u) == 0;
    if (aligned) {
        // one block per 1024 four-channel groups of the largest plane; the
        // loss adds one atomic per block with work
        const unsigned bx = (unsigned)((max_cells / 4 + 256 * g4d::kTvSteps - 1) / (256 * g4d::kTvSteps));
        hipLaunchKernelGGL(g4d::k_tv4, dim3(bx, (unsigned)T.n_planes), dim3(256), 0, s, T, loss);
    } else {
        // up to 128 blocks per plane, grid-stride
        const unsigned bx = (unsigned)std::min<size_t>((max_cells + 255) / 256, 128);
        hipLaunchKernelGGL(g4d::k_tv, dim3(bx, (unsigned)T.n_planes), dim3(256), 0, s, T, loss);
    }
    G4D_HIP_CHECK(hipGetLastError());
    return G4D_OK;
}

extern "C" g4d_status g4d_adam_step(const g4d_adam_tensor *t, int32_t n, float beta1, float beta2, float eps,
                                    int32_t step, void *stream) {
    if (!t || n < 1 || n > 64 || step < 1 || !(beta1 >= 0.0f && beta1 < 1.0f) || !(beta2 >= 0.0f && beta2 < 1.0f))
        return G4D_EINVAL;
    g4d::AdamList A{};
    uint32_t most = 0;
    for (int i = 0; i < n; ++i) {
        if (!t[i].param || !t[i].grad || !t[i].m || !t[i].v || t[i].count < 0 || t[i].count > 0xffffffffLL)
            return G4D_EINVAL;
        A.param[i] = t[i].param; A.grad[i] = t[i].grad; A.m[i] = t[i].m; A.v[i] = t[i].v;
        A.count[i] = (uint32_t)t[i].count;
        A.lr[i] = t[i].lr;
        most = std::max(most, A.count[i]);
    }
    A.n = n;
    A.b1 = beta1; A.b2 = beta2; A.eps = eps;
    A.c1 = (float)(1.0 / (1.0 - std::pow((double)beta1, step)));
    A.c2 = (float)(1.0 / (1.0 - std::pow((double)beta2, step)));
    hipStream_t s = reinterpret_cast<hipStream_t>(stream);
    const unsigned bx = (unsigned)std::max<uint32_t>(1, std::min<uint32_t>((most / 4 + 255) / 256, 1024));
    hipLaunchKernelGGL(g4d::k_adam, dim3(bx, (unsigned)n), dim3(256), 0, s, A);
    G4D_HIP_CHECK(hipGetLastError());
    return G4D_OK;
}
