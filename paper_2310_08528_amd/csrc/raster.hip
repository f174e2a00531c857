// Tile rasterizer of the splatting renderer S(M, G') on gfx950
// (Sec. 3.1, Eq. 1-4; Sec. 4.1).
//
// Pipeline per frame (all on one stream, no host synchronisation):
//   k_zero        clear status words, digit histograms, look-back state, tile ranges
//   k_preprocess  per Gaussian: EWA projection (Eq. 2-3), cull, radius, tile
//                 rectangle, depth key, conic, SH colour; depth digit histograms
//   k_sort_pass x4  stable LSD radix sort of (depth bits, index) over Gaussians
//   k_scan_offsets  exclusive scan of tiles-per-Gaussian in depth order -> K
//   k_emit        one (tile id, Gaussian) instance per touched tile, in depth order
//                 (and counts the first tile digit per sort tile)
//   k_sort_up / k_spine / k_sort_down  x1-2  stable LSD radix sort of the
//                 instances by tile id (reduce-then-scan passes)
//   k_ranges      [start, end) of every tile in the sorted list
//   k_tile_order  blend order of the tiles, longest list first
//   k_blend       one 256-thread block per 16x16 tile: front-to-back compositing
//                 (Eq. 1, Eq. 4) over LDS-staged batches with early exit
//
// Sorting the depth digits before the fan-out to tiles is the same LSD radix
// sort of the 64-bit key (tile << 32) | depth_bits: every instance of a
// Gaussian carries the same depth digits, so the low-digit passes can run
// once per Gaussian (N keys) instead of once per instance (K keys); the
// remaining passes sort K instances by the tile digits only, stably.
//
// This translation unit is compiled without FMA contraction, with correctly
// rounded division and square root and without denormal flushing: the
// discrete structure (cull, radius, rectangle, depth key) and the per-pixel
// skip/stop decisions are fixed binary32 operation sequences.
#include "g4d_internal.h"

#include <vector>

namespace g4d {
namespace {

// ---------------------------------------------------------------- helpers

__device__ __forceinline__ uint32_t atomic_load_u32(const uint32_t *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_store_u32(uint32_t *p, uint32_t v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ unsigned long long atomic_load_u64(const unsigned long long *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_store_u64(unsigned long long *p, unsigned long long v) {
    __hip_atomic_store(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ uint64_t lanemask_lt64() {
    const int lane = __lane_id();
    return lane == 0 ? 0ull : (~0ull >> (64 - lane));
}

// Inclusive sum over the lanes of a wave (all 64 lanes active) with DPP:
// shifts by 1, 2, 4 and 8 inside each row of 16 lanes (lanes shifted in
// from outside the row read 0), then each row adds the last lane of the row
// before (row broadcast 15) and rows 2 and 3 the last lane of row 1
// (row broadcast 31).  No LDS round trips.
template <int CTRL, int ROW_MASK, bool BOUND0>
__device__ __forceinline__ uint32_t dpp_u32(uint32_t v) {
    return (uint32_t)__builtin_amdgcn_update_dpp(0, (int)v, CTRL, ROW_MASK, 0xf, BOUND0);
}
// (unsigned: sums wrap modulo 2^32)
__device__ __forceinline__ uint32_t wave_inclusive_sum(uint32_t v) {
    v += dpp_u32<0x111, 0xf, true>(v);   // row_shr:1
    v += dpp_u32<0x112, 0xf, true>(v);   // row_shr:2
    v += dpp_u32<0x114, 0xf, true>(v);   // row_shr:4
    v += dpp_u32<0x118, 0xf, true>(v);   // row_shr:8
    v += dpp_u32<0x142, 0xa, false>(v);  // row_bcast:15 into rows 1 and 3
    v += dpp_u32<0x143, 0xc, false>(v);  // row_bcast:31 into rows 2 and 3
    return v;
}

// Frame descriptor as the kernels read it: camera, background and output
// pointers.  It lives in the workspace: the first kernel of a render
// (k_zero) writes it from its launch argument, so a captured render graph
// takes a new view and new output buffers through that one node's
// parameters.
struct CamK {
    float v[12];
    float fx, fy, cx, cy, tanx, tany, near_plane;
    float campos[3];
    float bg[3];
    int width, height, tiles_x, tiles_y;
    float *image;
    float *final_T;
    int32_t *n_contrib;
};

// Tile-count difference grids of up to kGridLdsCells cells ((tiles_x + 1) x
// (tiles_y + 1), 64 KB) are accumulated in LDS per preprocess block.
constexpr int kGridLdsCells = 16384;
std::atomic<uint64_t> g_preprocess_lds{0};   // per device: the preprocess's dynamic-LDS limit raised
std::atomic<uint64_t> g_order_lds{0};        // per device: k_tile_order's dynamic-LDS limit raised

// ---------------------------------------------------------------- k_zero

__global__ void k_zero(uint4 *__restrict__ p, size_t n16, CamK cam, CamK *__restrict__ camd) {
    if (blockIdx.x == 0 && threadIdx.x == 0) *camd = cam;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0u, 0u, 0u, 0u);
}

// ---------------------------------------------------------------- k_preprocess

// Real SH basis constants (degree <= 3), Cartesian form on a unit direction.
#define SH_C0 0.28209479177387814f
#define SH_C1 0.4886025119029199f

__device__ __forceinline__ float3 sh_colour(int deg, const float (&c)[16][3], float x, float y, float z) {
    float r = SH_C0 * c[0][0], gg = SH_C0 * c[0][1], b = SH_C0 * c[0][2];
    if (deg >= 1) {
        const float y1 = -SH_C1 * y, y2 = SH_C1 * z, y3 = -SH_C1 * x;
        r += y1 * c[1][0] + y2 * c[2][0] + y3 * c[3][0];
        gg += y1 * c[1][1] + y2 * c[2][1] + y3 * c[3][1];
        b += y1 * c[1][2] + y2 * c[2][2] + y3 * c[3][2];
        if (deg >= 2) {
            const float xx = x * x, yy = y * y, zz = z * z, xy = x * y, yz = y * z, xz = x * z;
            const float Y[5] = {1.0925484305920792f * xy, -1.0925484305920792f * yz,
                                0.31539156525252005f * (2.0f * zz - xx - yy), -1.0925484305920792f * xz,
                                0.5462742152960396f * (xx - yy)};
#pragma unroll
            for (int k = 0; k < 5; ++k) {
                r += Y[k] * c[4 + k][0];
                gg += Y[k] * c[4 + k][1];
                b += Y[k] * c[4 + k][2];
            }
            if (deg >= 3) {
                const float Z[7] = {-0.5900435899266435f * y * (3.0f * xx - yy),
                                    2.890611442640554f * xy * z,
                                    -0.4570457994644658f * y * (4.0f * zz - xx - yy),
                                    0.3731763325901154f * z * (2.0f * zz - 3.0f * xx - 3.0f * yy),
                                    -0.4570457994644658f * x * (4.0f * zz - xx - yy),
                                    1.445305721320277f * z * (xx - yy),
                                    -0.5900435899266435f * x * (xx - 3.0f * yy)};
#pragma unroll
                for (int k = 0; k < 7; ++k) {
                    r += Z[k] * c[9 + k][0];
                    gg += Z[k] * c[9 + k][1];
                    b += Z[k] * c[9 + k][2];
                }
            }
        }
    }
    float3 out;
    out.x = fmaxf(r + 0.5f, 0.0f);
    out.y = fmaxf(gg + 0.5f, 0.0f);
    out.z = fmaxf(b + 0.5f, 0.0f);
    return out;
}

// Blend cull bounds of a Gaussian (stored with its record): every pixel
// offset d = (u - px, v - py) at which the blend can composite it (alpha >=
// 1/255 and power <= 0, as the blend evaluates them in binary32) lies in the
// ellipse q(d) = d^T K d <= thr_c, K the binary32 conic (A, B, C) and
// thr_c = 2 ln(255 o) widened by a margin: 1e-3 (1 + |thr|) for the
// exponential and logarithm roundings, and the factor (1 + 2 e) for the
// binary32 evaluation of q (about nine roundings, each relative to
// A dx^2 + 2|B dx dy| + C dy^2 <= q (1 + rho) / (1 - rho)), whose error is at
// most e q(d) with e = 16 u (1 + rho) / (1 - rho), rho = |B| / sqrt(AC), u = 2^-24.  From that
// ellipse: its half-extents hx = sqrt(thr_c (K^-1)_xx), hy = sqrt(thr_c
// (K^-1)_yy), and the reach of a pixel square of half-side 3.5 (a blend
// quadrant, inside a disc of radius r_b = 3.5 sqrt 2 about its centre c):
// if some pixel of the square can be composited then, K-norms being norms,
// sqrt(q(c)) <= sqrt(thr_c) + r_b sqrt(lambda_max(K)), so q(c) evaluated in
// binary32 is at most reach = (sqrt(thr_c) + r_b sqrt(lambda_max))^2 (1 + 2 e).
// Computed in double and rounded up.  A Gaussian that can never be
// composited (thr_c < 0) gets reach -1; one whose conic is too elongated for
// the bound (rho >= 0.999) is never culled (infinite bounds).
__device__ __forceinline__ float4 cull_bounds(float b, float A, float B, float C, float o) {
    const double thr = 2.0 * log(255.0 * (double)o);
    const double thr_m = thr + 1e-3 * (1.0 + fabs(thr));
    if (!(thr_m >= 0.0)) return make_float4(b, 0.0f, 0.0f, -1.0f);
    const double a = A, bb = B, c = C;
    const double rho = fabs(bb) / sqrt(a * c);
    if (!(a > 0.0 && c > 0.0 && rho < 0.999)) return make_float4(b, INFINITY, INFINITY, INFINITY);
    const double e = 16.0 * 0x1p-24 * (1.0 + rho) / (1.0 - rho);
    const double thr_c = thr_m * (1.0 + 2.0 * e);
    const double det = a * c - bb * bb;
    const double hx = sqrt(thr_c * c / det), hy = sqrt(thr_c * a / det);
    const double lmax = 0.5 * (a + c) + sqrt(0.25 * (a - c) * (a - c) + bb * bb);
    const double rb = 4.949747468305833;   // 3.5 sqrt 2
    const double r = sqrt(thr_c) + rb * sqrt(lmax);
    const double reach = r * r * (1.0 + 2.0 * e);
    return make_float4(b, (float)(hx * (1.0 + 1e-6) + 1e-3), (float)(hy * (1.0 + 1e-6) + 1e-3),
                       (float)(reach * (1.0 + 1e-6) + 1e-6));
}

// 1024 threads per block: the per-block depth-digit histograms are folded
// into the device-wide ones with device-scope atomics, whose count (and
// contention on the few live top-digit bins) falls with the block count.
__global__ __launch_bounds__(1024) void k_preprocess(int n, int sh_degree, const float *__restrict__ means,
                                                    const float *__restrict__ scales,
                                                    const float *__restrict__ quats,
                                                    const float *__restrict__ opac, const float *__restrict__ sh,
                                                    const CamK *__restrict__ camd, float4 *__restrict__ recA,
                                                    float4 *__restrict__ recB,
                                                    float4 *__restrict__ recC, uint2 *__restrict__ rect,
                                                    uint32_t *__restrict__ touched, uint32_t *__restrict__ dkeys,
                                                    uint32_t *__restrict__ depth_hist, DevStatus *__restrict__ st,
                                                    int32_t *__restrict__ tgrid, int grid_lds) {
    __shared__ uint32_t h[4][256];
    __shared__ uint32_t s_vis;
    extern __shared__ int32_t s_grid[];   // the block's difference grid, when it fits in LDS
    for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) (&h[0][0])[i] = 0;
    for (int i = threadIdx.x; i < grid_lds; i += blockDim.x) s_grid[i] = 0;
    if (threadIdx.x == 0) s_vis = 0;
    __syncthreads();
    const CamK cam = *camd;
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    bool vis = false;
    if (g < n) {
        uint32_t key = 0xffffffffu, cnt = 0;
        uint2 rc = make_uint2(0u, 0u);
        float4 A = make_float4(0.f, 0.f, 0.f, 0.f), B = A;
        float4 Cb = make_float4(0.f, 0.f, 0.f, -1.0f);
        const float mx = means[g], my = means[(size_t)n + g], mz = means[2 * (size_t)n + g];
        const float sx = scales[g], sy = scales[(size_t)n + g], sz = scales[2 * (size_t)n + g];
        const float qw = quats[g], qx = quats[(size_t)n + g], qy = quats[2 * (size_t)n + g],
                    qz = quats[3 * (size_t)n + g];
        const bool finite = isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(sx) && isfinite(sy) &&
                            isfinite(sz) && isfinite(qw) && isfinite(qx) && isfinite(qy) && isfinite(qz);
        const float *V = cam.v;
        const float px = ((V[0] * mx + V[1] * my) + V[2] * mz) + V[3];
        const float py = ((V[4] * mx + V[5] * my) + V[6] * mz) + V[7];
        const float pz = ((V[8] * mx + V[9] * my) + V[10] * mz) + V[11];
        if (finite && pz > cam.near_plane) {
            // SH coefficients, loaded before the projection so that their
            // latency overlaps it
            const int ncoef = (sh_degree + 1) * (sh_degree + 1);
            float coef[16][3];
#pragma unroll
            for (int k = 0; k < 16; ++k)
#pragma unroll
                for (int ch = 0; ch < 3; ++ch)
                    coef[k][ch] = k < ncoef ? sh[((size_t)k * 3 + ch) * n + g] : 0.0f;
            // Eq. 2: Sigma = R S S^T R^T
            const float xx = qx * qx, yy = qy * qy, zz = qz * qz;
            const float xy = qx * qy, xz = qx * qz, yz = qy * qz;
            const float wx = qw * qx, wy = qw * qy, wz = qw * qz;
            const float R00 = 1.0f - 2.0f * (yy + zz), R01 = 2.0f * (xy - wz), R02 = 2.0f * (xz + wy);
            const float R10 = 2.0f * (xy + wz), R11 = 1.0f - 2.0f * (xx + zz), R12 = 2.0f * (yz - wx);
            const float R20 = 2.0f * (xz - wy), R21 = 2.0f * (yz + wx), R22 = 1.0f - 2.0f * (xx + yy);
            const float M00 = R00 * sx, M01 = R01 * sy, M02 = R02 * sz;
            const float M10 = R10 * sx, M11 = R11 * sy, M12 = R12 * sz;
            const float M20 = R20 * sx, M21 = R21 * sy, M22 = R22 * sz;
            const float S00 = (M00 * M00 + M01 * M01) + M02 * M02;
            const float S01 = (M00 * M10 + M01 * M11) + M02 * M12;
            const float S02 = (M00 * M20 + M01 * M21) + M02 * M22;
            const float S11 = (M10 * M10 + M11 * M11) + M12 * M12;
            const float S12 = (M10 * M20 + M11 * M21) + M12 * M22;
            const float S22 = (M20 * M20 + M21 * M21) + M22 * M22;
            // Eq. 3: Sigma' = J W Sigma W^T J^T, J at the (clamped) camera-space mean
            const float limx = 1.3f * cam.tanx, limy = 1.3f * cam.tany;
            const float rx = px / pz, ry = py / pz;
            const float tx = fminf(limx, fmaxf(-limx, rx)) * pz;
            const float ty = fminf(limy, fmaxf(-limy, ry)) * pz;
            const float z2 = pz * pz;
            const float j00 = cam.fx / pz, j02 = -((cam.fx * tx) / z2);
            const float j11 = cam.fy / pz, j12 = -((cam.fy * ty) / z2);
            const float T00 = j00 * V[0] + j02 * V[8], T01 = j00 * V[1] + j02 * V[9], T02 = j00 * V[2] + j02 * V[10];
            const float T10 = j11 * V[4] + j12 * V[8], T11 = j11 * V[5] + j12 * V[9], T12 = j11 * V[6] + j12 * V[10];
            const float U00 = (T00 * S00 + T01 * S01) + T02 * S02;
            const float U01 = (T00 * S01 + T01 * S11) + T02 * S12;
            const float U02 = (T00 * S02 + T01 * S12) + T02 * S22;
            const float U10 = (T10 * S00 + T11 * S01) + T12 * S02;
            const float U11 = (T10 * S01 + T11 * S11) + T12 * S12;
            const float U12 = (T10 * S02 + T11 * S12) + T12 * S22;
            float ca = (U00 * T00 + U01 * T01) + U02 * T02;
            const float cb = (U00 * T10 + U01 * T11) + U02 * T12;
            float cc = (U10 * T10 + U11 * T11) + U12 * T12;
            ca = ca + 0.3f;
            cc = cc + 0.3f;
            const float det = ca * cc - cb * cb;
            if (det > 0.0f) {
                const float mid = 0.5f * (ca + cc);
                const float disc = fmaxf(0.1f, mid * mid - det);
                const float lam = mid + sqrtf(disc);
                const float rad = ceilf(3.0f * sqrtf(lam));
                const float u = cam.fx * rx + cam.cx;
                const float v = cam.fy * ry + cam.cy;
                if (isfinite(u) && isfinite(v) && isfinite(rad)) {
                    const float fx0 = floorf((u - rad) * 0.0625f);
                    const float fx1 = floorf((u + rad) * 0.0625f) + 1.0f;
                    const float fy0 = floorf((v - rad) * 0.0625f);
                    const float fy1 = floorf((v + rad) * 0.0625f) + 1.0f;
                    const int x0 = (int)fminf(fmaxf(fx0, 0.0f), (float)cam.tiles_x);
                    const int x1 = (int)fminf(fmaxf(fx1, 0.0f), (float)cam.tiles_x);
                    const int y0 = (int)fminf(fmaxf(fy0, 0.0f), (float)cam.tiles_y);
                    const int y1 = (int)fminf(fmaxf(fy1, 0.0f), (float)cam.tiles_y);
                    if (x1 > x0 && y1 > y0) {
                        vis = true;
                        cnt = (uint32_t)((x1 - x0) * (y1 - y0));
                        rc = make_uint2((uint32_t)x0 | ((uint32_t)y0 << 16), (uint32_t)x1 | ((uint32_t)y1 << 16));
                        key = __float_as_uint(pz);
                        const float inv = 1.0f / det;
                        const float cA = cc * inv, cB = -(cb * inv), cC = ca * inv;
                        // view-dependent colour from SH at the deformed mean
                        float dx = mx - cam.campos[0], dy = my - cam.campos[1], dz = mz - cam.campos[2];
                        const float il = 1.0f / sqrtf(dx * dx + dy * dy + dz * dz);
                        dx *= il; dy *= il; dz *= il;
                        const float3 col = sh_colour(sh_degree, coef, dx, dy, dz);
                        const float o = opac[g];
                        A = make_float4(u, v, -0.5f * cA, -0.5f * cC);
                        B = make_float4(-cB, o, col.x, col.y);
                        Cb = cull_bounds(col.z, cA, cB, cC, o);
                    }
                }
            }
        }
        recA[g] = A;
        recB[g] = B;
        recC[g] = Cb;
        rect[g] = rc;
        touched[g] = cnt;
        dkeys[g] = key;   // per-Gaussian depth key (kept for export and as the first sort input)
        if (cnt) {
            // the tile rectangle into the difference grid: its 2D prefix sum
            // is the number of instances of each tile
            const int x0 = rc.x & 0xffff, y0 = rc.x >> 16, x1 = rc.y & 0xffff, y1 = rc.y >> 16;
            const int gw = cam.tiles_x + 1;
            int32_t *gr = grid_lds ? s_grid : tgrid;
            atomicAdd(&gr[y0 * gw + x0], 1);
            atomicAdd(&gr[y0 * gw + x1], -1);
            atomicAdd(&gr[y1 * gw + x0], -1);
            atomicAdd(&gr[y1 * gw + x1], 1);
        }
        atomicAdd(&h[0][key & 255u], 1u);
        atomicAdd(&h[1][(key >> 8) & 255u], 1u);
        atomicAdd(&h[2][(key >> 16) & 255u], 1u);
        atomicAdd(&h[3][key >> 24], 1u);
    }
    const uint64_t vb = __ballot(vis);
    if (__lane_id() == 0 && vb) atomicAdd(&s_vis, (uint32_t)__popcll(vb));
    __syncthreads();
    for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) {
        const uint32_t c = (&h[0][0])[i];
        if (c) atomicAdd(&depth_hist[i], c);
    }
    for (int i = threadIdx.x; i < grid_lds; i += blockDim.x) {
        const int32_t c = s_grid[i];
        if (c) atomicAdd(&tgrid[i], c);
    }
    if (threadIdx.x == 0 && s_vis) atomicAdd(&st->visible, s_vis);
}

// ---------------------------------------------------------------- k_sort_pass
//
// One stable LSD radix pass over (key, value) pairs with a `bits`-wide digit
// at `shift` (onesweep: global digit counts are known in advance; blocks take
// tiles in launch order from a ticket counter and chain their per-digit
// counts through a decoupled look-back).  Each wave ranks a contiguous 1024-
// key sub-tile: wave-wide digit matching with ballots, running per-wave digit
// counters in LDS.  Waits are bounded; a wait that gives up sets sort_error.
//
// Depth sort routing: pass p of the four 8-bit passes over the per-Gaussian
// depth keys.  A pass whose digit is the same for every key (its histogram
// has one bin holding all n keys) is the identity permutation and is skipped
// outright; the m passes that remain alternate between the two ping-pong
// buffers so that the last one writes buffer 0 (the depth order), the first
// reading the depth keys with the identity as values.  Every block derives
// the same routing from the four histograms, which the preprocess completed.
// With m = 0 (all keys equal) pass 3 writes the identity order itself.

template <int ITEMS>
__global__ __launch_bounds__(kSortThreads) void k_sort_pass(
    int n, int p, const uint32_t *__restrict__ dgid, uint32_t *__restrict__ dk0, uint32_t *__restrict__ dk1,
    uint32_t *__restrict__ dv0, uint32_t *__restrict__ dv1, const uint32_t *__restrict__ hist4,
    uint32_t *__restrict__ lookback, uint32_t *__restrict__ ticket, uint32_t *__restrict__ err) {
    __shared__ uint32_t s_wcnt[4][256];
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_g[256];
    __shared__ uint32_t s_tile;
    __shared__ int s_triv[4];
    constexpr uint32_t TILE = kSortThreads * ITEMS;
    constexpr int bits = 8;
    const int shift = 8 * p;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int NB = 1 << bits;
    const uint32_t mask = (uint32_t)NB - 1u;
    const uint32_t count = (uint32_t)n;
    if (tid < 4) s_triv[tid] = 0;
    for (int i = tid; i < 4 * 256; i += kSortThreads) (&s_wcnt[0][0])[i] = 0;
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const uint32_t h = hist4[q * 256 + tid];
        if (q == p) s_g[tid] = h;
        if (h == count) s_triv[q] = 1;   // every key has this digit
    }
    __syncthreads();
    int m = 0, pidx = 0;   // non-trivial passes, and those before this one
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        m += !s_triv[q];
        pidx += q < p && !s_triv[q];
    }
    uint32_t *bk[2] = {dk0, dk1};
    uint32_t *bv[2] = {dv0, dv1};
    if (s_triv[p]) {
        if (m == 0 && p == 3) {
            for (uint32_t i = blockIdx.x * kSortThreads + tid; i < count; i += gridDim.x * kSortThreads) {
                dk0[i] = dgid[i];
                dv0[i] = i;
            }
        }
        return;
    }
    const uint32_t *kin = pidx == 0 ? dgid : bk[(m - pidx) & 1];
    const uint32_t *vin = pidx == 0 ? nullptr : bv[(m - pidx) & 1];
    uint32_t *kout = bk[(m - 1 - pidx) & 1];
    uint32_t *vout = bv[(m - 1 - pidx) & 1];
    if (tid == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t ntiles = (count + TILE - 1) / TILE;
    if (tile >= ntiles) return;

    uint32_t keys[ITEMS], vals[ITEMS], rank[ITEMS];
    const uint32_t base_idx = tile * TILE + wave * (ITEMS * 64);
    const uint64_t lt = lanemask_lt64();
    // issue every load of the tile before ranking (independent of each other)
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = base_idx + r * 64 + lane;
        keys[r] = idx < count ? kin[idx] : 0u;
    }
    if (vin) {
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) {
            const uint32_t idx = base_idx + r * 64 + lane;
            vals[r] = idx < count ? vin[idx] : 0u;
        }
    } else {
#pragma unroll
        for (int r = 0; r < ITEMS; ++r) vals[r] = base_idx + r * 64 + lane;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = base_idx + r * 64 + lane;
        const bool valid = idx < count;
        const uint32_t k = keys[r];
        const uint32_t d = (k >> shift) & mask;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        uint32_t old = 0;
        if (valid) old = s_wcnt[wave][d];
        if (valid && (peers & lt) == 0) s_wcnt[wave][d] = old + (uint32_t)__popcll(peers);
        rank[r] = old + (uint32_t)__popcll(peers & lt);
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // Per-digit totals and per-wave exclusive prefixes of this tile.
    __shared__ uint32_t s_tot[256];
    if (tid < NB) {
        const int d = tid;
        const uint32_t t0 = s_wcnt[0][d], t1 = s_wcnt[1][d], t2 = s_wcnt[2][d], t3 = s_wcnt[3][d];
        const uint32_t total = t0 + t1 + t2 + t3;
        s_wcnt[0][d] = 0;
        s_wcnt[1][d] = t0;
        s_wcnt[2][d] = t0 + t1;
        s_wcnt[3][d] = t0 + t1 + t2;
        s_tot[d] = total;
        // publish early so that successors can proceed
        atomic_store_u32(lookback + (size_t)tile * NB + d,
                         ((tile == 0 ? kFlagInclusive : kFlagAggregate) << kFlagShift) | total);
    }
    __syncthreads();
    // Windowed look-back: LB = 256 / NB consecutive threads per digit; thread
    // k of a digit reads predecessors at distances k, k + LB, k + 2 LB, k + 3 LB
    // (four independent loads), so a step covers 4 LB predecessors; the
    // nearest inclusive prefix ends the walk.
    {
        const int LB = min(kSortThreads / NB, 64);   // a group never spans two waves
        constexpr int M = 4;
        const int d = tid / LB, k = tid % LB;
        uint32_t excl = 0;
        if (tile > 0 && d < NB) {
            int j = (int)tile - 1;
            while (true) {
                uint32_t stv[M];
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const int jj = j - k - LB * m;
                    stv[m] = (kFlagInclusive << kFlagShift);   // before tile 0: inclusive zero
                    if (jj >= 0) stv[m] = atomic_load_u32(lookback + (size_t)jj * NB + d);
                }
#pragma unroll
                for (int m = 0; m < M; ++m) {
                    const int jj = j - k - LB * m;
                    uint32_t spins = 0;
                    while ((stv[m] >> kFlagShift) == 0u && spins < kSpinLimit) {
                        __builtin_amdgcn_s_sleep(1);
                        stv[m] = atomic_load_u32(lookback + (size_t)jj * NB + d);
                        ++spins;
                    }
                    if ((stv[m] >> kFlagShift) == 0u) {
                        atomicOr(err, 1u);
                        stv[m] = (kFlagInclusive << kFlagShift);
                    }
                }
                // nearest inclusive entry of this thread, then of the group
                int near = 1 << 30;
#pragma unroll
                for (int m = M - 1; m >= 0; --m)
                    if ((stv[m] >> kFlagShift) == kFlagInclusive) near = k + LB * m;
                for (int o = 1; o < LB; o <<= 1) near = min(near, __shfl_xor(near, o, 64));
                uint32_t v = 0;
#pragma unroll
                for (int m = 0; m < M; ++m)
                    if (k + LB * m <= near) v += stv[m] & kValueMask;
                for (int o = 1; o < LB; o <<= 1) v += __shfl_xor(v, o, 64);
                excl += v;
                if (near < (1 << 30)) break;
                j -= LB * M;
            }
        }
        if (tile > 0 && d < NB && k == 0)
            atomic_store_u32(lookback + (size_t)tile * NB + d, (kFlagInclusive << kFlagShift) | (excl + s_tot[d]));
        if (d < NB && k == 0) s_base[d] = excl;
    }
    __syncthreads();
    // global exclusive digit prefix (over all keys) and this tile's exclusive
    // digit prefix, by block scans over the NB digits
    {
        const uint32_t g = tid < NB ? s_g[tid] : 0u;
        const uint32_t t = tid < NB ? s_tot[tid] : 0u;
        const uint32_t gi = wave_inclusive_sum(g), ti = wave_inclusive_sum(t);
        __shared__ uint32_t s_wg[4], s_wt[4];
        if (lane == 63) {
            s_wg[wave] = gi;
            s_wt[wave] = ti;
        }
        __syncthreads();
        uint32_t go = 0, to = 0;
        for (int w = 0; w < wave; ++w) {
            go += s_wg[w];
            to += s_wt[w];
        }
        if (tid < NB) {
            s_base[tid] += go + gi - g;          // where digit tid starts in the output, for this tile
            s_tot[tid] = to + ti - t;            // where digit tid starts inside this tile
        }
        // the digit counts must account for every key exactly
        if (tid == NB - 1 && tile == 0 && go + gi != count) atomicOr(err, 8u);
    }
    __syncthreads();
    // Reorder the tile by digit in LDS, then write runs of equal digits with
    // consecutive threads to consecutive addresses.
    __shared__ uint32_t s_k[TILE], s_v[TILE];
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = base_idx + r * 64 + lane;
        if (idx < count) {
            const uint32_t d = (keys[r] >> shift) & mask;
            const uint32_t lpos = s_tot[d] + s_wcnt[wave][d] + rank[r];
            s_k[lpos] = keys[r];
            s_v[lpos] = vals[r];
        }
    }
    __syncthreads();
    const uint32_t in_tile = min(TILE, count - tile * TILE);
    for (uint32_t li = tid; li < in_tile; li += kSortThreads) {
        const uint32_t k = s_k[li];
        const uint32_t d = (k >> shift) & mask;
        const uint32_t pos = s_base[d] + (li - s_tot[d]);
        if (pos < count) {
            kout[pos] = k;
            vout[pos] = s_v[li];
        } else {
            atomicOr(err, 4u);   // inconsistent counts: never write out of bounds
        }
    }
}

// ---------------------------------------------------------------- k_morton
//
// Morton codes of the canonical means for a spatial processing order of the
// deformation: 10 bits per axis over the box, interleaved (x highest), with
// the four byte histograms of the codes for the radix passes.

__device__ __forceinline__ uint32_t spread10(uint32_t v) {
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000ffu;
    v = (v | (v << 8)) & 0x0300f00fu;
    v = (v | (v << 4)) & 0x030c30c3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}

__global__ __launch_bounds__(1024) void k_morton(int n, const float *__restrict__ means, float bx, float by,
                                                 float bz, float sx, float sy, float sz,
                                                 uint32_t *__restrict__ codes, uint32_t *__restrict__ hist4) {
    __shared__ uint32_t h[4][256];
    for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) (&h[0][0])[i] = 0;
    __syncthreads();
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g < n) {
        auto cell = [](float x, float b, float sc) -> uint32_t {
            return (uint32_t)fminf(fmaxf((x - b) * sc, 0.0f), 1023.0f);   // a NaN maps to 0
        };
        const uint32_t qx = cell(means[g], bx, sx), qy = cell(means[(size_t)n + g], by, sy);
        const uint32_t qz = cell(means[2 * (size_t)n + g], bz, sz);
        const uint32_t code = (spread10(qx) << 2) | (spread10(qy) << 1) | spread10(qz);
        codes[g] = code;
        atomicAdd(&h[0][code & 255u], 1u);
        atomicAdd(&h[1][(code >> 8) & 255u], 1u);
        atomicAdd(&h[2][(code >> 16) & 255u], 1u);
        atomicAdd(&h[3][code >> 24], 1u);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < 4 * 256; i += blockDim.x) {
        const uint32_t c = (&h[0][0])[i];
        if (c) atomicAdd(&hist4[i], c);
    }
}

// ---------------------------------------------------------------- k_scan_offsets
//
// offsets[i] = sum_{j < i} touched[order[j]] (64-bit), single pass with a
// decoupled look-back over 4096-element tiles; the last tile records the
// total K and the capacity verdict.

constexpr unsigned long long kF64Agg = 1ull << 62;
constexpr unsigned long long kF64Inc = 2ull << 62;
constexpr unsigned long long kV64Mask = (1ull << 62) - 1ull;

__global__ __launch_bounds__(256) void k_scan_offsets(int n, const uint32_t *__restrict__ order,
                                                      const uint32_t *__restrict__ touched,
                                                      unsigned long long *__restrict__ offsets,
                                                      unsigned long long *__restrict__ lookback,
                                                      uint32_t *__restrict__ ticket, DevStatus *__restrict__ st,
                                                      uint32_t capacity) {
    __shared__ unsigned long long s_w[4];
    __shared__ unsigned long long s_prefix;
    __shared__ uint32_t s_tile;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (tid == 0) s_tile = atomicAdd(ticket, 1u);
    __syncthreads();
    const uint32_t tile = s_tile;
    const uint32_t ntiles = ((uint32_t)n + kScanTile - 1) / kScanTile;
    if (tile >= ntiles) return;
    // 16 consecutive items per thread (64-byte aligned: whole-vector loads)
    const uint32_t base = tile * kScanTile + tid * 16;
    uint32_t v[16], gs[16];
    if (base + 16 <= (uint32_t)n) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const uint4 q = *reinterpret_cast<const uint4 *>(order + base + 4 * r);
            gs[4 * r] = q.x; gs[4 * r + 1] = q.y; gs[4 * r + 2] = q.z; gs[4 * r + 3] = q.w;
        }
    } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) gs[r] = base + r < (uint32_t)n ? order[base + r] : 0xffffffffu;
    }
#pragma unroll
    for (int r = 0; r < 16; ++r) v[r] = gs[r] < (uint32_t)n ? touched[gs[r]] : 0u;
    // wave inclusive scan of per-thread sums: a Gaussian touches at most
    // 65536 tiles (the largest frame), so a wave's 1024 Gaussians sum to
    // below 2^26 and the scan runs in 32 bits
    uint32_t sum32 = 0;
#pragma unroll
    for (int r = 0; r < 16; ++r) sum32 += v[r];
    const unsigned long long sum = sum32;
    const unsigned long long x = wave_inclusive_sum(sum32);
    if (lane == 63) s_w[wave] = x;
    __syncthreads();
    unsigned long long wpre = 0, btotal = 0;
    for (int w = 0; w < 4; ++w) {
        if (w < wave) wpre += s_w[w];
        btotal += s_w[w];
    }
    // decoupled look-back, one wave reading up to 64 predecessors at once:
    // sum the aggregates back to the nearest inclusive prefix
    if (wave == 0) {
        unsigned long long *mine = lookback + tile;
        unsigned long long excl = 0;
        if (tile == 0) {
            if (lane == 0) atomic_store_u64(mine, kF64Inc | btotal);
        } else {
            if (lane == 0) atomic_store_u64(mine, kF64Agg | btotal);
            int j = (int)tile - 1;   // nearest predecessor not yet summed
            uint32_t spins = 0;
            while (true) {
                const int idx = j - lane;
                const unsigned long long sv = idx >= 0 ? atomic_load_u64(lookback + idx) : kF64Inc;
                const uint64_t inc = __ballot((sv & kF64Inc) != 0ull);
                const uint64_t none = __ballot((sv >> 62) == 0ull);
                const int first_inc = inc ? __ffsll((long long)inc) - 1 : 64;
                const uint64_t need = first_inc < 63 ? (2ull << first_inc) - 1ull : ~0ull;
                if (none & need) {
                    if (++spins >= kSpinLimit) {
                        if (lane == 0) atomicOr(&st->sort_error, 2u);
                        break;
                    }
                    __builtin_amdgcn_s_sleep(1);
                    continue;
                }
                unsigned long long part = lane <= first_inc ? (sv & kV64Mask) : 0ull;
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) part += __shfl_xor(part, o, 64);
                excl += part;
                if (first_inc < 64) break;
                j -= 64;
            }
            if (lane == 0) atomic_store_u64(mine, kF64Inc | (excl + btotal));
        }
        if (lane == 0) {
            s_prefix = excl;
            if (tile == ntiles - 1) {
                const unsigned long long K = excl + btotal;
                st->k_total = K;
                st->k_used = (uint32_t)(K < capacity ? K : capacity);
                st->overflow = K > capacity ? 1u : 0u;
            }
        }
    }
    __syncthreads();
    unsigned long long run = s_prefix + wpre + (x - sum);
    if (base + 16 <= (uint32_t)n) {
#pragma unroll
        for (int r = 0; r < 8; ++r) {
            ulonglong2 q;
            q.x = run;
            run += v[2 * r];
            q.y = run;
            run += v[2 * r + 1];
            *reinterpret_cast<ulonglong2 *>(offsets + base + 2 * r) = q;
        }
    } else {
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const uint32_t i = base + r;
            if (i < (uint32_t)n) offsets[i] = run;
            run += v[r];
        }
    }
}

// ---------------------------------------------------------------- k_emit
//
// Load-balanced fan-out: wave w writes instance slots [512 w, 512 (w+1)),
// whatever Gaussians they belong to.  It finds the Gaussian (in depth order)
// owning its first slot with a 64-way cooperative search over the offsets,
// then walks batches of 64 consecutive Gaussians; within a batch each lane
// finds the owner of its slot by a binary search over the batch's offsets
// (shuffles).  Stores are coalesced.  (Nearby Gaussians, first in depth
// order, cover thousands of tiles, so balancing by Gaussian would not do.)

constexpr int kEmitSlots = 512;    // instance slots per wave

// The work of one wave: slots [512 w, 512 (w+1)) below K, counting the
// low tile digit of each instance (consecutive slots of a Gaussian are
// consecutive tiles of a row, so the lanes hit different LDS words).
__device__ __forceinline__ void emit_wave(int n, const uint32_t *__restrict__ order,
                                          const unsigned long long *__restrict__ offsets,
                                          const uint2 *__restrict__ rect, int tiles_x,
                                          const DevStatus *__restrict__ st, uint32_t *__restrict__ tkeys,
                                          uint32_t *__restrict__ tvals, int pack_bits, int bits0, uint32_t *h0) {
    const int lane = threadIdx.x & 63;
    const unsigned long long K = st->k_used;
    const unsigned long long s0 = ((unsigned long long)blockIdx.x * 4 + (threadIdx.x >> 6)) * kEmitSlots;
    if (s0 >= K || n <= 0) return;   // wave-uniform
    const unsigned long long s1 = min(s0 + (unsigned long long)kEmitSlots, K);
    // last Gaussian i with offsets[i] <= s0 (offsets[0] == 0)
    int lo = 0, hi = n;
    while (hi - lo > 64) {
        const int step = (hi - lo + 63) / 64;
        const int p = lo + lane * step;
        const bool ok = p < hi && offsets[p] <= s0;
        const int c = (int)__popcll(__ballot(ok));   // lanes 0..c-1 (lane 0 always)
        lo = lo + (c - 1) * step;
        hi = min(hi, lo + step);
    }
    {
        const bool ok = lo + lane < hi && offsets[lo + lane] <= s0;
        lo = lo + (int)__popcll(__ballot(ok)) - 1;
    }
    unsigned long long cur = s0;
    for (int ib = lo; cur < s1 && ib < n; ib += 64) {
        const int i = ib + lane;
        uint32_t g = 0xffffffffu;
        int x0 = 0, y0 = 0, w = 1, rel = 0x7fffffff;
        if (i < n) {
            g = order[i];
            if (g < (uint32_t)n) {
                const uint2 rc = rect[g];
                x0 = rc.x & 0xffff;
                y0 = rc.x >> 16;
                w = max((int)(rc.y & 0xffff) - x0, 1);
            }
            rel = (int)((long long)offsets[i] - (long long)s0);   // |rel| < 2^30
        }
        // the batch covers slots up to the next batch's first offset
        const int next = ib + 64 < n ? (int)((long long)offsets[ib + 64] - (long long)s0) : (int)(K - s0);
        const unsigned long long bend = min(s1, s0 + (unsigned long long)max(next, 0));
        for (unsigned long long c0 = cur; c0 < bend; c0 += 64) {
            const int j = (int)(c0 - s0) + lane;
            int ow = 0;
#pragma unroll
            for (int step = 32; step >= 1; step >>= 1) {
                const int cand = ow + step;
                const int e = __shfl(rel, cand < 64 ? cand : 63, 64);
                if (cand < 64 && e <= j) ow = cand;
            }
            const int r = j - __shfl(rel, ow, 64);
            const int ww = __shfl(w, ow, 64);
            const int ox = __shfl(x0, ow, 64);
            const int oy = __shfl(y0, ow, 64);
            const uint32_t og = __shfl(g, ow, 64);
            const unsigned long long o = s0 + (unsigned long long)j;
            const bool live = o < bend;
            uint32_t t = 0xffffffffu;
            if (live) {
                // r / ww by a float reciprocal, corrected to the exact quotient
                // (r < 2^16 and ww <= 256 tiles: the estimate is within one)
                int ry = (int)((float)r * __builtin_amdgcn_rcpf((float)ww));
                ry += (ry + 1) * ww <= r;
                ry -= ry * ww > r;
                t = (uint32_t)((oy + ry) * tiles_x + ox + (r - ry * ww));
                if (pack_bits) {
                    tkeys[o] = (t << pack_bits) | og;
                } else {
                    tkeys[o] = t;
                    tvals[o] = og;
                }
                atomicAdd(&h0[t & ((1u << bits0) - 1u)], 1u);
            }
        }
        cur = bend;
    }
}

static_assert(4 * kEmitSlots == kSortTile, "an emit block must cover exactly one sort tile");

__global__ __launch_bounds__(256) void k_emit(int n, const uint32_t *__restrict__ order,
                                              const unsigned long long *__restrict__ offsets,
                                              const uint2 *__restrict__ rect, int tiles_x,
                                              const DevStatus *__restrict__ st, uint32_t *__restrict__ tkeys,
                                              uint32_t *__restrict__ tvals, int pack_bits, int bits0,
                                              uint32_t *__restrict__ cnt, int cnt_stride) {
    __shared__ uint32_t h0[256];
    for (int q = threadIdx.x; q < 256; q += blockDim.x) h0[q] = 0;
    __syncthreads();
    emit_wave(n, order, offsets, rect, tiles_x, st, tkeys, tvals, pack_bits, bits0, h0);
    __syncthreads();
    // this block's digit counts for the first instance-sort pass (its slots
    // are exactly sort tile blockIdx.x)
    for (int q = threadIdx.x; q < (1 << bits0); q += blockDim.x) cnt[(size_t)q * cnt_stride + blockIdx.x] = h0[q];
}

// ---------------------------------------------------------------- instance sort
//
// Reduce-then-scan LSD passes over the K instances by tile digit: per-tile
// digit counts (the first pass's from k_emit, later ones from k_sort_up), a
// per-digit exclusive scan over the tiles (k_spine), then k_sort_down ranks
// each tile stably and scatters it.  No block waits on another.

// counts of `bits`-wide digits at `shift` in sort tile blockIdx.x
__global__ __launch_bounds__(kSortThreads) void k_sort_up(const uint32_t *__restrict__ kin,
                                                          const DevStatus *__restrict__ st, uint32_t cap,
                                                          int shift, int bits, uint32_t *__restrict__ cnt,
                                                          int cnt_stride) {
    if (st->overflow) return;
    __shared__ uint32_t h[256];
    const int NB = 1 << bits;
    const uint32_t count = min(st->k_used, cap);
    const uint32_t tile = blockIdx.x;
    if (tile * (uint32_t)kSortTile >= count) return;
    for (int q = threadIdx.x; q < NB; q += blockDim.x) h[q] = 0;
    __syncthreads();
    uint32_t k[kSortItems];
#pragma unroll
    for (int r = 0; r < kSortItems; ++r) {
        const uint32_t idx = tile * kSortTile + r * kSortThreads + threadIdx.x;
        k[r] = idx < count ? kin[idx] : 0xffffffffu;
    }
#pragma unroll
    for (int r = 0; r < kSortItems; ++r)
        if (k[r] != 0xffffffffu) atomicAdd(&h[(k[r] >> shift) & (uint32_t)(NB - 1)], 1u);
    __syncthreads();
    for (int q = threadIdx.x; q < NB; q += blockDim.x) cnt[(size_t)q * cnt_stride + tile] = h[q];
}

// per digit (one block each): exclusive scan of its counts over the live
// tiles, in place, and the digit's total.  Each thread sums a run of 16
// counts, the block scans the 256 run sums, and the runs are rewritten.
__global__ __launch_bounds__(256) void k_spine(uint32_t *__restrict__ cnt, int cnt_stride, int NB,
                                               const DevStatus *__restrict__ st, uint32_t cap,
                                               uint32_t *__restrict__ dtot) {
    if (st->overflow) return;
    const int d = blockIdx.x;
    if (d >= NB) return;
    __shared__ uint32_t s_w[4];
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint32_t count = min(st->k_used, cap);
    const int nlive = (int)((count + kSortTile - 1) / kSortTile);
    uint32_t *row = cnt + (size_t)d * cnt_stride;
    constexpr int R = 16;
    uint32_t carry = 0;
    for (int s0 = 0; s0 < nlive; s0 += 256 * R) {
        const int b = s0 + tid * R;
        uint32_t v[R];
        uint32_t sum = 0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            v[r] = b + r < nlive ? row[b + r] : 0u;
            sum += v[r];
        }
        const uint32_t x = wave_inclusive_sum(sum);
        if (lane == 63) s_w[wave] = x;
        __syncthreads();
        uint32_t before = carry;
        for (int w = 0; w < wave; ++w) before += s_w[w];
        const uint32_t seg_total = s_w[0] + s_w[1] + s_w[2] + s_w[3];
        uint32_t run = before + x - sum;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            if (b + r < nlive) row[b + r] = run;
            run += v[r];
        }
        carry += seg_total;
        __syncthreads();   // s_w is rewritten by the next segment
    }
    if (tid == 0) dtot[d] = carry;
}

// PACKED: an instance is one word (tile << pack_bits) | index; no value array
template <int ITEMS, bool PACKED>
__global__ __launch_bounds__(kSortThreads) void k_sort_down(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout, const DevStatus *__restrict__ st, uint32_t cap, int shift, int bits,
    const uint32_t *__restrict__ cnt, int cnt_stride, const uint32_t *__restrict__ dtot,
    uint32_t *__restrict__ err) {
    if (st->overflow) return;   // an overflowed frame is invalid; reads below stay in bounds
    constexpr uint32_t TILE = kSortThreads * ITEMS;
    __shared__ uint32_t s_wcnt[4][256];
    __shared__ uint32_t s_base[256];
    __shared__ uint32_t s_tot[256];
    __shared__ uint32_t s_wg[4], s_wt[4];
    __shared__ uint32_t s_k[TILE];
    __shared__ uint32_t s_v[PACKED ? 1 : TILE];
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int NB = 1 << bits;
    const uint32_t mask = (uint32_t)NB - 1u;
    const uint32_t count = min(st->k_used, cap);
    const uint32_t tile = blockIdx.x;
    if (tile * TILE >= count) return;
    for (int i = tid; i < 4 * 256; i += kSortThreads) (&s_wcnt[0][0])[i] = 0;
    __syncthreads();
    uint32_t keys[ITEMS], vals[ITEMS], rank[ITEMS];
    const uint32_t base_idx = tile * TILE + wave * (ITEMS * 64);
    const uint64_t lt = lanemask_lt64();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = base_idx + r * 64 + lane;
        keys[r] = idx < count ? kin[idx] : 0u;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = base_idx + r * 64 + lane;
        vals[r] = !PACKED && idx < count ? vin[idx] : 0u;
    }
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = base_idx + r * 64 + lane;
        const bool valid = idx < count;
        const uint32_t d = (keys[r] >> shift) & mask;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < bits; ++b) {
            const bool bit = (d >> b) & 1u;
            const uint64_t bb = __ballot(bit);
            peers &= bit ? bb : ~bb;
        }
        uint32_t old = 0;
        if (valid) old = s_wcnt[wave][d];
        if (valid && (peers & lt) == 0) s_wcnt[wave][d] = old + (uint32_t)__popcll(peers);
        rank[r] = old + (uint32_t)__popcll(peers & lt);
        __builtin_amdgcn_wave_barrier();
    }
    __syncthreads();
    // per digit: wave prefixes and tile total; then the block scans of the
    // digit totals (global) and of this tile's totals
    uint32_t g = 0, t = 0;
    if (tid < NB) {
        const uint32_t t0 = s_wcnt[0][tid], t1 = s_wcnt[1][tid], t2 = s_wcnt[2][tid], t3 = s_wcnt[3][tid];
        t = t0 + t1 + t2 + t3;
        s_wcnt[0][tid] = 0;
        s_wcnt[1][tid] = t0;
        s_wcnt[2][tid] = t0 + t1;
        s_wcnt[3][tid] = t0 + t1 + t2;
        g = dtot[tid];
    }
    const uint32_t gi = wave_inclusive_sum(g), ti = wave_inclusive_sum(t);
    if (lane == 63) {
        s_wg[wave] = gi;
        s_wt[wave] = ti;
    }
    __syncthreads();
    uint32_t go = 0, to = 0;
    for (int w = 0; w < wave; ++w) {
        go += s_wg[w];
        to += s_wt[w];
    }
    if (tid < NB) {
        s_base[tid] = go + gi - g + cnt[(size_t)tid * cnt_stride + tile];   // output start of (digit, tile)
        s_tot[tid] = to + ti - t;                                           // start inside the tile
    }
    if (tid == NB - 1 && tile == 0 && go + gi != count) atomicOr(err, 8u);
    __syncthreads();
#pragma unroll
    for (int r = 0; r < ITEMS; ++r) {
        const uint32_t idx = base_idx + r * 64 + lane;
        if (idx < count) {
            const uint32_t d = (keys[r] >> shift) & mask;
            const uint32_t lpos = s_tot[d] + s_wcnt[wave][d] + rank[r];
            s_k[lpos] = keys[r];
            if constexpr (!PACKED) s_v[lpos] = vals[r];
        }
    }
    __syncthreads();
    const uint32_t in_tile = min(TILE, count - tile * TILE);
    for (uint32_t li = tid; li < in_tile; li += kSortThreads) {
        const uint32_t k = s_k[li];
        const uint32_t d = (k >> shift) & mask;
        const uint32_t pos = s_base[d] + (li - s_tot[d]);
        if (pos < count) {
            kout[pos] = k;
            if constexpr (!PACKED) vout[pos] = s_v[li];
        } else {
            atomicOr(err, 4u);   // inconsistent counts: never write out of bounds
        }
    }
}

// ---------------------------------------------------------------- k_tile_order
//
// Tile ranges and blend order, one block.  The instances of a tile are the
// Gaussians whose rectangle covers it, so its count is the 2D prefix sum of
// the difference grid the preprocess filled (+1 / -1 at the rectangle's four
// corners); the sorted list holds the tiles in id order, so a tile's range
// starts at the exclusive scan of the counts in tile order.  An empty tile
// gets [0, 0); an overflowed frame (its sort skipped) gets empty ranges
// everywhere, and a count sum that differs from K is flagged.  The blend
// order is by list length, longest first, in power-of-two classes (order
// inside a class is arbitrary; each tile's result does not depend on it):
// blocks are dispatched in index order and spread round-robin over the XCDs,
// so the longest tiles start first and land on different XCDs.
// order[k] = (tile, start, end, 0): the blend reads its tile's range with its id.

__global__ __launch_bounds__(1024) void k_tile_order(DevStatus *__restrict__ st, int32_t *__restrict__ tgrid,
                                                     int tiles_x, int tiles_y, uint2 *__restrict__ ranges,
                                                     uint4 *__restrict__ order, int grid_lds) {
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    constexpr int NW = 1024 / 64;
    const int gw = tiles_x + 1;
    const int n_tiles = tiles_x * tiles_y;
    // the grid in LDS when it fits (else worked on in place in the workspace)
    extern __shared__ int32_t s_g[];
    int32_t *gr = tgrid;
    if (grid_lds) {
        for (int i = tid; i < grid_lds; i += 1024) s_g[i] = tgrid[i];
        gr = s_g;
    }
    __syncthreads();
    // inclusive prefix sums along the rows, then down the columns: one wave
    // per row (column), 64 cells per step with a shuffle scan
    for (int y = wave; y < tiles_y; y += NW) {
        int32_t carry = 0;
        for (int x0 = 0; x0 < tiles_x; x0 += 64) {
            const int x = x0 + lane;
            const int32_t v = (int32_t)wave_inclusive_sum(x < tiles_x ? (uint32_t)gr[y * gw + x] : 0u);
            if (x < tiles_x) gr[y * gw + x] = carry + v;
            carry += __builtin_amdgcn_readlane(v, 63);
        }
    }
    __syncthreads();
    for (int x = wave; x < tiles_x; x += NW) {
        int32_t carry = 0;
        for (int y0 = 0; y0 < tiles_y; y0 += 64) {
            const int y = y0 + lane;
            const int32_t v = (int32_t)wave_inclusive_sum(y < tiles_y ? (uint32_t)gr[y * gw + x] : 0u);
            if (y < tiles_y) gr[y * gw + x] = carry + v;
            carry += __builtin_amdgcn_readlane(v, 63);
        }
    }
    __syncthreads();
    // exclusive scan of the counts in tile order: a contiguous run of at most
    // kOrderRun tiles per thread (kept in registers), then a block scan of the
    // run sums
    const bool ovf = st->overflow != 0;
    const int q = (n_tiles + 1023) / 1024;
    const int a0 = min(n_tiles, tid * q), a1 = min(n_tiles, a0 + q);
    uint32_t part = 0;
    {
        int y = a0 / tiles_x, x = a0 - y * tiles_x;
        for (int t = a0; t < a1; ++t) {
            part += (uint32_t)gr[y * gw + x];
            if (++x == tiles_x) { x = 0; ++y; }
        }
    }
    const uint32_t xs = wave_inclusive_sum(part);
    __shared__ uint32_t s_w[NW];
    __shared__ uint32_t hist[33];
    if (lane == 63) s_w[wave] = xs;
    if (tid < 33) hist[tid] = 0;
    __syncthreads();
    uint32_t base = xs - part;
    for (int w = 0; w < wave; ++w) base += s_w[w];
    auto cls = [](uint32_t len) -> int { return 32 - __clz(len); };
    {
        int y = a0 / tiles_x, x = a0 - y * tiles_x;
        for (int t = a0; t < a1; ++t) {
            const uint32_t c = (uint32_t)gr[y * gw + x];
            const uint32_t len = ovf ? 0u : c;
            ranges[t] = len ? make_uint2(base, base + c) : make_uint2(0u, 0u);
            atomicAdd(&hist[cls(len)], 1u);
            base += c;
            if (++x == tiles_x) { x = 0; ++y; }
        }
    }
    if (tid == 1023 && (unsigned long long)base != st->k_total) atomicOr(&st->sort_error, 16u);
    __syncthreads();
    if (wave == 0) {
        // positions of the length classes, longest first: an exclusive scan
        // over classes 32 .. 0 (lane l holds class 32 - l)
        const int c = 32 - lane;
        const uint32_t h = c >= 0 ? hist[c] : 0u;
        const uint32_t e = wave_inclusive_sum(h);
        if (c >= 0) hist[c] = e - h;
    }
    __syncthreads();
    {
        base = xs - part;
        for (int w = 0; w < wave; ++w) base += s_w[w];
        int y = a0 / tiles_x, x = a0 - y * tiles_x;
        for (int t = a0; t < a1; ++t) {
            const uint32_t c = (uint32_t)gr[y * gw + x];
            const uint32_t len = ovf ? 0u : c;
            const uint2 r = len ? make_uint2(base, base + c) : make_uint2(0u, 0u);
            order[atomicAdd(&hist[cls(len)], 1u)] = make_uint4((uint32_t)t, r.x, r.y, 0u);
            base += c;
            if (++x == tiles_x) { x = 0; ++y; }
        }
    }
}

// ---------------------------------------------------------------- k_blend
//
// One 256-thread block per 16x16 tile; wave w owns the 8x8 quadrant
// (w & 1, w >> 1), lane l the pixel (l & 7, l >> 3) inside it.  The four
// waves run independently (no block barrier until the end).  Per step a wave
// takes the next 64 list entries, one per lane, and keeps those that can be
// composited at some pixel of its quadrant, by two conservative tests on the
// bounds the preprocess stored with each record (see cull_bounds): the
// axis-aligned extent of the entry's alpha >= 1/255 ellipse must meet the
// quadrant, and the binary32 quadratic form at the quadrant centre must not
// exceed the entry's reach.  An entry that fails either is skipped by every
// pixel of the quadrant anyway (alpha 0: no colour, no change of T, no stop),
// so leaving it out changes no output bit.  The kept entries are packed in
// list order into the wave's LDS slots (list positions stored) and
// composited with a branch-free body; the wave leaves once all its pixels are
// done.
//
// TRACK: also write n_contrib / final_T and count, per tile, the list
// entries the pixels visit up to their stop (the evaluation count of the
// method) and the kept entries they composite; without it the loop carries
// none of that bookkeeping.

constexpr int kBlendUnroll = 4;   // entries composited per step of the loop (power of two, <= 64)

template <bool TRACK>
__global__ __launch_bounds__(kTilePixels) void k_blend(const uint4 *__restrict__ order,
                                                       const uint32_t *__restrict__ gids, uint32_t gmask,
                                                       const float4 *__restrict__ recA,
                                                       const float4 *__restrict__ recB,
                                                       const float4 *__restrict__ recC, int width, int height,
                                                       int tiles_x, int n_tiles, const CamK *__restrict__ camd,
                                                       DevStatus *__restrict__ st,
                                                       unsigned long long *__restrict__ tile_evals,
                                                       unsigned long long *__restrict__ tile_comp, int passes,
                                                       int n) {
    constexpr int NW = kTilePixels / 64;   // waves = quadrants
    // per wave: a queue of packed records.  Each step appends its kept
    // entries, composites whole groups of kBlendUnroll and carries the rest
    // (fewer than kBlendUnroll) to the front for the next step; the last step
    // pads with blank records (log2 o = -inf, so alpha = 0).  A slot is three
    // float4 = (u, v, -A/2, -C/2), (-B, log2 o, r, g), (b, list position + 1
    // as bits, -, -).
    constexpr int kQueue = 64 + kBlendUnroll;
    __shared__ float4 sR[NW][kQueue * 3];
    const int b = (int)blockIdx.x;
    if (b >= n_tiles) return;
    const uint4 ord = order[b];   // block b blends tile order[b]: the longest lists start first
    const int tile = (int)ord.x;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    if (b == 0 && tid == 0) {
        st->tiles = (uint32_t)n_tiles;
        st->passes = (uint32_t)passes;
        st->pack_bits = gmask == 0xffffffffu ? 0u : (uint32_t)__popc(gmask);
        st->tracked = TRACK ? 1u : 0u;
    }
    const int qx0 = tx * kTile + (wave & 1) * 8, qy0 = ty * kTile + (wave >> 1) * 8;
    const int px = qx0 + (lane & 7), py = qy0 + (lane >> 3);
    const bool inside = px < width && py < height;
    const size_t pix = inside ? (size_t)py * width + px : 0;
    const int start = (int)ord.y, end = (int)ord.z;
    const float fpx = (float)px, fpy = (float)py;
    // this quadrant's rectangle of pixel centres, clipped to the image (empty
    // if the quadrant lies outside), and the centre of the full quadrant
    const float x_lo = (float)qx0, y_lo = (float)qy0;
    const float x_hi = fminf(x_lo + 7.0f, (float)(width - 1));
    const float y_hi = fminf(y_lo + 7.0f, (float)(height - 1));
    const bool quad_live = x_hi >= x_lo && y_hi >= y_lo;
    const float qcx = x_lo + 3.5f, qcy = y_lo + 3.5f;
    float T = 1.0f, cr = 0.0f, cg = 0.0f, cbl = 0.0f;
    bool live = inside;   // false once the pixel stopped (or outside)
    int last = 0, evals = inside ? end - start : 0;   // TRACK only
    unsigned comp = 0;                                // TRACK only
    const float a_min = 1.0f / 255.0f;
    const uint64_t lt = lanemask_lt64();
    float4 *__restrict__ R = sR[wave];
    const float4 zero4 = make_float4(0.f, 0.f, 0.f, 0.f);
    const float4 blank1 = make_float4(0.f, -INFINITY, 0.f, 0.f);
    // Software pipeline over the steps: while step k is culled and
    // composited, the records of step k + 1 and the ids of step k + 2 are in
    // flight (ids are checked where they are used, so no wait follows their
    // load; g >= n only if the sort failed, which is flagged there).
    auto load_gid = [&](int i) -> uint32_t { return i < end ? gids[i] : 0u; };
    auto safe = [&](uint32_t w) -> uint32_t {
        const uint32_t g = w & gmask;
        return g < (uint32_t)n ? g : 0u;
    };
    float4 nA = zero4, nB = zero4, nC = zero4;
    if (start + lane < end) {
        const uint32_t g = safe(load_gid(start + lane));
        nA = recA[g];
        nB = recB[g];
        nC = recC[g];
    }
    uint32_t g_next = load_gid(start + 64 + lane);
    int queued = 0;   // records carried over from the previous step (< kBlendUnroll)
    for (int b0 = start; b0 < end; b0 += 64) {
        if (__builtin_amdgcn_ballot_w64(live) == 0) break;
        const int i = b0 + lane;
        const float4 A4 = nA, B4 = nB, C4 = nC;
        if (i + 64 < end) {
            const uint32_t g = safe(g_next);
            nA = recA[g];
            nB = recB[g];
            nC = recC[g];
        }
        g_next = load_gid(i + 128);
        bool keep = false;
        if (i < end && quad_live) {
            // extent of the alpha >= 1/255 ellipse against the quadrant (0.01
            // pixel covers the rounding of u +- hx), then the reach test on
            // the quadratic form at the quadrant centre
            const bool box = A4.x + C4.y >= x_lo - 0.01f && A4.x - C4.y <= x_hi + 0.01f &&
                             A4.y + C4.z >= y_lo - 0.01f && A4.y - C4.z <= y_hi + 0.01f;
            const float cx = A4.x - qcx, cy = A4.y - qcy;
            const float pc = __builtin_fmaf(cx, __builtin_fmaf(A4.z, cx, B4.x * cy), (A4.w * cy) * cy);
            keep = box && -2.0f * pc <= C4.w;
        }
        const uint64_t km = __builtin_amdgcn_ballot_w64(keep);
        const int total = queued + (int)__popcll(km);
        const bool last_step = b0 + 64 >= end;
        // whole groups now; at the end of the list, everything (padded)
        const int kept4 = last_step ? (total + kBlendUnroll - 1) & ~(kBlendUnroll - 1)
                                    : total & ~(kBlendUnroll - 1);
        // append the kept entries in list order behind the carried ones
        if (keep) {
            const int slot = queued + (int)__popcll(km & lt);
            R[3 * slot] = A4;
            R[3 * slot + 1] = make_float4(B4.x, __log2f(B4.y), B4.z, B4.w);
            R[3 * slot + 2] = make_float4(C4.x, __int_as_float(i - start + 1), 0.0f, 0.0f);
        }
        if (lane < kept4 - total) {
            R[3 * (total + lane)] = zero4;
            R[3 * (total + lane) + 1] = blank1;
            R[3 * (total + lane) + 2] = zero4;
        }
        queued = total - kept4;   // 0 at the last step
        if (kept4 == 0) continue;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        // ---- composite the packed entries (branch-free body)
        for (int j = 0; j < kept4; j += kBlendUnroll) {
#pragma unroll
            for (int u = 0; u < kBlendUnroll; ++u) {
                const float4 R0 = R[3 * (j + u)];
                const float4 R1 = R[3 * (j + u) + 1];
                const float2 R2 = *reinterpret_cast<const float2 *>(&R[3 * (j + u) + 2]);
                const float dx = R0.x - fpx, dy = R0.y - fpy;
                // -(A dx^2 + C dy^2)/2 - B dx dy = dx (-A/2 dx - B dy) + (-C/2 dy) dy
                const float power = __builtin_fmaf(dx, __builtin_fmaf(R0.z, dx, R1.x * dy), (R0.w * dy) * dy);
                // skipped entries (power > 0, alpha < 1/255) get alpha 0, and so
                // does every entry after the pixel stopped: then T (1 - alpha)
                // = T >= 1e-4, nothing stops, adds or moves
                const float e = __builtin_amdgcn_exp2f(__builtin_fmaf(power, 1.44269504f, R1.y));
                // min(0.99, e) as a median (e >= 0): one instruction
                const float alpha = (power > 0.0f || e < a_min || !live) ? 0.0f : __builtin_amdgcn_fmed3f(e, 0.0f, 0.99f);
                const float test = __builtin_fmaf(-alpha, T, T);   // T (1 - alpha), one rounding
                const bool stop = test < 0.0001f;
                // the weight alpha T is the drop in transmittance
                const float Tn = stop ? T : test;
                const float w = T - Tn;
                cr = __builtin_fmaf(R1.z, w, cr);
                cg = __builtin_fmaf(R1.w, w, cg);
                cbl = __builtin_fmaf(R2.x, w, cbl);
                if constexpr (TRACK) {
                    const int pos1 = __float_as_int(R2.y);
                    comp += (live && pos1 != 0) ? 1u : 0u;
                    evals = (stop && live) ? pos1 : evals;
                    last = w > 0.0f ? pos1 : last;
                }
                live = live && !stop;
                T = Tn;
            }
            if (__builtin_amdgcn_ballot_w64(live) == 0) break;
        }
        // carry the remainder to the front (kept4 >= kBlendUnroll > queued, so
        // the source and destination slots never overlap)
        if (lane < queued) {
            const float4 c0 = R[3 * (kept4 + lane)], c1 = R[3 * (kept4 + lane) + 1];
            const float4 c2 = R[3 * (kept4 + lane) + 2];
            R[3 * lane] = c0;
            R[3 * lane + 1] = c1;
            R[3 * lane + 2] = c2;
        }
        // the next step rewrites the slots: finish this step's reads first
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
    }
    if constexpr (TRACK) {
        __shared__ unsigned long long s_ev[NW], s_cp[NW];
        unsigned long long e = (unsigned long long)evals, c = comp;
#pragma unroll
        for (int o = 32; o >= 1; o >>= 1) {
            e += __shfl_xor(e, o, 64);
            c += __shfl_xor(c, o, 64);
        }
        if (lane == 0) {
            s_ev[wave] = e;
            s_cp[wave] = c;
        }
        __syncthreads();
        if (tid == 0) {
            unsigned long long se = 0, sc = 0;
            for (int w = 0; w < NW; ++w) {
                se += s_ev[w];
                sc += s_cp[w];
            }
            tile_evals[tile] = se;   // summed on the host by read_status (no contended atomic)
            tile_comp[tile] = sc;
        }
    }
    if (inside) {
        float *__restrict__ image = camd->image;
        const float bg0 = camd->bg[0], bg1 = camd->bg[1], bg2 = camd->bg[2];
        const size_t plane = (size_t)width * height;
        image[pix] = cr + T * bg0;
        image[plane + pix] = cg + T * bg1;
        image[2 * plane + pix] = cbl + T * bg2;
        if constexpr (TRACK) {
            if (float *__restrict__ final_T = camd->final_T) final_T[pix] = T;
            if (int32_t *__restrict__ n_contrib = camd->n_contrib) n_contrib[pix] = last;
        }
    }
}

// ---------------------------------------------------------------- k_export

__global__ void k_export_keys(const DevStatus *__restrict__ st, const uint32_t *__restrict__ tkeys,
                              const uint32_t *__restrict__ tvals, const uint32_t *__restrict__ dkeys_by_gid,
                              unsigned long long *__restrict__ out, uint32_t k) {
    const uint32_t K = min(st->k_used, k);
    const uint32_t pb = st->pack_bits;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < K; i += gridDim.x * blockDim.x) {
        const uint32_t t = pb ? tkeys[i] >> pb : tkeys[i];
        const uint32_t g = pb ? tkeys[i] & ((1u << pb) - 1u) : tvals[i];
        out[i] = ((unsigned long long)t << 32) | dkeys_by_gid[g];
    }
}
__global__ void k_export_gids(const DevStatus *__restrict__ st, const uint32_t *__restrict__ tkeys,
                              const uint32_t *__restrict__ tvals, uint32_t *__restrict__ out, uint32_t k) {
    const uint32_t K = min(st->k_used, k);
    const uint32_t pb = st->pack_bits;
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < K; i += gridDim.x * blockDim.x)
        out[i] = pb ? tkeys[i] & ((1u << pb) - 1u) : tvals[i];
}

__global__ void k_export_splat2d(int n, const float4 *__restrict__ recA, const float4 *__restrict__ recB,
                                 const float4 *__restrict__ recC, float *__restrict__ out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const float4 A = recA[g], B = recB[g];
    float *o = out + (size_t)g * 12;
    o[0] = A.x; o[1] = A.y; o[2] = A.z; o[3] = A.w;
    o[4] = B.x; o[5] = B.y; o[6] = B.z; o[7] = B.w;
    o[8] = recC[g].x; o[9] = 0.f; o[10] = 0.f; o[11] = 0.f;
}

__global__ void k_export_rect(int n, const uint2 *__restrict__ rect, int32_t *__restrict__ out) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    const uint2 r = rect[g];
    out[4 * g + 0] = r.x & 0xffff;
    out[4 * g + 1] = r.x >> 16;
    out[4 * g + 2] = r.y & 0xffff;
    out[4 * g + 3] = r.y >> 16;
}

__global__ void k_copy_u32(const uint32_t *__restrict__ src, uint32_t *__restrict__ dst, const DevStatus *st,
                           uint32_t k, int use_k) {
    uint32_t K = k;
    if (use_k) K = min(st->k_used, k);
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < K; i += gridDim.x * blockDim.x) dst[i] = src[i];
}

inline CamK make_cam(const g4d_camera *C) {
    CamK k{};
    for (int i = 0; i < 12; ++i) k.v[i] = C->viewmat[i];
    k.fx = C->fx; k.fy = C->fy; k.cx = C->cx; k.cy = C->cy;
    k.tanx = C->tan_half_fov_x; k.tany = C->tan_half_fov_y; k.near_plane = C->near_plane;
    for (int i = 0; i < 3; ++i) k.campos[i] = C->campos[i];
    for (int i = 0; i < 3; ++i) k.bg[i] = C->bg[i];
    k.width = C->width; k.height = C->height;
    k.tiles_x = (C->width + kTile - 1) / kTile;
    k.tiles_y = (C->height + kTile - 1) / kTile;
    return k;
}

template <typename T>
T *at(const g4d_workspace *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws->ptr) + off);
}

bool ws_layout(const g4d_workspace *ws, WsLayout *L) {
    if (!ws || !ws->ptr || (reinterpret_cast<uintptr_t>(ws->ptr) & 255)) return false;
    if (!make_layout(ws->n_max, ws->width_max, ws->height_max, ws->instance_capacity, L)) return false;
    return ws->bytes >= L->total;
}

}  // namespace

// Buffer roles (fixed, so that the export path needs no frame state):
//   dgid        per-Gaussian depth key, indexed by Gaussian
//   dk/dv       depth sort ping-pong: dgid -> 1 -> 0 -> 1 -> 0; order = dv0
//   tk/tv       tile sort: emitted into buffer 1 for one pass, 0 for two, so
//               the sorted instances always end in tk0/tv0
g4d_status render(const g4d_splats *G, const g4d_camera *C, const g4d_workspace *ws, float *image,
                  float *final_T, int32_t *n_contrib, hipStream_t s) {
    if (!G || !C || !ws || !image) return G4D_EINVAL;
    WsLayout L;
    if (!ws_layout(ws, &L)) return G4D_EINVAL;
    const int n = G->n;
    if (n < 0 || n > L.n_max || G->sh_degree < 0 || G->sh_degree > 3) return G4D_EINVAL;
    if (C->width < 1 || C->height < 1 || C->width > L.w_max || C->height > L.h_max) return G4D_EINVAL;
    if (n > 0 && (!G->means || !G->scales || !G->quats || !G->opacity || !G->sh)) return G4D_EINVAL;
    if (!(C->fx > 0.0f) || !(C->fy > 0.0f) || !(C->near_plane > 0.0f)) return G4D_EINVAL;
    CamK cam = make_cam(C);
    cam.image = image;
    cam.final_T = final_T;
    cam.n_contrib = n_contrib;
    const int tiles = cam.tiles_x * cam.tiles_y;
    const uint32_t cap = (uint32_t)L.cap;
    const TilePassPlan plan = tile_pass_plan(tiles);
    // An instance is packed into one word (tile << gbits) | index when the
    // tile ids and the Gaussian indices fit in 32 bits together; otherwise
    // tile ids and indices travel in two arrays.
    int gbits = 1, tbits = 0;
    while (gbits < 32 && (1u << gbits) < (uint32_t)n) ++gbits;
    while ((1 << tbits) < tiles) ++tbits;
    const bool packed = n > 0 && gbits + tbits <= 32;
    const int kshift = packed ? gbits : 0;

    DevStatus *st = at<DevStatus>(ws, L.status);
    CamK *camd = at<CamK>(ws, L.cam);
    uint32_t *depth_hist = at<uint32_t>(ws, L.depth_hist);
    uint32_t *lb_depth = at<uint32_t>(ws, L.lb_depth);
    unsigned long long *lb_scan = at<unsigned long long>(ws, L.lb_scan);
    uint2 *ranges = at<uint2>(ws, L.ranges);
    int32_t *tgrid = at<int32_t>(ws, L.tgrid);
    float4 *recA = at<float4>(ws, L.recA);
    float4 *recB = at<float4>(ws, L.recB);
    float4 *recC = at<float4>(ws, L.recC);
    uint2 *rect = at<uint2>(ws, L.rect);
    uint32_t *touched = at<uint32_t>(ws, L.touched);
    uint32_t *dgid = at<uint32_t>(ws, L.dgid);
    uint32_t *dk[2] = {at<uint32_t>(ws, L.dk0), at<uint32_t>(ws, L.dk1)};
    uint32_t *dv[2] = {at<uint32_t>(ws, L.dv0), at<uint32_t>(ws, L.dv1)};
    unsigned long long *offsets = at<unsigned long long>(ws, L.offsets);
    uint32_t *tk[2] = {at<uint32_t>(ws, L.tk0), at<uint32_t>(ws, L.tk1)};
    uint32_t *tv[2] = {at<uint32_t>(ws, L.tv0), at<uint32_t>(ws, L.tv1)};

    auto mark = [&](int i) {
        if (hipEvent_t e = stage_event(i)) (void)hipEventRecord(e, s);
    };
    mark(0);
    // 0. clear status, histograms, look-back state and ranges
    {
        const size_t n16 = L.zero_bytes / 16;
        const int blocks = (int)std::min<size_t>((n16 + 255) / 256, 2048);
        hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, reinterpret_cast<uint4 *>(ws->ptr), n16, cam, camd);
    }
    mark(1);
    uint4 *order = at<uint4>(ws, L.order);
    if (n > 0) {
        const int nb_n = (n + 1023) / 1024;
        // 1. preprocess
        // the tile-count difference grid in LDS per block when it fits, else
        // added straight into the workspace's grid
        const int gcells = (cam.tiles_x + 1) * (cam.tiles_y + 1);
        const int glds = gcells <= kGridLdsCells ? gcells : 0;
        if (g4d_status e = ensure_max_lds(reinterpret_cast<const void *>(k_preprocess), g_preprocess_lds,
                                          kGridLdsCells * 4))
            return e;
        hipLaunchKernelGGL(k_preprocess, dim3(nb_n), dim3(1024), glds * 4, s, n, G->sh_degree, G->means, G->scales,
                           G->quats, G->opacity, G->sh, camd, recA, recB, recC, rect, touched, dgid, depth_hist, st,
                           tgrid, glds);
        mark(2);
        // 2. depth sort: four 8-bit passes over n keys (constant-digit passes
        //    skipped on the device); values start as the identity
        const int sblocks = (n + kSortTileN - 1) / kSortTileN;
        for (int p = 0; p < 4; ++p) {
            hipLaunchKernelGGL(k_sort_pass<kSortItemsN>, dim3(sblocks), dim3(kSortThreads), 0, s, n, p, dgid, dk[0],
                               dk[1], dv[0], dv[1], depth_hist, lb_depth + (size_t)p * L.nblk_n * 256,
                               &st->tile_counter[p], &st->sort_error);
        }
        mark(3);
        const uint32_t *order = dv[0];
        // 3. instance offsets in depth order and K
        const int scan_blocks = (n + kScanTile - 1) / kScanTile;
        hipLaunchKernelGGL(k_scan_offsets, dim3(scan_blocks), dim3(256), 0, s, n, order, touched, offsets, lb_scan,
                           &st->tile_counter[4], st, cap);
        mark(4);
        // 4. emit instances (first tile-sort buffer chosen so the result lands in tk0/tv0)
        const int e = plan.passes == 1 ? 1 : 0;
        uint32_t *tcnt = at<uint32_t>(ws, L.tcnt);
        uint32_t *tdtot = at<uint32_t>(ws, L.tdtot);
        const int cstride = L.nblk_k;
        const int kblocks = L.nblk_k;
        hipLaunchKernelGGL(k_emit, dim3(kblocks), dim3(256), 0, s, n, order, offsets, rect, cam.tiles_x, st, tk[e],
                           tv[e], packed ? gbits : 0, plan.bits[0], tcnt, cstride);
        mark(5);
        // 5. instance sort by tile digits (reduce-then-scan passes)
        int cur = e;
        for (int p = 0; p < plan.passes; ++p) {
            uint32_t *pc = tcnt + (size_t)p * 256 * cstride;
            uint32_t *pt = tdtot + 256 * p;
            const int NB = 1 << plan.bits[p];
            if (p > 0)
                hipLaunchKernelGGL(k_sort_up, dim3(kblocks), dim3(kSortThreads), 0, s, tk[cur], st, cap,
                                   kshift + plan.shift[p], plan.bits[p], pc, cstride);
            hipLaunchKernelGGL(k_spine, dim3(NB), dim3(256), 0, s, pc, cstride, NB, st, cap, pt);
            if (packed)
                hipLaunchKernelGGL((k_sort_down<kSortItems, true>), dim3(kblocks), dim3(kSortThreads), 0, s, tk[cur],
                                   tv[cur], tk[cur ^ 1], tv[cur ^ 1], st, cap, kshift + plan.shift[p], plan.bits[p],
                                   pc, cstride, pt, &st->sort_error);
            else
                hipLaunchKernelGGL((k_sort_down<kSortItems, false>), dim3(kblocks), dim3(kSortThreads), 0, s, tk[cur],
                                   tv[cur], tk[cur ^ 1], tv[cur ^ 1], st, cap, plan.shift[p], plan.bits[p], pc,
                                   cstride, pt, &st->sort_error);
            cur ^= 1;
        }
        mark(6);
    } else {
        for (int i = 2; i <= 6; ++i) mark(i);
    }
    // 6. ranges from the tile counts, and the blend order of the tiles
    {
        const int gcells = (cam.tiles_x + 1) * (cam.tiles_y + 1);
        const int glds = gcells <= kGridLdsCells ? gcells : 0;
        if (g4d_status e = ensure_max_lds(reinterpret_cast<const void *>(k_tile_order), g_order_lds,
                                          kGridLdsCells * 4))
            return e;
        hipLaunchKernelGGL(k_tile_order, dim3(1), dim3(1024), glds * 4, s, st, tgrid, cam.tiles_x, cam.tiles_y,
                           ranges, order, glds);
    }
    mark(7);
    // 7. blend (with n == 0 every range is empty and the image is the background)
    // the bookkeeping variant when the caller wants n_contrib or final_T
    auto blend = (final_T || n_contrib) ? k_blend<true> : k_blend<false>;
    hipLaunchKernelGGL(blend, dim3(tiles), dim3(kTilePixels), 0, s, order, packed ? tk[0] : tv[0],
                       packed ? (1u << gbits) - 1u : 0xffffffffu, recA, recB, recC, C->width,
                       C->height, cam.tiles_x, tiles, camd, st, at<unsigned long long>(ws, L.evals),
                       at<unsigned long long>(ws, L.comp), plan.passes, std::max(n, 1));
    mark(8);
    G4D_HIP_CHECK(hipGetLastError());
    return G4D_OK;
}

g4d_status read_status(const g4d_workspace *ws, g4d_device_status *out, hipStream_t s) {
    WsLayout L;
    if (!out || !ws_layout(ws, &L)) return G4D_EINVAL;
    DevStatus h{};
    G4D_HIP_CHECK(hipMemcpyAsync(&h, at<DevStatus>(ws, L.status), sizeof(h), hipMemcpyDeviceToHost, s));
    G4D_HIP_CHECK(hipStreamSynchronize(s));
    out->instances = (int64_t)h.k_total;
    out->overflow = (int32_t)h.overflow;
    out->sort_error = (int32_t)h.sort_error;
    out->visible = (int32_t)h.visible;
    out->tiles = (int32_t)h.tiles;
    // blend work, one count per tile of the last frame (a render that wrote
    // n_contrib or final_T counts it; -1 otherwise)
    out->blend_evals = -1;
    out->blend_composited = -1;
    if (h.tracked && h.tiles > 0 && (int64_t)h.tiles <= (int64_t)L.tiles_max) {
        std::vector<unsigned long long> te(2 * (size_t)h.tiles);
        G4D_HIP_CHECK(hipMemcpyAsync(te.data(), at<unsigned long long>(ws, L.evals), (size_t)h.tiles * 8,
                                     hipMemcpyDeviceToHost, s));
        G4D_HIP_CHECK(hipMemcpyAsync(te.data() + h.tiles, at<unsigned long long>(ws, L.comp), (size_t)h.tiles * 8,
                                     hipMemcpyDeviceToHost, s));
        G4D_HIP_CHECK(hipStreamSynchronize(s));
        int64_t evals = 0, comp = 0;
        for (uint32_t t = 0; t < h.tiles; ++t) {
            evals += (int64_t)te[t];
            comp += (int64_t)te[h.tiles + t];
        }
        out->blend_evals = evals;
        out->blend_composited = comp;
    }
    return G4D_OK;
}

// Spatial processing order of a Gaussian set: Morton codes of the means, then
// the four radix passes of the render's depth sort (stable, so ties keep
// index order) in the workspace's buffers; the order lands in dv0.
g4d_status spatial_order(const g4d_gaussians *G, const float bmin[3], const float bmax[3],
                         const g4d_workspace *ws, uint32_t *order, hipStream_t s) {
    WsLayout L;
    if (!G || !bmin || !bmax || !order || !ws_layout(ws, &L)) return G4D_EINVAL;
    const int n = G->n;
    if (n < 0 || n > L.n_max || (n > 0 && !G->means)) return G4D_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (!(bmax[k] > bmin[k])) return G4D_EINVAL;
    if (n == 0) return G4D_OK;
    DevStatus *st = at<DevStatus>(ws, L.status);
    uint32_t *hist = at<uint32_t>(ws, L.depth_hist);
    uint32_t *codes = at<uint32_t>(ws, L.dgid);
    uint32_t *dk0 = at<uint32_t>(ws, L.dk0), *dk1 = at<uint32_t>(ws, L.dk1);
    uint32_t *dv0 = at<uint32_t>(ws, L.dv0), *dv1 = at<uint32_t>(ws, L.dv1);
    {
        const size_t n16 = L.zero_bytes / 16;
        const int blocks = (int)std::min<size_t>((n16 + 255) / 256, 2048);
        hipLaunchKernelGGL(k_zero, dim3(blocks), dim3(256), 0, s, reinterpret_cast<uint4 *>(ws->ptr), n16, CamK{},
                           at<CamK>(ws, L.cam));
    }
    float sc[3];
    for (int k = 0; k < 3; ++k) sc[k] = (float)(1024.0 / ((double)bmax[k] - (double)bmin[k]));
    hipLaunchKernelGGL(k_morton, dim3((n + 1023) / 1024), dim3(1024), 0, s, n, G->means, bmin[0], bmin[1], bmin[2],
                       sc[0], sc[1], sc[2], codes, hist);
    const int sblocks = (n + kSortTileN - 1) / kSortTileN;
    uint32_t *lb = at<uint32_t>(ws, L.lb_depth);
    for (int p = 0; p < 4; ++p)
        hipLaunchKernelGGL(k_sort_pass<kSortItemsN>, dim3(sblocks), dim3(kSortThreads), 0, s, n, p, codes, dk0, dk1,
                           dv0, dv1, hist, lb + (size_t)p * L.nblk_n * 256, &st->tile_counter[p], &st->sort_error);
    hipLaunchKernelGGL(k_copy_u32, dim3((n + 255) / 256), dim3(256), 0, s, dv0, order, st, (uint32_t)n, 0);
    G4D_HIP_CHECK(hipGetLastError());
    return G4D_OK;
}

g4d_status render_export(const g4d_workspace *ws, int32_t kind, int32_t n, int64_t k, void *dst, size_t bytes,
                         hipStream_t s) {
    WsLayout L;
    if (!dst || !ws_layout(ws, &L) || n < 0 || n > L.n_max || k < 0) return G4D_EINVAL;
    const DevStatus *st = at<DevStatus>(ws, L.status);
    const int nb = std::max(1, (n + 255) / 256);
    switch (kind) {
        case G4D_EXPORT_SORTED_KEYS: {
            if (k > L.cap || bytes < (size_t)k * 8) return G4D_EINVAL;
            if (k == 0) return G4D_OK;
            hipLaunchKernelGGL(k_export_keys, dim3(256), dim3(256), 0, s, st, at<uint32_t>(ws, L.tk0),
                               at<uint32_t>(ws, L.tv0), at<uint32_t>(ws, L.dgid),
                               static_cast<unsigned long long *>(dst), (uint32_t)k);
            break;
        }
        case G4D_EXPORT_SORTED_GIDS: {
            if (k > L.cap || bytes < (size_t)k * 4) return G4D_EINVAL;
            if (k == 0) return G4D_OK;
            hipLaunchKernelGGL(k_export_gids, dim3(256), dim3(256), 0, s, st, at<uint32_t>(ws, L.tk0),
                               at<uint32_t>(ws, L.tv0), static_cast<uint32_t *>(dst), (uint32_t)k);
            break;
        }
        case G4D_EXPORT_RECT: {
            if (bytes < (size_t)n * 16) return G4D_EINVAL;
            if (n == 0) return G4D_OK;
            hipLaunchKernelGGL(k_export_rect, dim3(nb), dim3(256), 0, s, n, at<uint2>(ws, L.rect),
                               static_cast<int32_t *>(dst));
            break;
        }
        case G4D_EXPORT_DEPTH_BITS:
        case G4D_EXPORT_DEPTH_ORDER: {
            if (bytes < (size_t)n * 4) return G4D_EINVAL;
            if (n == 0) return G4D_OK;
            const uint32_t *src = at<uint32_t>(ws, kind == G4D_EXPORT_DEPTH_BITS ? L.dgid : L.dv0);
            hipLaunchKernelGGL(k_copy_u32, dim3(nb), dim3(256), 0, s, src, static_cast<uint32_t *>(dst), st,
                               (uint32_t)n, 0);
            break;
        }
        case G4D_EXPORT_RANGES: {
            // k = number of tiles of the frame
            if (k > L.tiles_max || bytes < (size_t)k * 8) return G4D_EINVAL;
            if (k == 0) return G4D_OK;
            hipLaunchKernelGGL(k_copy_u32, dim3(256), dim3(256), 0, s, at<uint32_t>(ws, L.ranges),
                               static_cast<uint32_t *>(dst), st, (uint32_t)(2 * k), 0);
            break;
        }
        case G4D_EXPORT_SPLAT2D: {
            if (bytes < (size_t)n * 48) return G4D_EINVAL;
            if (n == 0) return G4D_OK;
            hipLaunchKernelGGL(k_export_splat2d, dim3(nb), dim3(256), 0, s, n, at<float4>(ws, L.recA),
                               at<float4>(ws, L.recB), at<float4>(ws, L.recC), static_cast<float *>(dst));
            break;
        }
        default:
            return G4D_EINVAL;
    }
    G4D_HIP_CHECK(hipGetLastError());
    return G4D_OK;
}

// ---------------------------------------------------------------- graphs
//
// A render captured into a graph keeps every pointer and launch shape of its
// workspace, input set and frame size; the view and the output buffers enter
// only through k_zero's frame argument.  These helpers find that node and
// rewrite its parameters.

g4d_status graph_find_camera_node(hipGraph_t g, hipGraphNode_t *out) {
    size_t count = 0;
    G4D_HIP_CHECK(hipGraphGetNodes(g, nullptr, &count));
    std::vector<hipGraphNode_t> nodes(count);
    G4D_HIP_CHECK(hipGraphGetNodes(g, nodes.data(), &count));
    for (hipGraphNode_t nd : nodes) {
        hipGraphNodeType ty;
        G4D_HIP_CHECK(hipGraphNodeGetType(nd, &ty));
        if (ty != hipGraphNodeTypeKernel) continue;
        hipKernelNodeParams kp{};
        G4D_HIP_CHECK(hipGraphKernelNodeGetParams(nd, &kp));
        if (kp.func == reinterpret_cast<void *>(k_zero)) {
            *out = nd;
            return G4D_OK;
        }
    }
    return G4D_EDEVICE;
}

g4d_status graph_set_frame(hipGraphExec_t exec, hipGraphNode_t node, const g4d_workspace *ws,
                           const g4d_camera *C, float *image, float *final_T, int32_t *n_contrib) {
    WsLayout L;
    if (!C || !image || !ws_layout(ws, &L)) return G4D_EINVAL;
    uint4 *p = reinterpret_cast<uint4 *>(ws->ptr);
    size_t n16 = L.zero_bytes / 16;
    CamK cam = make_cam(C);
    cam.image = image;
    cam.final_T = final_T;
    cam.n_contrib = n_contrib;
    CamK *camd = at<CamK>(ws, L.cam);
    void *args[4] = {&p, &n16, &cam, &camd};
    hipKernelNodeParams kp{};
    kp.func = reinterpret_cast<void *>(k_zero);
    kp.gridDim = dim3((unsigned)std::min<size_t>((n16 + 255) / 256, 2048));
    kp.blockDim = dim3(256);
    kp.sharedMemBytes = 0;
    kp.kernelParams = args;
    kp.extra = nullptr;
    G4D_HIP_CHECK(hipGraphExecKernelNodeSetParams(exec, node, &kp));
    return G4D_OK;
}

size_t status_offset(const g4d_workspace *ws) {
    WsLayout L;
    if (!ws_layout(ws, &L)) return (size_t)-1;
    return L.status;
}

}  // namespace g4d
