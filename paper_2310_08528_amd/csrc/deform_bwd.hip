// Backward of the Gaussian deformation field on gfx950 (Sec. 4.2, Eq. 7-8).
//
// One 256-thread block per 64 Gaussians (16 up to 4096 Gaussians, so that
// small sets still spread over the compute units), FP32 decoder.  The block first
// recomputes the forward (encoder f_h, hidden h, head outputs) in LDS, then:
//   Eq. 8 + activations   d(X + dX) -> dX and dX_canonical; d exp(log s + ds)
//                         -> d log s = d ds = ds' s'; d normalise(r + dr) ->
//                         (I - r' r'^T) dr' / |r + dr|; d sigmoid(logit
//                         [+ dalpha]) -> s (1 - s) do'; C [+ dC] -> dC = dC'.
//   heads                 dh = W2^T ddelta (ReLU mask), dW2 += ddelta h^T,
//                         db2 += ddelta (block sums, one atomic per weight)
//   feature merger        dW1 += dz f_h^T, db1 += dz, df_h = W1^T dz
//   encoder (Eq. 7)       per scale, the product rule over the six planes
//                         (prefix and suffix products), then the bilinear
//                         query's four corners receive weight x gradient by
//                         atomic scatter into the plane gradients, and the
//                         grid coordinates receive the bilinear slopes
//                         (zero at and beyond the box border, as the border
//                         clamp of the query has no slope there).
// Plane-cell updates are summed per block before they reach memory: for
// every plane the block takes the window of cells its Gaussians touch (the
// range of their corner cells along each grid axis; the time axis has the two
// rows of the frame's t), and the windows that fit in the LDS left free by
// the decoder phases accumulate the updates with LDS atomics; each window is
// then added to the plane gradients with one global atomic per nonzero value.
// A block whose Gaussians are spatially close (a set stored in spatial order)
// has small windows; a plane whose window does not fit scatters straight to
// global memory.
// The decoder products of a 64-Gaussian block (h, the head outputs, dz,
// dW2, dW1 and df_h: 64 x 64 x 64 at the headline sizes) run on 16x16x4 FP32
// MFMA tiles with operands in LDS, except W1, whose fragments each wave loads
// from global memory (L2-resident: every block reads it) into registers ahead
// of the phase that uses them.  Blocks of 16 Gaussians (small sets) use FMA
// loops.  The head weights, their biases and the per-row gradient pointers
// are staged in LDS once per block (the heads are selected by a runtime row
// index, which in the inner loops would be a dependent kernel-argument load
// per step); f_h, h, the deltas and dz live in LDS.
#include "g4d_internal.h"

#include <vector>

namespace g4d {
namespace {

constexpr int kGB = 64;        // Gaussians per block
constexpr int kGBSmall = 16;   // ... when 64 would leave most compute units idle
constexpr int kSmallN = 4096;  // up to this many Gaussians (64 blocks of 64; measured crossover)
constexpr int kThreads = 256;
constexpr int kMaxScalesB = 3;

struct BwdJob {
    const float *means, *log_scales, *quats, *opac, *sh;
    const float *planes[kMaxScalesB * 6];
    const float *w1, *b1;
    const float *hw[5], *hb[5];          // head weights / biases: dx, dr, ds, dC, dalpha (null when absent)
    int hrows[5];                        // rows of each head (3, 4, 3, 3 (d+1)^2 or 0, 1 or 0)
    const float *g_means, *g_scales, *g_quats, *g_opac, *g_sh;   // dL/d render-ready set
    float *d_means, *d_log_scales, *d_quats, *d_opac, *d_sh;     // canonical (written)
    float *d_planes[kMaxScalesB * 6];    // accumulated
    float *d_w1, *d_b1;
    float *d_hw[5], *d_hb[5];
    int res[kMaxScalesB][4];
    float gscale[kMaxScalesB][4];
    float bmin[3], bmax[3];
    int n, n_sh_rows;                    // n_sh_rows: 3 (d+1)^2 of the Gaussians
    float t;
};

constexpr size_t kLdsMax = 160 * 1024;   // LDS per CU (and per block) on gfx950

typedef float float4_t __attribute__((ext_vector_type(4)));

// Row stride (floats) of an LDS matrix read by 16x16x4 MFMA fragments.  A
// fragment read touches 16 consecutive rows at one column per k-group
// (address row*ld + k) or, read transposed, 4 rows of 16 consecutive columns
// (k*ld + col); a stride whose residue mod 64 is 12, 20, ..., 52 makes the
// first conflict-free over the 64 banks and the second at most two-way.
__host__ __device__ constexpr int mfma_ld(int x) {
    int ld = x + 1;
    while ((ld & 7) != 4 || (ld & 63) == 4 || (ld & 63) == 60) ++ld;
    return ld;
}

// LDS layout of a block, shared by the kernel and the launch:
//   s_fh [gb][fh] | s_dm [gb][3] | s_h [gb][hh] | s_dz [gb][hh] | s_dd [gb][ds] | s_w2 [rp][hh] | s_b2 [rp]
// rp: head rows padded to whole 16-row tiles (zero rows).  64-Gaussian
// blocks run the decoder on MFMA with padded strides; 16-Gaussian blocks use
// FMA loops with odd strides.
struct BwdLds {
    int fh, hh, ds, rp;
    int o_dm, o_h, o_dz, o_dd, o_w2, o_b2, total;
};
__host__ __device__ inline BwdLds bwd_lds(int gb, int K, int HID, int rows) {
    BwdLds b{};
    b.rp = (rows + 15) & ~15;
    const bool mf = gb == 64;
    b.fh = mf ? mfma_ld(K) : K + 1;
    b.hh = mf ? mfma_ld(HID) : HID + 1;
    b.ds = mf ? mfma_ld(b.rp) : 65;
    b.o_dm = gb * b.fh;
    b.o_h = b.o_dm + gb * 3;
    b.o_dz = b.o_h + gb * b.hh;
    b.o_dd = b.o_dz + gb * b.hh;
    b.o_w2 = b.o_dd + gb * b.ds;
    b.o_b2 = b.o_w2 + b.rp * b.hh;
    b.total = b.o_b2 + b.rp;
    return b;
}

__device__ constexpr int axis_a(int p) { return p == 2 ? 1 : (p == 5 ? 2 : (p == 4 ? 1 : 0)); }
__device__ constexpr int axis_b(int p) { return p == 0 ? 1 : (p == 1 || p == 2 ? 2 : 3); }

__device__ __forceinline__ void grid_coord(float x, float scale, int n, int &i0, float &w) {
    float g = x * scale;
    g = fminf(fmaxf(g, 0.0f), (float)(n - 1));
    int i = (int)floorf(g);
    i = min(i, n - 2);
    i0 = i;
    w = g - (float)i;
}

// Head row r of the concatenated heads: (head, row within it)
__device__ __forceinline__ bool head_of(const BwdJob &J, int r, int &h, int &k) {
    int base = 0;
#pragma unroll
    for (int q = 0; q < 5; ++q) {
        if (r < base + J.hrows[q]) {
            h = q;
            k = r - base;
            return true;
        }
        base += J.hrows[q];
    }
    return false;
}

template <int F, int L, int HID, int GB>
__global__ __launch_bounds__(kThreads) void k_deform_bwd(BwdJob J, int rows) {
    constexpr int K = F * L;
    constexpr bool kMfma = GB == 64;
    static_assert(!kMfma || (K % 16 == 0 && HID % 16 == 0), "MFMA tiles need 16-multiples");
    constexpr int FH = kMfma ? mfma_ld(K) : K + 1, HH = kMfma ? mfma_ld(HID) : HID + 1;
    const BwdLds lay = bwd_lds(GB, K, HID, rows);
    const int DS = lay.ds, RP = lay.rp;
    extern __shared__ __attribute__((aligned(16))) float smem[];
    float *s_fh = smem;                  // [GB][FH]: f_h, later df_h
    float *s_dm = smem + lay.o_dm;       // [GB][3]: dL/d canonical mean
    float *s_h = smem + lay.o_h;         // [GB][HH]: h (after ReLU)
    float *s_dz = smem + lay.o_dz;       // [GB][HH]: dL/d(pre-activation)
    float *s_dd = smem + lay.o_dd;       // [GB][DS]: head outputs, then their gradients
    float *s_w2 = smem + lay.o_w2;       // [RP][HH]: head weights (zero padding rows)
    float *s_b2 = smem + lay.o_b2;       // [RP]
    // the plane-cell windows of the encoder backward reuse everything from
    // s_h on (dead once df_h is computed)
    float *s_win = s_h;
    const int win_cap = lay.total - lay.o_h;
    __shared__ float *s_dw[64];          // gradient row of head row r (null: padding)
    __shared__ float *s_db[64];
    const int tid = threadIdx.x;
    const int g0 = blockIdx.x * GB;
    const int n = J.n;
    if (tid < RP) {
        int hq, k;
        if (tid < rows && head_of(J, tid, hq, k)) {
            s_dw[tid] = J.d_hw[hq] + (size_t)k * HID;
            s_db[tid] = J.d_hb[hq] + k;
            s_b2[tid] = J.hb[hq][k];
        } else {
            s_dw[tid] = nullptr;
            s_db[tid] = nullptr;
            s_b2[tid] = 0.0f;
        }
    }
    for (int idx = tid; idx < RP * HID; idx += kThreads) {
        const int r = idx / HID, j = idx - r * HID;
        int hq, k;
        s_w2[r * HH + j] = r < rows && head_of(J, r, hq, k) ? J.hw[hq][(size_t)k * HID + j] : 0.0f;
    }
    const int wave_u = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    const int lrow = lane & 15, lk = lane >> 4;     // MFMA fragment: row / column 0..15, k group 0..3
    // W1 fragments of h = W1 f_h (wave w: output columns of tiles w, w + 4):
    // lane (lrow, lk) holds W1[c*16 + lrow][4 kk + lk].  Loaded before the
    // encoder so that their latency hides under its gathers.
    constexpr int NC1 = kMfma ? (HID / 16 + 3) / 4 : 0;
    float w1f[NC1 > 0 ? NC1 : 1][kMfma ? K / 4 : 1];
    if constexpr (kMfma) {
#pragma unroll
        for (int ci = 0; ci < NC1; ++ci) {
            const int c = wave_u + 4 * ci;
#pragma unroll
            for (int kk = 0; kk < K / 4; ++kk)
                w1f[ci][kk] = c < HID / 16 ? J.w1[(size_t)(c * 16 + lrow) * K + kk * 4 + lk] : 0.0f;
        }
    }

    // ---- A. encoder (as in the forward)
    constexpr int LPG = F / 4;
    constexpr int GPP = kThreads / LPG;
    constexpr int NPASS = (GB + GPP - 1) / GPP;   // a block of fewer Gaussians than GPP leaves threads idle
#pragma unroll
    for (int pass = 0; pass < NPASS; ++pass) {
        const int gl = pass * GPP + tid / LPG, c4 = tid % LPG, g = g0 + gl;
        const bool in_blk = gl < GB;
        const bool valid = in_blk && g < n;
        float x[4];
#pragma unroll
        for (int k = 0; k < 3; ++k) x[k] = valid ? J.means[(size_t)k * n + g] - J.bmin[k] : 0.0f;
        x[3] = J.t;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            float4 prod = make_float4(1.f, 1.f, 1.f, 1.f);
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const int a = axis_a(p), b = axis_b(p);
                const int na = J.res[l][a], nb = J.res[l][b];
                int ia, ib;
                float wa, wb;
                grid_coord(x[a], J.gscale[l][a], na, ia, wa);
                grid_coord(x[b], J.gscale[l][b], nb, ib, wb);
                const float *base = J.planes[l * 6 + p] + ((size_t)ib * na + ia) * F + 4 * c4;
                const float4 v00 = *reinterpret_cast<const float4 *>(base);
                const float4 v10 = *reinterpret_cast<const float4 *>(base + F);
                const float4 v01 = *reinterpret_cast<const float4 *>(base + (size_t)na * F);
                const float4 v11 = *reinterpret_cast<const float4 *>(base + (size_t)na * F + F);
                const float w00 = (1.0f - wa) * (1.0f - wb), w10 = wa * (1.0f - wb);
                const float w01 = (1.0f - wa) * wb, w11 = wa * wb;
                prod.x *= w00 * v00.x + w10 * v10.x + w01 * v01.x + w11 * v11.x;
                prod.y *= w00 * v00.y + w10 * v10.y + w01 * v01.y + w11 * v11.y;
                prod.z *= w00 * v00.z + w10 * v10.z + w01 * v01.z + w11 * v11.z;
                prod.w *= w00 * v00.w + w10 * v10.w + w01 * v01.w + w11 * v11.w;
            }
            if (!valid) prod = make_float4(0.f, 0.f, 0.f, 0.f);
            if (in_blk) {
                float *dst = s_fh + gl * FH + l * F + 4 * c4;
                dst[0] = prod.x; dst[1] = prod.y; dst[2] = prod.z; dst[3] = prod.w;
            }
        }
    }
    __syncthreads();
    // ---- B. h = ReLU(W1 f_h + b1).  64-Gaussian blocks: 16x16x4 MFMA tiles
    // with the forward kernel's operands and k order (per tile the same chain
    // over k = 4 kk + lk), so the recomputed h rounds as the forward's does.
    // 16-Gaussian blocks: FMA loops, Gaussian fastest (a weight is one
    // broadcast load).
    if constexpr (kMfma) {
#pragma unroll
        for (int ci = 0; ci < NC1; ++ci) {
            const int c = wave_u + 4 * ci;
            if (c < HID / 16) {
                float4_t acc[4];
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) acc[rt] = float4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int kk = 0; kk < K / 4; ++kk) {
#pragma unroll
                    for (int rt = 0; rt < 4; ++rt) {
                        const float a = s_fh[(rt * 16 + lrow) * FH + kk * 4 + lk];
                        acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, w1f[ci][kk], acc[rt], 0, 0, 0);
                    }
                }
                const int col = c * 16 + lrow;
                const float bias = J.b1[col];
#pragma unroll
                for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) s_h[(rt * 16 + 4 * lk + i) * HH + col] = fmaxf(acc[rt][i] + bias, 0.0f);
            }
        }
    } else {
        for (int idx = tid; idx < GB * HID; idx += kThreads) {
            const int g = idx % GB, j = idx / GB;
            float acc = J.b1[j];
            const float *w = J.w1 + (size_t)j * K;
            for (int i = 0; i < K; ++i) acc += w[i] * s_fh[g * FH + i];
            s_h[g * HH + j] = fmaxf(acc, 0.0f);
        }
    }
    // W1 fragments of df_h = W1^T dz (wave w: df_h columns of tiles w, w + 4):
    // lane (lrow, lk) holds W1[4 kk + lk][c*16 + lrow]; in flight until the
    // last decoder phase
    constexpr int NC7 = kMfma ? (K / 16 + 3) / 4 : 0;
    float w1g[NC7 > 0 ? NC7 : 1][kMfma ? HID / 4 : 1];
    if constexpr (kMfma) {
#pragma unroll
        for (int ci = 0; ci < NC7; ++ci) {
            const int c = wave_u + 4 * ci;
#pragma unroll
            for (int kk = 0; kk < HID / 4; ++kk)
                w1g[ci][kk] = c < K / 16 ? J.w1[(size_t)(kk * 4 + lk) * K + c * 16 + lrow] : 0.0f;
        }
    }
    __syncthreads();
    // ---- C. head outputs delta = W2 h + b2 (padding rows: zero weights);
    // MFMA tiles as in the forward (wave w: Gaussians 16w..16w+15)
    if constexpr (kMfma) {
        const int row0 = wave_u * 16;
        for (int c = 0; c < RP / 16; ++c) {
            float4_t acc = float4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 8
            for (int kk = 0; kk < HID / 4; ++kk) {
                const float a = s_h[(row0 + lrow) * HH + kk * 4 + lk];
                const float b = s_w2[(c * 16 + lrow) * HH + kk * 4 + lk];
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) s_dd[(row0 + 4 * lk + i) * DS + c * 16 + lrow] = acc[i] + s_b2[c * 16 + lrow];
        }
    } else {
        for (int idx = tid; idx < GB * rows; idx += kThreads) {
            const int g = idx % GB, r = idx / GB;
            float acc = s_b2[r];
            const float *w = s_w2 + r * HH;
            for (int j = 0; j < HID; ++j) acc += w[j] * s_h[g * HH + j];
            s_dd[g * DS + r] = acc;
        }
    }
    __syncthreads();
    // ---- Eq. 8 + activations, backward (one Gaussian per thread of wave 0);
    // the other waves copy the SH gradient (C' = C [+ dC]: dL/dC = dL/dC')
    if (tid < GB) {
        const int gl = tid, g = g0 + gl;
        float *dd = s_dd + gl * DS;
        if (g < n) {
            // means: X' = X + dX
            for (int k = 0; k < 3; ++k) {
                const float gm = J.g_means[(size_t)k * n + g];
                dd[k] = gm;
                s_dm[gl * 3 + k] = gm;
            }
            // quaternion: r' = (r + dr) / |r + dr|
            float q[4], gq[4], qn = 0.0f;
            for (int k = 0; k < 4; ++k) {
                q[k] = J.quats[(size_t)k * n + g] + dd[3 + k];
                gq[k] = J.g_quats[(size_t)k * n + g];
                qn += q[k] * q[k];
            }
            float dq[4] = {0.f, 0.f, 0.f, 0.f};
            if (qn > 0.0f) {
                const float inv = 1.0f / sqrtf(qn);
                float dot = 0.0f;
                for (int k = 0; k < 4; ++k) dot += q[k] * inv * gq[k];
                for (int k = 0; k < 4; ++k) dq[k] = (gq[k] - q[k] * inv * dot) * inv;
            }
            for (int k = 0; k < 4; ++k) {
                dd[3 + k] = dq[k];
                J.d_quats[(size_t)k * n + g] = dq[k];
            }
            // scales: s' = exp(log s + ds)
            for (int k = 0; k < 3; ++k) {
                const float sc = expf(J.log_scales[(size_t)k * n + g] + dd[7 + k]);
                const float d = J.g_scales[(size_t)k * n + g] * sc;
                dd[7 + k] = d;
                J.d_log_scales[(size_t)k * n + g] = d;
            }
            // colour head: dC rows
            const int nc = J.hrows[3];
            for (int r = 0; r < nc; ++r) dd[10 + r] = J.g_sh[(size_t)r * n + g];
            // opacity: o' = sigmoid(logit [+ dalpha])
            const float logit = J.opac[g] + (J.hrows[4] ? dd[10 + nc] : 0.0f);
            const float sg = 1.0f / (1.0f + expf(-logit));
            const float dl = J.g_opac[g] * sg * (1.0f - sg);
            J.d_opac[g] = dl;
            if (J.hrows[4]) dd[10 + nc] = dl;
            for (int r = 10 + nc + J.hrows[4]; r < RP; ++r) dd[r] = 0.0f;
        } else {
            for (int r = 0; r < RP; ++r) dd[r] = 0.0f;
            for (int k = 0; k < 3; ++k) s_dm[gl * 3 + k] = 0.0f;
        }
    } else if (J.d_sh) {
        for (int idx = tid - GB; idx < GB * J.n_sh_rows; idx += kThreads - GB) {
            const int gl = idx % GB, r = idx / GB, g = g0 + gl;
            if (g < n) J.d_sh[(size_t)r * n + g] = J.g_sh[(size_t)r * n + g];
        }
    }
    __syncthreads();
    // ---- heads backward: dz = (W2^T ddelta) * [h > 0];
    // dW2 += ddelta^T h, db2 += ddelta (sums over the block's Gaussians)
    if constexpr (kMfma) {
        {
            const int row0 = wave_u * 16;
            const int kr = (rows + 3) >> 2;          // k steps over the head rows (zero padded)
            float4_t acc[HID / 16];
#pragma unroll
            for (int c = 0; c < HID / 16; ++c) acc[c] = float4_t{0.0f, 0.0f, 0.0f, 0.0f};
            for (int kk = 0; kk < kr; ++kk) {
                const float a = s_dd[(row0 + lrow) * DS + kk * 4 + lk];
#pragma unroll
                for (int c = 0; c < HID / 16; ++c) {
                    const float b = s_w2[(kk * 4 + lk) * HH + c * 16 + lrow];
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
                }
            }
#pragma unroll
            for (int c = 0; c < HID / 16; ++c)
#pragma unroll
                for (int i = 0; i < 4; ++i) {
                    const int o = (row0 + 4 * lk + i) * HH + c * 16 + lrow;
                    s_dz[o] = s_h[o] > 0.0f ? acc[c][i] : 0.0f;
                }
        }
        const int ntile = (RP / 16) * (HID / 16);
        for (int t = wave_u; t < ntile; t += 4) {
            const int rt = t / (HID / 16), ct = t - rt * (HID / 16);
            float4_t acc = float4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 8
            for (int kk = 0; kk < GB / 4; ++kk) {
                const float a = s_dd[(kk * 4 + lk) * DS + rt * 16 + lrow];
                const float b = s_h[(kk * 4 + lk) * HH + ct * 16 + lrow];
                acc = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc, 0, 0, 0);
            }
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const int r = rt * 16 + 4 * lk + i;
                if (r < rows && acc[i] != 0.0f) atomicAdd(s_dw[r] + ct * 16 + lrow, acc[i]);
            }
        }
        if (tid < rows) {
            float acc = 0.0f;
            for (int g = 0; g < GB; ++g) acc += s_dd[g * DS + tid];
            if (acc != 0.0f) atomicAdd(s_db[tid], acc);
        }
    } else {
        for (int idx = tid; idx < GB * HID; idx += kThreads) {
            const int g = idx % GB, j = idx / GB;
            float acc = 0.0f;
            for (int r = 0; r < rows; ++r) acc += s_w2[r * HH + j] * s_dd[g * DS + r];
            s_dz[g * HH + j] = s_h[g * HH + j] > 0.0f ? acc : 0.0f;
        }
        for (int idx = tid; idx < rows * (HID + 1); idx += kThreads) {
            const int r = idx / (HID + 1), j = idx % (HID + 1);
            if (!s_dw[r]) continue;
            float acc = 0.0f;
            if (j < HID) {
                for (int g = 0; g < GB; ++g) acc += s_dd[g * DS + r] * s_h[g * HH + j];
                if (acc != 0.0f) atomicAdd(s_dw[r] + j, acc);
            } else {
                for (int g = 0; g < GB; ++g) acc += s_dd[g * DS + r];
                if (acc != 0.0f) atomicAdd(s_db[r], acc);
            }
        }
    }
    __syncthreads();
    // ---- feature merger: dW1 += dz^T f_h, db1 += dz
    if constexpr (kMfma) {
        constexpr int NI = K / 16;
        for (int jt = wave_u; jt < HID / 16; jt += 4) {
            float4_t acc[NI];
#pragma unroll
            for (int it = 0; it < NI; ++it) acc[it] = float4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll 4
            for (int kk = 0; kk < GB / 4; ++kk) {
                const float a = s_dz[(kk * 4 + lk) * HH + jt * 16 + lrow];
#pragma unroll
                for (int it = 0; it < NI; ++it) {
                    const float b = s_fh[(kk * 4 + lk) * FH + it * 16 + lrow];
                    acc[it] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[it], 0, 0, 0);
                }
            }
#pragma unroll
            for (int it = 0; it < NI; ++it)
#pragma unroll
                for (int i = 0; i < 4; ++i)
                    if (acc[it][i] != 0.0f)
                        atomicAdd(&J.d_w1[(size_t)(jt * 16 + 4 * lk + i) * K + it * 16 + lrow], acc[it][i]);
        }
        if (tid < HID) {
            float acc = 0.0f;
            for (int g = 0; g < GB; ++g) acc += s_dz[g * HH + tid];
            if (acc != 0.0f) atomicAdd(&J.d_b1[tid], acc);
        }
    } else {
        for (int idx = tid; idx < HID * (K + 1); idx += kThreads) {
            const int j = idx / (K + 1), i = idx % (K + 1);
            float acc = 0.0f;
            if (i < K) {
                for (int g = 0; g < GB; ++g) acc += s_dz[g * HH + j] * s_fh[g * FH + i];
                if (acc != 0.0f) atomicAdd(&J.d_w1[(size_t)j * K + i], acc);
            } else {
                for (int g = 0; g < GB; ++g) acc += s_dz[g * HH + j];
                if (acc != 0.0f) atomicAdd(&J.d_b1[j], acc);
            }
        }
    }
    __syncthreads();
    // df_h = W1^T dz (overwrites f_h)
    if constexpr (kMfma) {
#pragma unroll
        for (int ci = 0; ci < NC7; ++ci) {
            const int c = wave_u + 4 * ci;
            if (c < K / 16) {
                float4_t acc[4];
#pragma unroll
                for (int rt = 0; rt < 4; ++rt) acc[rt] = float4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
                for (int kk = 0; kk < HID / 4; ++kk) {
#pragma unroll
                    for (int rt = 0; rt < 4; ++rt) {
                        const float a = s_dz[(rt * 16 + lrow) * HH + kk * 4 + lk];
                        acc[rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, w1g[ci][kk], acc[rt], 0, 0, 0);
                    }
                }
#pragma unroll
                for (int rt = 0; rt < 4; ++rt)
#pragma unroll
                    for (int i = 0; i < 4; ++i) s_fh[(rt * 16 + 4 * lk + i) * FH + c * 16 + lrow] = acc[rt][i];
            }
        }
    } else {
        for (int idx = tid; idx < GB * K; idx += kThreads) {
            const int g = idx % GB, i = idx / GB;
            float acc = 0.0f;
            for (int j = 0; j < HID; ++j) acc += J.w1[(size_t)j * K + i] * s_dz[g * HH + j];
            s_fh[g * FH + i] = acc;
        }
    }
    __syncthreads();
    // ---- plane-cell windows of this block: the range of the Gaussians'
    // lower corner cells along each spatial grid axis, per scale; a window
    // spans that range plus one (the upper corners).  A cell takes F + 1
    // floats there: with F (a multiple of 32) the eight Gaussians of a wave
    // would add into only 16 of the 64 LDS banks (4-way conflicts).
    constexpr int WF = F + 1;
    __shared__ int s_lo[kMaxScalesB * 3], s_hi[kMaxScalesB * 3];
    __shared__ int s_woff[kMaxScalesB * 6], s_wa0[kMaxScalesB * 6], s_wb0[kMaxScalesB * 6];
    __shared__ int s_wn[kMaxScalesB * 6], s_wm[kMaxScalesB * 6];
    __shared__ int s_wtotal;
    if (wave_u == 0) {
        // lane = Gaussian of the block; the extremes by wave reductions (LDS
        // atomics from all 64 lanes on one address would serialise)
        const int g = g0 + lane;
        const bool ok = lane < GB && g < n;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float xk = ok ? J.means[(size_t)k * n + g] - J.bmin[k] : 0.0f;
#pragma unroll
            for (int l = 0; l < L; ++l) {
                int i0;
                float w;
                grid_coord(xk, J.gscale[l][k], J.res[l][k], i0, w);
                int lo = ok ? i0 : 0x7fffffff, hi = ok ? i0 : -1;
#pragma unroll
                for (int o = 32; o >= 1; o >>= 1) {
                    lo = min(lo, __shfl_xor(lo, o, 64));
                    hi = max(hi, __shfl_xor(hi, o, 64));
                }
                if (lane == 0) {
                    s_lo[l * 3 + k] = lo;
                    s_hi[l * 3 + k] = hi;
                }
            }
        }
    }
    __syncthreads();
    if (tid == 0) {
        int used = 0;
        for (int l = 0; l < L; ++l) {
            int it;
            float wt;
            grid_coord(J.t, J.gscale[l][3], J.res[l][3], it, wt);
            for (int p = 0; p < 6; ++p) {
                const int a = axis_a(p), b = axis_b(p), q = l * 6 + p;
                const int la = s_lo[l * 3 + a], ha = s_hi[l * 3 + a];
                const int lb = b == 3 ? it : s_lo[l * 3 + b], hb = b == 3 ? it : s_hi[l * 3 + b];
                const int wn = ha - la + 2, wm = hb - lb + 2;
                const int need = wn * wm * WF;
                if (ha >= la && hb >= lb && used + need <= win_cap) {
                    s_woff[q] = used;
                    s_wa0[q] = la;
                    s_wb0[q] = lb;
                    s_wn[q] = wn;
                    s_wm[q] = wm;
                    used += need;
                } else {
                    s_woff[q] = -1;
                }
            }
        }
        s_wtotal = used;
    }
    __syncthreads();
    for (int i = tid; i < s_wtotal; i += kThreads) s_win[i] = 0.0f;
    __syncthreads();
    // ---- encoder backward (Eq. 7).  The Gaussians of a wave are taken 4 NPASS
    // apart in the block (Gaussian j of wave w in pass p is j * 4 NPASS +
    // 4 p + w): spatially ordered neighbours share plane cells, and the LDS
    // adds of one instruction into a shared cell serialise.
#pragma unroll
    for (int pass = 0; pass < NPASS; ++pass) {
        constexpr int WPG = GPP / 4;   // Gaussians per wave and pass
        const int q = tid / LPG;
        const int gl = (q % WPG) * (4 * NPASS) + pass * 4 + q / WPG, c4 = tid % LPG, g = g0 + gl;
        const bool valid = gl < GB && g < n;
        float x[4];
        bool inner[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float m = valid ? J.means[(size_t)k * n + g] : J.bmin[k];
            x[k] = m - J.bmin[k];
            inner[k] = m > J.bmin[k] && m < J.bmax[k];   // strictly inside the box: the clamp has slope 1
        }
        x[3] = J.t;
        float dx3[3] = {0.f, 0.f, 0.f};
        if (valid) {
#pragma unroll
            for (int l = 0; l < L; ++l) {
                float4 val[6];
                float wa_[6], wb_[6];
                size_t off[6];
                int na_[6], ia_[6], ib_[6];
#pragma unroll
                for (int p = 0; p < 6; ++p) {
                    const int a = axis_a(p), b = axis_b(p);
                    const int na = J.res[l][a], nb = J.res[l][b];
                    int ia, ib;
                    float wa, wb;
                    grid_coord(x[a], J.gscale[l][a], na, ia, wa);
                    grid_coord(x[b], J.gscale[l][b], nb, ib, wb);
                    off[p] = ((size_t)ib * na + ia) * F + 4 * c4;
                    na_[p] = na;
                    ia_[p] = ia;
                    ib_[p] = ib;
                    wa_[p] = wa;
                    wb_[p] = wb;
                    const float *base = J.planes[l * 6 + p] + off[p];
                    const float4 v00 = *reinterpret_cast<const float4 *>(base);
                    const float4 v10 = *reinterpret_cast<const float4 *>(base + F);
                    const float4 v01 = *reinterpret_cast<const float4 *>(base + (size_t)na * F);
                    const float4 v11 = *reinterpret_cast<const float4 *>(base + (size_t)na * F + F);
                    const float w00 = (1.0f - wa) * (1.0f - wb), w10 = wa * (1.0f - wb);
                    const float w01 = (1.0f - wa) * wb, w11 = wa * wb;
                    val[p].x = w00 * v00.x + w10 * v10.x + w01 * v01.x + w11 * v11.x;
                    val[p].y = w00 * v00.y + w10 * v10.y + w01 * v01.y + w11 * v11.y;
                    val[p].z = w00 * v00.z + w10 * v10.z + w01 * v01.z + w11 * v11.z;
                    val[p].w = w00 * v00.w + w10 * v10.w + w01 * v01.w + w11 * v11.w;
                }
                const float *df = s_fh + gl * FH + l * F + 4 * c4;
                const float4 dF = make_float4(df[0], df[1], df[2], df[3]);
                // products of the other five planes: prefix x suffix
                float4 pre[6], suf[6];
                pre[0] = make_float4(1.f, 1.f, 1.f, 1.f);
                suf[5] = pre[0];
#pragma unroll
                for (int p = 1; p < 6; ++p) {
                    pre[p] = make_float4(pre[p - 1].x * val[p - 1].x, pre[p - 1].y * val[p - 1].y,
                                         pre[p - 1].z * val[p - 1].z, pre[p - 1].w * val[p - 1].w);
                    const int q = 5 - p;
                    suf[q] = make_float4(suf[q + 1].x * val[q + 1].x, suf[q + 1].y * val[q + 1].y,
                                         suf[q + 1].z * val[q + 1].z, suf[q + 1].w * val[q + 1].w);
                }
#pragma unroll
                for (int p = 0; p < 6; ++p) {
                    const float4 dv = make_float4(dF.x * pre[p].x * suf[p].x, dF.y * pre[p].y * suf[p].y,
                                                  dF.z * pre[p].z * suf[p].z, dF.w * pre[p].w * suf[p].w);
                    const float wa = wa_[p], wb = wb_[p];
                    const float w00 = (1.0f - wa) * (1.0f - wb), w10 = wa * (1.0f - wb);
                    const float w01 = (1.0f - wa) * wb, w11 = wa * wb;
                    const size_t rowF = (size_t)na_[p] * F;
                    const float dvv[4] = {dv.x, dv.y, dv.z, dv.w};
                    const int q = l * 6 + p;
                    const int wo = s_woff[q];
                    if (wo >= 0) {
                        // this block's window of the plane, in LDS
                        const int wrow = s_wn[q] * WF;
                        float *lb = s_win + wo + ((ib_[p] - s_wb0[q]) * s_wn[q] + (ia_[p] - s_wa0[q])) * WF + 4 * c4;
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            if (dvv[c] == 0.0f) continue;
                            if (w00 != 0.0f) atomicAdd(lb + c, w00 * dvv[c]);
                            if (w10 != 0.0f) atomicAdd(lb + WF + c, w10 * dvv[c]);
                            if (w01 != 0.0f) atomicAdd(lb + wrow + c, w01 * dvv[c]);
                            if (w11 != 0.0f) atomicAdd(lb + wrow + WF + c, w11 * dvv[c]);
                        }
                    } else {
                        float *gb = J.d_planes[q] + off[p];
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            if (dvv[c] == 0.0f) continue;
                            if (w00 != 0.0f) atomicAdd(gb + c, w00 * dvv[c]);
                            if (w10 != 0.0f) atomicAdd(gb + F + c, w10 * dvv[c]);
                            if (w01 != 0.0f) atomicAdd(gb + rowF + c, w01 * dvv[c]);
                            if (w11 != 0.0f) atomicAdd(gb + rowF + F + c, w11 * dvv[c]);
                        }
                    }
                    // slopes of the bilinear query along its two grid axes
                    const int a = axis_a(p), b = axis_b(p);
                    const float *base = J.planes[l * 6 + p] + off[p];
                    const float4 v00 = *reinterpret_cast<const float4 *>(base);
                    const float4 v10 = *reinterpret_cast<const float4 *>(base + F);
                    const float4 v01 = *reinterpret_cast<const float4 *>(base + rowF);
                    const float4 v11 = *reinterpret_cast<const float4 *>(base + rowF + F);
                    const float sa = dv.x * ((1.0f - wb) * (v10.x - v00.x) + wb * (v11.x - v01.x)) +
                                     dv.y * ((1.0f - wb) * (v10.y - v00.y) + wb * (v11.y - v01.y)) +
                                     dv.z * ((1.0f - wb) * (v10.z - v00.z) + wb * (v11.z - v01.z)) +
                                     dv.w * ((1.0f - wb) * (v10.w - v00.w) + wb * (v11.w - v01.w));
                    const float sb = dv.x * ((1.0f - wa) * (v01.x - v00.x) + wa * (v11.x - v10.x)) +
                                     dv.y * ((1.0f - wa) * (v01.y - v00.y) + wa * (v11.y - v10.y)) +
                                     dv.z * ((1.0f - wa) * (v01.z - v00.z) + wa * (v11.z - v10.z)) +
                                     dv.w * ((1.0f - wa) * (v01.w - v00.w) + wa * (v11.w - v10.w));
                    if (a < 3 && inner[a]) dx3[a] += sa * J.gscale[l][a];
                    if (b < 3 && inner[b]) dx3[b] += sb * J.gscale[l][b];
                }
            }
        }
        // sum over the LPG lanes of this Gaussian
#pragma unroll
        for (int o = LPG / 2; o >= 1; o >>= 1) {
#pragma unroll
            for (int k = 0; k < 3; ++k) dx3[k] += __shfl_xor(dx3[k], o, 64);
        }
        if (c4 == 0 && valid) {
#pragma unroll
            for (int k = 0; k < 3; ++k) s_dm[gl * 3 + k] += dx3[k];
        }
    }
    __syncthreads();
    if (tid < GB && g0 + tid < n) {
#pragma unroll
        for (int k = 0; k < 3; ++k) J.d_means[(size_t)k * n + g0 + tid] = s_dm[tid * 3 + k];
    }
    // the block's windows into the plane gradients, one global atomic per
    // nonzero value (consecutive threads: consecutive values of a row)
    for (int q = 0; q < L * 6; ++q) {
        const int wo = s_woff[q];
        if (wo < 0) continue;
        const int wn = s_wn[q], cnt = wn * s_wm[q] * F;
        const int na = J.res[q / 6][axis_a(q % 6)];
        float *dst = J.d_planes[q] + ((size_t)s_wb0[q] * na + s_wa0[q]) * F;
        for (int i = tid; i < cnt; i += kThreads) {
            const int cell = i / F, f = i - cell * F;
            const float v = s_win[wo + cell * WF + f];
            if (v == 0.0f) continue;
            const int cb = cell / wn, ca = cell - cb * wn;
            atomicAdd(dst + ((size_t)cb * na + ca) * F + f, v);
        }
    }
}

// Up to 40 arrays cleared in one launch.
struct FillList {
    float *ptr[40];
    uint32_t count[40];
    int n;
};

__global__ void k_fill_list(FillList f) {
    const int a = blockIdx.y;
    if (a >= f.n) return;
    float *p = f.ptr[a];
    for (uint32_t i = blockIdx.x * blockDim.x + threadIdx.x; i < f.count[a]; i += gridDim.x * blockDim.x) p[i] = 0.0f;
}

using BwdKernel = void (*)(BwdJob, int);
struct BwdEntry {
    int feat, scales, hidden;
    BwdKernel fn, fn_small;   // kGB and kGBSmall Gaussians per block
};
#define G4D_BWD_ENTRY(F, L, H) {F, L, H, k_deform_bwd<F, L, H, kGB>, k_deform_bwd<F, L, H, kGBSmall>}
const BwdEntry kBwdKernels[] = {
    G4D_BWD_ENTRY(16, 1, 32), G4D_BWD_ENTRY(16, 1, 64), G4D_BWD_ENTRY(16, 1, 128), G4D_BWD_ENTRY(16, 2, 64),
    G4D_BWD_ENTRY(16, 3, 64), G4D_BWD_ENTRY(32, 1, 64), G4D_BWD_ENTRY(32, 2, 64), G4D_BWD_ENTRY(32, 2, 128),
    G4D_BWD_ENTRY(32, 3, 64), G4D_BWD_ENTRY(32, 3, 128),
};

size_t bwd_smem(int gb, int K, int HID, int rows) { return (size_t)bwd_lds(gb, K, HID, rows).total * 4; }

}  // namespace

g4d_status deform_backward(const g4d_gaussians *G, const g4d_planes *P, const g4d_mlp *M, float t,
                           const g4d_splats_grad *gout, const g4d_deform_grad *d, hipStream_t s) {
    if (!G || !P || !M || !gout || !d) return G4D_EINVAL;
    if (G->n < 0 || G->sh_degree < 0 || G->sh_degree > 3 || !(t >= 0.0f && t <= 1.0f)) return G4D_EINVAL;
    if (P->n_scales < 1 || P->n_scales > kMaxScalesB || (P->feat != 16 && P->feat != 32)) return G4D_EINVAL;
    for (int k = 0; k < 3; ++k)
        if (!(P->bmax[k] > P->bmin[k])) return G4D_EINVAL;
    if (M->in_dim != P->feat * P->n_scales) return G4D_EINVAL;
    if (M->precision != G4D_MLP_F32) return G4D_EUNSUPPORTED;
    if ((M->wc == nullptr) != (M->bc == nullptr) || (M->wa == nullptr) != (M->ba == nullptr)) return G4D_EINVAL;
    const BwdEntry *ke = nullptr;
    for (const auto &e : kBwdKernels)
        if (e.feat == P->feat && e.scales == P->n_scales && e.hidden == M->hidden) ke = &e;
    if (!ke) return G4D_EUNSUPPORTED;
    const int n = G->n, hid = M->hidden, K = M->in_dim;
    const int n_sh = 3 * (G->sh_degree + 1) * (G->sh_degree + 1);
    BwdJob J{};
    J.means = G->means; J.log_scales = G->log_scales; J.quats = G->quats; J.opac = G->opacity_logits; J.sh = G->sh;
    J.w1 = M->w1; J.b1 = M->b1;
    const float *hw[5] = {M->wx, M->wr, M->ws, M->wc, M->wa};
    const float *hb[5] = {M->bx, M->br, M->bs, M->bc, M->ba};
    const int hr[5] = {3, 4, 3, M->wc ? n_sh : 0, M->wa ? 1 : 0};
    float *dhw[5] = {d->wx, d->wr, d->ws, d->wc, d->wa};
    float *dhb[5] = {d->bx, d->br, d->bs, d->bc, d->ba};
    int rows = 0;
    for (int q = 0; q < 5; ++q) {
        J.hw[q] = hw[q]; J.hb[q] = hb[q]; J.hrows[q] = hr[q];
        J.d_hw[q] = dhw[q]; J.d_hb[q] = dhb[q];
        if (hr[q] && (!hw[q] || !hb[q] || !dhw[q] || !dhb[q])) return G4D_EINVAL;
        rows += hr[q];
    }
    if (!M->w1 || !M->b1 || !d->w1 || !d->b1) return G4D_EINVAL;
    J.d_w1 = d->w1;
    J.d_b1 = d->b1;
    J.g_means = gout->means; J.g_scales = gout->scales; J.g_quats = gout->quats; J.g_opac = gout->opacity;
    J.g_sh = gout->sh;
    J.d_means = d->means; J.d_log_scales = d->log_scales; J.d_quats = d->quats; J.d_opac = d->opacity_logits;
    J.d_sh = d->sh;
    if (n > 0 && (!G->means || !G->log_scales || !G->quats || !G->opacity_logits || !gout->means ||
                  !gout->scales || !gout->quats || !gout->opacity || !d->means || !d->log_scales || !d->quats ||
                  !d->opacity_logits))
        return G4D_EINVAL;
    if (n > 0 && (M->wc || d->sh) && !gout->sh) return G4D_EINVAL;
    FillList fl{};
    auto add = [&](float *p, size_t cnt) {
        if (p && cnt) { fl.ptr[fl.n] = p; fl.count[fl.n] = (uint32_t)cnt; ++fl.n; }
    };
    for (int l = 0; l < P->n_scales; ++l) {
        for (int p = 0; p < 6; ++p) {
            static const int ax[6][2] = {{0, 1}, {0, 2}, {1, 2}, {0, 3}, {1, 3}, {2, 3}};
            if (!P->plane[l][p] || !d->plane[l][p]) return G4D_EINVAL;
            J.planes[l * 6 + p] = P->plane[l][p];
            J.d_planes[l * 6 + p] = d->plane[l][p];
            add(d->plane[l][p], (size_t)P->res[l][ax[p][0]] * P->res[l][ax[p][1]] * P->feat);
        }
        for (int k = 0; k < 4; ++k) {
            if (P->res[l][k] < 2) return G4D_EINVAL;
            J.res[l][k] = P->res[l][k];
        }
        for (int k = 0; k < 3; ++k)
            J.gscale[l][k] = (float)((double)(P->res[l][k] - 1) / ((double)P->bmax[k] - (double)P->bmin[k]));
        J.gscale[l][3] = (float)(P->res[l][3] - 1);
    }
    add(d->w1, (size_t)hid * K);
    add(d->b1, (size_t)hid);
    for (int q = 0; q < 5; ++q)
        if (hr[q]) { add(dhw[q], (size_t)hr[q] * hid); add(dhb[q], (size_t)hr[q]); }
    for (int k = 0; k < 3; ++k) { J.bmin[k] = P->bmin[k]; J.bmax[k] = P->bmax[k]; }
    J.n = n;
    J.n_sh_rows = n_sh;
    J.t = t;
    hipLaunchKernelGGL(k_fill_list, dim3(64, (unsigned)fl.n), dim3(256), 0, s, fl);
    if (n > 0) {
        const bool small = n <= kSmallN;
        const int gb = small ? kGBSmall : kGB;
        const BwdKernel fn = small ? ke->fn_small : ke->fn;
        const size_t smem = bwd_smem(gb, K, hid, rows);
        static std::atomic<uint64_t> attr_done[2][sizeof(kBwdKernels) / sizeof(kBwdKernels[0])];
        const size_t idx = (size_t)(ke - kBwdKernels);
        // the largest head count (64 rows) sets the limit
        if (g4d_status st = ensure_max_lds(reinterpret_cast<const void *>(fn), attr_done[small][idx],
                                           (int)std::min(bwd_smem(gb, K, hid, 64), kLdsMax)))
            return st;
        hipLaunchKernelGGL(fn, dim3((n + gb - 1) / gb), dim3(kThreads), smem, s, J, rows);
    }
    G4D_HIP_CHECK(hipGetLastError());
    return G4D_OK;
}

}  // namespace g4d

extern "C" g4d_status g4d_deform_backward(const g4d_gaussians *G, const g4d_planes *P, const g4d_mlp *M, float t,
                                          const g4d_splats_grad *grad_out, const g4d_deform_grad *grad,
                                          void *stream) {
    return g4d::deform_backward(G, P, M, t, grad_out, grad, reinterpret_cast<hipStream_t>(stream));
}
