// Gaussian deformation field on gfx950 (Sec. 4.2, Eq. 7-8).
//
// One thread block of 256 threads (four wave64s) deforms 64 Gaussians:
//   A. HexPlane encoder (Eq. 7): for every scale and each of the six planes,
//      an align-corners bilinear query at the canonical mean (and t), the
//      element-wise product over the six planes, concatenation over scales.
//      feat/4 lanes share one Gaussian and each loads float4 slices of the
//      four channels-last corner rows, so a corner of a 32-feature plane is
//      one 128-byte line read by eight lanes.  f_h stays in LDS.
//   B. Feature merger h = ReLU(W1 f_h + b1) as a [64 x in] x [in x hidden]
//      product on MFMA (v_mfma_f32_16x16x4_f32, or 16x16x32 bf16 with FP32
//      accumulation in the bf16 mode); each wave owns 16 Gaussians.
//   C. The heads, concatenated into one [hidden x 16 NT] matrix (rows dx 0-2,
//      dr 3-6, ds 7-9; with the colour and opacity heads of the appendix,
//      dC 10 .. 10 + 3 (d+1)^2 - 1 and dalpha next; zero padding) on MFMA.
//   D. Eq. 8 and activations: X + dX, exp(log s + ds), normalise(r + dr),
//      sigmoid(opacity logit [+ dalpha]), SH coefficients C [+ dC]; in a
//      composition, the scene's placement and its index range of the
//      combined set; structure-of-arrays stores.
// A launch carries up to G4D_MAX_BATCH_JOBS jobs (continuous batching); a
// block never mixes jobs, so a job's result does not depend on its batch.
#include "g4d_internal.h"

#include <cmath>
#include <vector>

namespace g4d {

constexpr int kMaxScales = 3;   // scales the kernels support (<= G4D_MAX_SCALES)
static_assert(kMaxScales <= G4D_MAX_SCALES, "scale count");

// One job of a launch.  Kept compact: a launch passes G4D_MAX_BATCH_JOBS of
// them by value as kernel arguments (at most 4 KB).
struct DeformJob {
    const float *means, *log_scales, *quats, *opac;
    const float *planes[kMaxScales * 6];
    const float *w1, *b1, *wx, *bx, *wr, *br, *ws, *bs;
    const float *wc, *bc, *wa, *ba;      // colour / opacity heads (null when absent)
    const float *sh_in;                  // canonical SH coefficients [n_sh_in][n]
    float *out_means, *out_scales, *out_quats, *out_opac;
    float *out_sh;                       // [n_sh_out][out_stride] (C [+ dC], zero rows past n_sh_in)
    int16_t n_sh_head;                   // 3 (d+1)^2 colour-head rows, 0 without a colour head
    int16_t n_sh_in, n_sh_out;           // SH rows read / written (0: SH not written)
    int16_t placed;                      // apply the placement below
    int out_stride, out_offset;          // output row stride and this job's first index
    float place_q[4], place_s, place_t[3];   // unit quaternion, uniform scale, translation
    float *out_features;                 // non-null: write f_h and stop after phase A
    int res[kMaxScales][4];
    float gscale[kMaxScales][4];         // (res - 1) / (bmax - bmin) per axis; res_t - 1 for t
    float bmin[3];
    int n;
    float t;
    int block_begin;
};

struct DeformBatch {
    int n_jobs;
    int n_blocks;   // blocks of work (the grid is padded to a multiple of 8)
    DeformJob job[G4D_MAX_BATCH_JOBS];
};
static_assert(sizeof(DeformBatch) <= 4096, "a launch's jobs travel as kernel arguments");

namespace {

constexpr int kGB = 64;        // Gaussians per block
constexpr int kThreads = 256;
static_assert(kGB == 64 && kThreads >= 3 * 64, "Eq. 8 phase: one Gaussian per lane, one wave per output group");
static_assert(48 * kGB % kThreads == 0, "SH phase: whole rows of (d+1)^2 x 3 <= 48 coefficients per thread");

typedef float float4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
    uint32_t u = __float_as_uint(f);
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

// Plane (a, b) axis pairs in storage order xy, xz, yz, xt, yt, zt.
__device__ constexpr int plane_axis_a(int p) { return p == 2 ? 1 : (p == 5 ? 2 : (p == 4 ? 1 : 0)); }
__device__ constexpr int plane_axis_b(int p) { return p == 0 ? 1 : (p == 1 || p == 2 ? 2 : 3); }

// Align-corners grid coordinate: with u = 2 (x - bmin) / (bmax - bmin) - 1,
// g = (u + 1) / 2 (n - 1) = (x - bmin) * scale, evaluated with two roundings.
__device__ __forceinline__ void grid_coord(float x, float scale, int n, int &i0, float &w) {
    float g = x * scale;
    g = fminf(fmaxf(g, 0.0f), (float)(n - 1));
    int i = (int)floorf(g);
    i = min(i, n - 2);
    i0 = i;
    w = g - (float)i;
}

template <int F, int L, int HID, bool BF16, int NT>
struct Smem {
    static constexpr int K = F * L;                        // in_dim
    static constexpr int KP = BF16 ? ((K + 31) / 32) * 32 : K;   // padded K
    static constexpr int FH_LD = BF16 ? KP + 8 : K + 4;    // row strides (elements)
    static constexpr int H_LD = BF16 ? HID + 8 : HID + 4;
    static constexpr int W1_LD = FH_LD;
    static constexpr int W2_LD = H_LD;
    using E = typename std::conditional<BF16, uint16_t, float>::type;
    static constexpr size_t fh_bytes = (size_t)kGB * FH_LD * sizeof(E);
    static constexpr size_t h_bytes = (size_t)kGB * H_LD * sizeof(E);
    static constexpr size_t act_bytes = fh_bytes > h_bytes ? fh_bytes : h_bytes;   // f_h, then h
    static constexpr int DS = 16 * NT + 1;                 // delta row stride (floats)
    static constexpr size_t w2_bytes = (size_t)16 * NT * W2_LD * sizeof(E);
    static constexpr size_t delta_bytes = (size_t)kGB * DS * sizeof(float);
    static constexpr size_t bias_bytes = (size_t)(HID + 16 * NT) * sizeof(float);
    // FP32 W1 is held in registers as MFMA fragments instead of an LDS copy
    // when that copy would hold the kernel below 3 blocks per CU (160 KB of
    // LDS) and dropping it lets more blocks in.  Otherwise the LDS copy is
    // the faster of the two: its global loads are coalesced.
    static constexpr size_t kLdsPerCu = 160 * 1024;
    static constexpr size_t w1_lds_bytes = (size_t)HID * W1_LD * sizeof(E);
    static constexpr size_t lds_without_w1 = act_bytes + bias_bytes + w2_bytes + delta_bytes;
    static constexpr size_t lds_with_w1 = act_bytes + bias_bytes +
        (w1_lds_bytes > w2_bytes + delta_bytes ? w1_lds_bytes : w2_bytes + delta_bytes);
    static constexpr bool W1_REGS = !BF16 && kLdsPerCu / lds_with_w1 < 3 &&
                                    kLdsPerCu / lds_without_w1 > kLdsPerCu / lds_with_w1;
    static constexpr size_t w1_bytes = W1_REGS ? 0 : w1_lds_bytes;
    // FP32 decoders whose W1 rows in flight through the encoder take at most
    // 16 registers fit 128 VGPRs without spilling: held to four waves per
    // SIMD (more plane gathers in flight); the others are left unconstrained
    static constexpr int W1_IN_FLIGHT = W1_REGS ? 0 : (HID * KP + 255) / 256;
    static constexpr int WAVES = !BF16 && NT == 1 && W1_IN_FLIGHT <= 16 ? 4 : 1;
    // W1 is dead once h is computed: the heads' weights and the deltas reuse its space
    static constexpr size_t wreg_bytes = w1_bytes > w2_bytes + delta_bytes ? w1_bytes : w2_bytes + delta_bytes;
    static constexpr size_t total = act_bytes + wreg_bytes + bias_bytes;
};

// Row r of the concatenated decoder heads: its weights (null for padding)
// and its bias.
__device__ __forceinline__ const float *head_w(const DeformJob &job, int r, int hid) {
    if (r < 3) return job.wx + r * hid;
    if (r < 7) return job.wr + (r - 3) * hid;
    if (r < 10) return job.ws + (r - 7) * hid;
    if (r < 10 + job.n_sh_head) return job.wc + (r - 10) * hid;
    if (r == 10 + job.n_sh_head && job.wa) return job.wa;
    return nullptr;
}
__device__ __forceinline__ float head_b(const DeformJob &job, int r) {
    if (r < 3) return job.bx[r];
    if (r < 7) return job.br[r - 3];
    if (r < 10) return job.bs[r - 7];
    if (r < 10 + job.n_sh_head) return job.bc[r - 10];
    if (r == 10 + job.n_sh_head && job.wa) return job.ba[0];
    return 0.0f;
}

// NT: 16-row tiles of decoder heads (1: dx dr ds; 4: with the colour and
// opacity heads, up to SH degree 3)
template <int F, int L, int HID, bool BF16, int NT>
__device__ __forceinline__ void deform_block(const DeformBatch &batch) {
    using S = Smem<F, L, HID, BF16, NT>;
    using E = typename S::E;
    constexpr int K = S::K;
    constexpr int KP = S::KP;
    extern __shared__ __attribute__((aligned(16))) unsigned char smem[];
    E *s_act = reinterpret_cast<E *>(smem);
    E *s_w1 = reinterpret_cast<E *>(smem + S::act_bytes);
    E *s_w2 = reinterpret_cast<E *>(smem + S::act_bytes);   // after phase B (W1 in registers: after the encoder)
    float *s_delta = reinterpret_cast<float *>(smem + S::act_bytes + S::w2_bytes);          // after phase C
    float *s_b1 = reinterpret_cast<float *>(smem + S::act_bytes + S::wreg_bytes);
    float *s_b2 = s_b1 + HID;

    // Block b runs on XCD b % 8; each XCD takes a contiguous run of the
    // work blocks, so spatially ordered Gaussians keep each XCD's share of
    // the feature planes compact in its own L2.
    const int per = (int)gridDim.x / 8;
    const int wb = ((int)blockIdx.x % 8) * per + (int)blockIdx.x / 8;
    if (wb >= batch.n_blocks) return;
    // job of this block
    int j = 0;
    for (int q = 1; q < batch.n_jobs; ++q)
        if (wb >= batch.job[q].block_begin) j = q;
    const DeformJob &job = batch.job[j];
    const int g0 = (wb - job.block_begin) * kGB;
    const int n = job.n;
    const int tid = threadIdx.x;
    const bool features_only = job.out_features != nullptr;
    // inputs of Eq. 8 for this block's Gaussians, loaded now so that their
    // latency hides behind the encoder: wave 0 means + opacity logit, wave 1
    // quaternion, wave 2 log-scales (lane = Gaussian)
    const int wave_d = tid >> 6, lane_g = tid & 63, dg = g0 + lane_g;
    float pin[4] = {0.0f, 0.0f, 0.0f, 0.0f};
    if (!features_only && dg < n) {
        if (wave_d == 0) {
#pragma unroll
            for (int k = 0; k < 3; ++k) pin[k] = job.means[(size_t)k * n + dg];
            pin[3] = job.opac[dg];
        } else if (wave_d == 1) {
#pragma unroll
            for (int k = 0; k < 4; ++k) pin[k] = job.quats[(size_t)k * n + dg];
        } else if (wave_d == 2) {
#pragma unroll
            for (int k = 0; k < 3; ++k) pin[k] = job.log_scales[(size_t)k * n + dg];
        }
    }

    // ---- decoder weights (rows of W1; heads padded to 16 rows): the loads
    // are issued here and stay in flight through the encoder's gathers: rows
    // of W1 for an LDS copy after the encoder or, with W1 in registers, each
    // wave's W1 fragments for phase B (output column tiles w, w + 4: lane
    // (r, k) holds W1[c*16 + r][4 kk + k]).
    constexpr bool kW1Regs = S::W1_REGS;
    constexpr int N1 = kW1Regs ? 0 : (HID * KP + kThreads - 1) / kThreads;
    constexpr int N2 = (16 * NT * HID + kThreads - 1) / kThreads;
    constexpr int NC1 = kW1Regs ? (HID / 16 + 3) / 4 : 0;
    // every wave owns a column tile in each of its NC1 groups unless HID / 16
    // is not a multiple of 4 (HID = 32: waves 2 and 3 idle in phase B)
    constexpr bool kAllOwn = (HID / 16) % 4 == 0;
    float v1[N1 > 0 ? N1 : 1], v2[N2];
    float w1f[NC1 > 0 ? NC1 : 1][kW1Regs ? K / 4 : 1];
    float vb1 = 0.0f, vb2 = 0.0f;
    const int wave_u = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (!features_only) {
#pragma unroll
        for (int q = 0; q < N1; ++q) {
            const int i = tid + q * kThreads;
            const int r = i / KP, c = i - r * KP;
            v1[q] = (i < HID * KP && c < K) ? job.w1[r * K + c] : 0.0f;
        }
        if constexpr (kW1Regs) {
            const int lr = tid & 15, lq = (tid >> 4) & 3;
#pragma unroll
            for (int ci = 0; ci < NC1; ++ci) {
                const int c = wave_u + 4 * ci;
#pragma unroll
                for (int kk = 0; kk < K / 4; ++kk)
                    w1f[ci][kk] = (kAllOwn || c < HID / 16) ? job.w1[(size_t)(c * 16 + lr) * K + kk * 4 + lq] : 0.0f;
            }
        }
#pragma unroll
        for (int q = 0; q < N2; ++q) {
            const int i = tid + q * kThreads;
            const int r = i / HID, c = i - r * HID;
            const float *src = i < 16 * NT * HID ? head_w(job, r, HID) : nullptr;
            v2[q] = src ? src[c] : 0.0f;
        }
        vb1 = tid < HID ? job.b1[tid] : 0.0f;
        if (tid < 16 * NT) vb2 = head_b(job, tid);
    }

    // ---- A. encoder: f_h for 64 Gaussians
    constexpr int LPG = F / 4;                 // lanes per Gaussian
    constexpr int GPP = kThreads / LPG;        // Gaussians per pass
#pragma unroll
    for (int pass = 0; pass < kGB / GPP; ++pass) {
        const int gl = pass * GPP + tid / LPG;
        const int c4 = tid % LPG;
        const int g = g0 + gl;
        float x[4];   // offsets from the box corner; t for the time axis
        const bool valid = g < n;
        if (valid) {
#pragma unroll
            for (int k = 0; k < 3; ++k) x[k] = job.means[(size_t)k * n + g] - job.bmin[k];
        } else {
            x[0] = x[1] = x[2] = 0.0f;
        }
        x[3] = job.t;
#pragma unroll
        for (int l = 0; l < L; ++l) {
            float4 prod = make_float4(1.0f, 1.0f, 1.0f, 1.0f);
#pragma unroll
            for (int p = 0; p < 6; ++p) {
                const int a = plane_axis_a(p), b = plane_axis_b(p);
                const int na = job.res[l][a], nb = job.res[l][b];
                int ia, ib;
                float wa, wb;
                grid_coord(x[a], job.gscale[l][a], na, ia, wa);
                grid_coord(x[b], job.gscale[l][b], nb, ib, wb);
                const float *base = job.planes[l * 6 + p] + ((size_t)ib * na + ia) * F + 4 * c4;
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
            if (!valid) prod = make_float4(0.0f, 0.0f, 0.0f, 0.0f);
            const int col = l * F + 4 * c4;
            if (features_only) {
                if (valid)
                    *reinterpret_cast<float4 *>(job.out_features + (size_t)g * K + col) = prod;
            } else if constexpr (BF16) {
                uint16_t *dst = reinterpret_cast<uint16_t *>(s_act) + gl * S::FH_LD + col;
                dst[0] = f32_to_bf16_rne(prod.x);
                dst[1] = f32_to_bf16_rne(prod.y);
                dst[2] = f32_to_bf16_rne(prod.z);
                dst[3] = f32_to_bf16_rne(prod.w);
            } else {
                *reinterpret_cast<float4 *>(reinterpret_cast<float *>(s_act) + gl * S::FH_LD + col) = prod;
            }
        }
    }
    if (features_only) return;
    {
#pragma unroll
        for (int q = 0; q < N1; ++q) {
            const int i = tid + q * kThreads;
            if (i < HID * KP) {
                const int r = i / KP, c = i - r * KP;
                if constexpr (BF16) s_w1[r * S::W1_LD + c] = f32_to_bf16_rne(v1[q]);
                else s_w1[r * S::W1_LD + c] = v1[q];
            }
        }
        if constexpr (kW1Regs) {
            // no W1 copy to alias: the heads' weights go to LDS now
#pragma unroll
            for (int q = 0; q < N2; ++q) {
                const int i = tid + q * kThreads;
                if (i < 16 * NT * HID) {
                    const int r = i / HID, c = i - r * HID;
                    s_w2[r * S::W2_LD + c] = v2[q];
                }
            }
        }
        if (tid < HID) s_b1[tid] = vb1;
        if (tid < 16 * NT) s_b2[tid] = vb2;
    }
    if constexpr (BF16 && KP > K) {
        // zero the padding columns K..KP of f_h
        for (int i = tid; i < kGB * (KP - K); i += kThreads) {
            int r = i / (KP - K), c = K + i % (KP - K);
            s_act[r * S::FH_LD + c] = 0;
        }
    }
    __syncthreads();

    const int wave = tid >> 6;
    const int lane = tid & 63;
    const int lrow = lane & 15;        // row (A) / column (B) inside a 16x16 tile
    const int lk = lane >> 4;          // k group of this lane
    const int row0 = wave * 16;        // this wave's Gaussians

    // ---- B. h = ReLU(W1 f_h + b1)
    if constexpr (kW1Regs) {
        // wave w computes output column tiles w, w + 4 for all 64 Gaussians,
        // B fragments from registers (the same products in the same k order
        // as the row split below, so h does not depend on the split)
        const float *fh = reinterpret_cast<const float *>(s_act);
        float4_t accb[NC1 > 0 ? NC1 : 1][kGB / 16];
#pragma unroll
        for (int ci = 0; ci < NC1; ++ci)
#pragma unroll
            for (int rt = 0; rt < kGB / 16; ++rt) accb[ci][rt] = float4_t{0.0f, 0.0f, 0.0f, 0.0f};
#pragma unroll
        for (int kk = 0; kk < K / 4; ++kk) {
#pragma unroll
            for (int rt = 0; rt < kGB / 16; ++rt) {
                const float a = fh[(rt * 16 + lrow) * S::FH_LD + kk * 4 + lk];
#pragma unroll
                for (int ci = 0; ci < NC1; ++ci)
                    if (kAllOwn || wave_u + 4 * ci < HID / 16)
                        accb[ci][rt] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, w1f[ci][kk], accb[ci][rt], 0, 0, 0);
            }
        }
        __syncthreads();   // all waves done reading f_h before h overwrites it
#pragma unroll
        for (int ci = 0; ci < NC1; ++ci) {
            const int c = wave_u + 4 * ci;
            if (kAllOwn || c < HID / 16) {
                const int col = c * 16 + lrow;
                const float bias = s_b1[col];
#pragma unroll
                for (int rt = 0; rt < kGB / 16; ++rt)
#pragma unroll
                    for (int i = 0; i < 4; ++i)
                        reinterpret_cast<float *>(s_act)[(rt * 16 + 4 * lk + i) * S::H_LD + col] =
                            fmaxf(accb[ci][rt][i] + bias, 0.0f);
            }
        }
    } else {
        // wave w computes its 16 Gaussians' rows, W1 tiles from LDS
        float4_t acc[HID / 16];
#pragma unroll
        for (int c = 0; c < HID / 16; ++c) acc[c] = float4_t{0.0f, 0.0f, 0.0f, 0.0f};
        if constexpr (!BF16) {
            const float *fh = reinterpret_cast<const float *>(s_act);
            const float *w1 = reinterpret_cast<const float *>(s_w1);
#pragma unroll 4
            for (int kk = 0; kk < K / 4; ++kk) {
                const float a = fh[(row0 + lrow) * S::FH_LD + kk * 4 + lk];
#pragma unroll
                for (int c = 0; c < HID / 16; ++c) {
                    const float b = w1[(c * 16 + lrow) * S::W1_LD + kk * 4 + lk];
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc[c], 0, 0, 0);
                }
            }
        } else {
            const uint16_t *fh = reinterpret_cast<const uint16_t *>(s_act);
            const uint16_t *w1 = reinterpret_cast<const uint16_t *>(s_w1);
#pragma unroll
            for (int kk = 0; kk < KP / 32; ++kk) {
                const bf16x8_t a = *reinterpret_cast<const bf16x8_t *>(fh + (row0 + lrow) * S::FH_LD + kk * 32 + lk * 8);
#pragma unroll
                for (int c = 0; c < HID / 16; ++c) {
                    const bf16x8_t b = *reinterpret_cast<const bf16x8_t *>(w1 + (c * 16 + lrow) * S::W1_LD + kk * 32 + lk * 8);
                    acc[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc[c], 0, 0, 0);
                }
            }
        }
        __syncthreads();   // all waves done reading f_h and W1 before h and W2 overwrite them
#pragma unroll
        for (int q = 0; q < N2; ++q) {
            const int i = tid + q * kThreads;
            if (i < 16 * NT * HID) {
                const int r = i / HID, c = i - r * HID;
                if constexpr (BF16) s_w2[r * S::W2_LD + c] = f32_to_bf16_rne(v2[q]);
                else s_w2[r * S::W2_LD + c] = v2[q];
            }
        }
        // bias + ReLU; lane holds rows row0 + 4*lk + i of column c*16 + lrow
#pragma unroll
        for (int c = 0; c < HID / 16; ++c) {
            const int col = c * 16 + lrow;
            const float bias = s_b1[col];
#pragma unroll
            for (int i = 0; i < 4; ++i) {
                const float h = fmaxf(acc[c][i] + bias, 0.0f);
                const int row = row0 + 4 * lk + i;
                if constexpr (BF16) reinterpret_cast<uint16_t *>(s_act)[row * S::H_LD + col] = f32_to_bf16_rne(h);
                else reinterpret_cast<float *>(s_act)[row * S::H_LD + col] = h;
            }
        }
    }
    __syncthreads();

    // ---- C. heads: delta[64 x 16 NT] = h W2^T + b2
    float4_t acc2[NT];
#pragma unroll
    for (int c = 0; c < NT; ++c) acc2[c] = float4_t{0.0f, 0.0f, 0.0f, 0.0f};
    if constexpr (!BF16) {
        const float *hs = reinterpret_cast<const float *>(s_act);
        const float *w2 = reinterpret_cast<const float *>(s_w2);
#pragma unroll 4
        for (int kk = 0; kk < HID / 4; ++kk) {
            const float a = hs[(row0 + lrow) * S::H_LD + kk * 4 + lk];
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                const float b = w2[(c * 16 + lrow) * S::W2_LD + kk * 4 + lk];
                acc2[c] = __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, acc2[c], 0, 0, 0);
            }
        }
    } else {
        const uint16_t *hs = reinterpret_cast<const uint16_t *>(s_act);
        const uint16_t *w2 = reinterpret_cast<const uint16_t *>(s_w2);
#pragma unroll
        for (int kk = 0; kk < HID / 32; ++kk) {
            const bf16x8_t a = *reinterpret_cast<const bf16x8_t *>(hs + (row0 + lrow) * S::H_LD + kk * 32 + lk * 8);
#pragma unroll
            for (int c = 0; c < NT; ++c) {
                const bf16x8_t b =
                    *reinterpret_cast<const bf16x8_t *>(w2 + (c * 16 + lrow) * S::W2_LD + kk * 32 + lk * 8);
                acc2[c] = __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, acc2[c], 0, 0, 0);
            }
        }
    }
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
        for (int i = 0; i < 4; ++i)
            s_delta[(row0 + 4 * lk + i) * S::DS + c * 16 + lrow] = acc2[c][i] + s_b2[c * 16 + lrow];
    __syncthreads();

    // ---- D. Eq. 8 + activations: wave 0 the means and opacity, wave 1 the
    // rotation, wave 2 the scales (inputs were loaded at the start)
    if (dg < n) {
        const float *d = s_delta + lane_g * S::DS;
        const size_t os = (size_t)job.out_stride, oi = (size_t)job.out_offset + dg;
        if (wave_d == 0) {
            float x[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) x[k] = pin[k] + d[k];
            if (job.placed) {
                // rotation matrix of the unit quaternion (w, x, y, z), row-major
                const float qw = job.place_q[0], qx = job.place_q[1], qy = job.place_q[2], qz = job.place_q[3];
                const float R[9] = {1.0f - 2.0f * (qy * qy + qz * qz), 2.0f * (qx * qy - qw * qz),
                                    2.0f * (qx * qz + qw * qy),        2.0f * (qx * qy + qw * qz),
                                    1.0f - 2.0f * (qx * qx + qz * qz), 2.0f * (qy * qz - qw * qx),
                                    2.0f * (qx * qz - qw * qy),        2.0f * (qy * qz + qw * qx),
                                    1.0f - 2.0f * (qx * qx + qy * qy)};
                float y[3];
#pragma unroll
                for (int k = 0; k < 3; ++k)
                    y[k] = job.place_s * (R[3 * k] * x[0] + R[3 * k + 1] * x[1] + R[3 * k + 2] * x[2]) +
                           job.place_t[k];
#pragma unroll
                for (int k = 0; k < 3; ++k) x[k] = y[k];
            }
#pragma unroll
            for (int k = 0; k < 3; ++k) job.out_means[k * os + oi] = x[k];
            const float logit = job.wa ? pin[3] + d[10 + job.n_sh_head] : pin[3];
            job.out_opac[oi] = 1.0f / (1.0f + expf(-logit));
        } else if (wave_d == 1) {
            float q[4];
            float qn = 0.0f;
#pragma unroll
            for (int k = 0; k < 4; ++k) {
                q[k] = pin[k] + d[3 + k];
                qn += q[k] * q[k];
            }
            if (qn > 0.0f) {
                const float inv = 1.0f / sqrtf(qn);
#pragma unroll
                for (int k = 0; k < 4; ++k) q[k] *= inv;
            } else {
                q[0] = 1.0f;
                q[1] = q[2] = q[3] = 0.0f;
            }
            if (job.placed) {
                // Hamilton product place_q (x) q: rotation matrix R(place_q) R(q)
                const float *a = job.place_q;
                const float w = a[0] * q[0] - a[1] * q[1] - a[2] * q[2] - a[3] * q[3];
                const float xq = a[0] * q[1] + a[1] * q[0] + a[2] * q[3] - a[3] * q[2];
                const float yq = a[0] * q[2] - a[1] * q[3] + a[2] * q[0] + a[3] * q[1];
                const float zq = a[0] * q[3] + a[1] * q[2] - a[2] * q[1] + a[3] * q[0];
                q[0] = w; q[1] = xq; q[2] = yq; q[3] = zq;
            }
#pragma unroll
            for (int k = 0; k < 4; ++k) job.out_quats[k * os + oi] = q[k];
        } else if (wave_d == 2) {
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                const float sc = expf(pin[k] + d[7 + k]);
                job.out_scales[k * os + oi] = job.placed ? job.place_s * sc : sc;
            }
        }
    }
    // ---- E. SH coefficients, when written (colour head, composition): all
    // threads, element (row, Gaussian) = (i / 64, i % 64) for a coalesced row
    // run per wave; every load is issued before the first store
    if (job.n_sh_out > 0) {
        constexpr int kShPer = 48 * kGB / kThreads;
        float shv[kShPer];
#pragma unroll
        for (int q = 0; q < kShPer; ++q) {
            const int i = tid + q * kThreads, r = i / kGB, g = g0 + i % kGB;
            shv[q] = (r < job.n_sh_in && g < n) ? job.sh_in[(size_t)r * n + g] : 0.0f;
        }
#pragma unroll
        for (int q = 0; q < kShPer; ++q) {
            const int i = tid + q * kThreads, r = i / kGB, gl = i % kGB, g = g0 + gl;
            if (r < job.n_sh_out && g < n) {
                const float dc = r < job.n_sh_head ? s_delta[gl * S::DS + 10 + r] : 0.0f;
                job.out_sh[(size_t)r * job.out_stride + job.out_offset + g] = shv[q] + dc;
            }
        }
    }
}

template <int F, int L, int HID, bool BF16>
__global__ __launch_bounds__(kThreads)
__attribute__((amdgpu_waves_per_eu(Smem<F, L, HID, BF16, 1>::WAVES))) void k_deform(DeformBatch batch) {
    deform_block<F, L, HID, BF16, 1>(batch);
}

// with the colour and opacity heads: held to three waves per SIMD (the LDS
// of the four head tiles allows three blocks per CU)
template <int F, int L, int HID>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(3))) void k_deform_heads(DeformBatch batch) {
    deform_block<F, L, HID, false, 4>(batch);
}

using DeformKernel = void (*)(DeformBatch);

struct KernelEntry {
    int feat, scales, hidden, bf16, nt;
    DeformKernel fn;
    size_t smem;
};

#define G4D_DEFORM_ENTRY(F, L, H, B) {F, L, H, B, 1, k_deform<F, L, H, (bool)B>, Smem<F, L, H, (bool)B, 1>::total}
#define G4D_DEFORM_ENTRY_CO(F, L, H) {F, L, H, 0, 4, k_deform_heads<F, L, H>, Smem<F, L, H, false, 4>::total}

const KernelEntry kDeformKernels[] = {
    G4D_DEFORM_ENTRY(16, 1, 32, 0), G4D_DEFORM_ENTRY(16, 1, 64, 0), G4D_DEFORM_ENTRY(16, 1, 128, 0),
    G4D_DEFORM_ENTRY(16, 2, 64, 0), G4D_DEFORM_ENTRY(16, 3, 64, 0),
    G4D_DEFORM_ENTRY(32, 1, 64, 0), G4D_DEFORM_ENTRY(32, 2, 64, 0), G4D_DEFORM_ENTRY(32, 2, 128, 0),
    G4D_DEFORM_ENTRY(32, 3, 64, 0), G4D_DEFORM_ENTRY(32, 3, 128, 0),
    G4D_DEFORM_ENTRY(16, 1, 32, 1), G4D_DEFORM_ENTRY(16, 1, 64, 1), G4D_DEFORM_ENTRY(16, 1, 128, 1),
    G4D_DEFORM_ENTRY(16, 2, 64, 1), G4D_DEFORM_ENTRY(16, 3, 64, 1),
    G4D_DEFORM_ENTRY(32, 1, 64, 1), G4D_DEFORM_ENTRY(32, 2, 64, 1), G4D_DEFORM_ENTRY(32, 2, 128, 1),
    G4D_DEFORM_ENTRY(32, 3, 64, 1), G4D_DEFORM_ENTRY(32, 3, 128, 1),
    // with the colour and opacity heads (FP32 decoder)
    G4D_DEFORM_ENTRY_CO(16, 1, 32), G4D_DEFORM_ENTRY_CO(16, 1, 64), G4D_DEFORM_ENTRY_CO(16, 1, 128),
    G4D_DEFORM_ENTRY_CO(16, 2, 64), G4D_DEFORM_ENTRY_CO(16, 3, 64),
    G4D_DEFORM_ENTRY_CO(32, 1, 64), G4D_DEFORM_ENTRY_CO(32, 2, 64), G4D_DEFORM_ENTRY_CO(32, 2, 128),
    G4D_DEFORM_ENTRY_CO(32, 3, 64), G4D_DEFORM_ENTRY_CO(32, 3, 128),
};

const KernelEntry *find_kernel(int feat, int scales, int hidden, int bf16, int nt = 1) {
    for (const auto &e : kDeformKernels)
        if (e.feat == feat && e.scales == scales && e.hidden == hidden && e.bf16 == bf16 && e.nt == nt) return &e;
    return nullptr;
}

bool planes_ok(const g4d_planes *P) {
    if (!P || P->n_scales < 1 || P->n_scales > kMaxScales || (P->feat != 16 && P->feat != 32)) return false;
    for (int k = 0; k < 3; ++k)
        if (!(P->bmax[k] > P->bmin[k])) return false;
    for (int l = 0; l < P->n_scales; ++l) {
        for (int k = 0; k < 4; ++k)
            if (P->res[l][k] < 2 || P->res[l][k] > 65536) return false;
        for (int p = 0; p < 6; ++p)
            if (!P->plane[l][p] || (reinterpret_cast<uintptr_t>(P->plane[l][p]) & 15)) return false;
    }
    return true;
}

g4d_status fill_job(const g4d_gaussians *G, const g4d_planes *P, const g4d_mlp *M, float t,
                    g4d_splats *out, float *features, DeformJob *J) {
    if (!G || !P || G->n < 0 || !planes_ok(P)) return G4D_EINVAL;
    if (!(t >= 0.0f && t <= 1.0f)) return G4D_EINVAL;
    if (G->n > 0 && (!G->means || !G->log_scales || !G->quats || !G->opacity_logits)) return G4D_EINVAL;
    *J = DeformJob{};
    J->means = G->means; J->log_scales = G->log_scales; J->quats = G->quats;
    J->opac = G->opacity_logits;
    for (int l = 0; l < P->n_scales; ++l) {
        for (int p = 0; p < 6; ++p) J->planes[l * 6 + p] = P->plane[l][p];
        for (int k = 0; k < 4; ++k) J->res[l][k] = P->res[l][k];
        for (int k = 0; k < 3; ++k)
            J->gscale[l][k] = (float)((double)(P->res[l][k] - 1) / ((double)P->bmax[k] - (double)P->bmin[k]));
        J->gscale[l][3] = (float)(P->res[l][3] - 1);
    }
    for (int k = 0; k < 3; ++k) J->bmin[k] = P->bmin[k];
    J->n = G->n;
    J->t = t;
    J->out_features = features;
    if (!features) {
        if (!M || !out || out->n != G->n) return G4D_EINVAL;
        if (M->in_dim != P->feat * P->n_scales) return G4D_EINVAL;
        if (G->n > 0 && (!out->means || !out->scales || !out->quats || !out->opacity)) return G4D_EINVAL;
        if (!M->w1 || !M->b1 || !M->wx || !M->bx || !M->wr || !M->br || !M->ws || !M->bs) return G4D_EINVAL;
        J->w1 = M->w1; J->b1 = M->b1; J->wx = M->wx; J->bx = M->bx;
        J->wr = M->wr; J->br = M->br; J->ws = M->ws; J->bs = M->bs;
        J->out_means = out->means; J->out_scales = out->scales;
        J->out_quats = out->quats; J->out_opac = out->opacity;
        // appendix heads: dC over all SH coefficients, dalpha on the opacity logit
        if ((M->wc == nullptr) != (M->bc == nullptr) || (M->wa == nullptr) != (M->ba == nullptr)) return G4D_EINVAL;
        J->out_stride = G->n;
        if (M->wc) {
            if (G->sh_degree < 0 || G->sh_degree > 3 || out->sh_degree != G->sh_degree) return G4D_EINVAL;
            if (G->n > 0 && (!G->sh || !out->sh || out->sh == G->sh)) return G4D_EINVAL;
            J->wc = M->wc; J->bc = M->bc;
            J->n_sh_head = J->n_sh_in = J->n_sh_out = (int16_t)(3 * (G->sh_degree + 1) * (G->sh_degree + 1));
            J->sh_in = G->sh; J->out_sh = out->sh;
        }
        if (M->wa) { J->wa = M->wa; J->ba = M->ba; }
    }
    return G4D_OK;
}

g4d_status launch(DeformBatch &B, const KernelEntry *ke, hipStream_t s) {
    int blocks = 0;
    for (int j = 0; j < B.n_jobs; ++j) {
        B.job[j].block_begin = blocks;
        blocks += (B.job[j].n + kGB - 1) / kGB;
    }
    if (blocks == 0) return G4D_OK;
    B.n_blocks = blocks;
    static std::atomic<uint64_t> attr_done[sizeof(kDeformKernels) / sizeof(kDeformKernels[0])];
    const size_t idx = (size_t)(ke - kDeformKernels);
    if (g4d_status st = ensure_max_lds(reinterpret_cast<const void *>(ke->fn), attr_done[idx], (int)ke->smem))
        return st;
    hipLaunchKernelGGL(ke->fn, dim3(8 * ((blocks + 7) / 8)), dim3(kThreads), ke->smem, s, B);
    G4D_HIP_CHECK(hipGetLastError());
    return G4D_OK;
}

}  // namespace

g4d_status deform_batched(const g4d_deform_job *jobs, int n_jobs, hipStream_t s) {
    if (!jobs || n_jobs < 1 || n_jobs > G4D_MAX_BATCH_JOBS) return G4D_EINVAL;
    DeformBatch B{};
    B.n_jobs = n_jobs;
    const KernelEntry *ke = nullptr;
    for (int j = 0; j < n_jobs; ++j) {
        const g4d_deform_job &q = jobs[j];
        if (!q.M || !q.P) return G4D_EINVAL;
        g4d_status st = fill_job(q.G, q.P, q.M, q.t, q.out, nullptr, &B.job[j]);
        if (st != G4D_OK) return st;
        // head rows dx dr ds [dC] [dalpha]: one 16-row tile, or four
        const int rows = B.job[j].n_sh_head + (q.M->wa ? 11 : 10);
        const int nt = rows <= 16 ? 1 : 4;
        const KernelEntry *e = find_kernel(q.P->feat, q.P->n_scales, q.M->hidden,
                                           q.M->precision == G4D_MLP_BF16 ? 1 : 0, nt);
        if (!e || (q.M->precision != G4D_MLP_F32 && q.M->precision != G4D_MLP_BF16)) return G4D_EUNSUPPORTED;
        if (ke && e != ke) return G4D_EINVAL;   // one shape class per launch
        ke = e;
    }
    return launch(B, ke, s);
}

g4d_status deform_features(const g4d_gaussians *G, const g4d_planes *P, float t, float *features,
                           hipStream_t s) {
    if (!features && G && G->n > 0) return G4D_EINVAL;
    DeformBatch B{};
    B.n_jobs = 1;
    g4d_status st = fill_job(G, P, nullptr, t, nullptr, features, &B.job[0]);
    if (st != G4D_OK) return st;
    const KernelEntry *e = find_kernel(P->feat, P->n_scales, 64, 0);
    if (!e) return G4D_EUNSUPPORTED;
    return launch(B, e, s);
}

// Sec. 5.4 composition: every item's deformed set, placed, into its index
// range of one render-ready set.  All items are validated before the first
// launch; consecutive items of one kernel variant share a launch.
g4d_status deform_compose(const g4d_compose_item *items, int n_items, g4d_splats *out, hipStream_t s) {
    if (!items || !out || n_items < 1 || n_items > G4D_MAX_COMPOSE_ITEMS) return G4D_EINVAL;
    if (out->n < 0 || out->sh_degree < 0 || out->sh_degree > 3) return G4D_EINVAL;
    int64_t total = 0;
    for (int i = 0; i < n_items; ++i) {
        const g4d_gaussians *G = items[i].G;
        if (!G || G->n < 0 || G->sh_degree < 0 || G->sh_degree > out->sh_degree) return G4D_EINVAL;
        if (G->n > 0 && (!G->sh || G->sh == out->sh)) return G4D_EINVAL;
        total += G->n;
    }
    if (total != out->n || total > (int64_t(1) << 26)) return G4D_EINVAL;
    if (total > 0 && (!out->means || !out->scales || !out->quats || !out->opacity || !out->sh))
        return G4D_EINVAL;
    const int rows_out = 3 * (out->sh_degree + 1) * (out->sh_degree + 1);
    std::vector<DeformJob> jobs((size_t)n_items);
    std::vector<const KernelEntry *> kern((size_t)n_items);
    int64_t offset = 0;
    for (int i = 0; i < n_items; ++i) {
        const g4d_compose_item &it = items[i];
        const g4d_gaussians *G = it.G;
        if (!it.P || !it.M) return G4D_EINVAL;
        // the item's own view of the output: its sizes, the combined arrays
        g4d_splats sub = *out;
        sub.n = G->n;
        sub.sh_degree = G->sh_degree;
        DeformJob &J = jobs[(size_t)i];
        g4d_status st = fill_job(G, it.P, it.M, it.t, &sub, nullptr, &J);
        if (st != G4D_OK) return st;
        J.out_stride = (int)total;
        J.out_offset = (int)offset;
        J.sh_in = G->sh;
        J.out_sh = out->sh;
        J.n_sh_in = (int16_t)(3 * (G->sh_degree + 1) * (G->sh_degree + 1));
        J.n_sh_out = (int16_t)rows_out;
        const g4d_placement &pl = it.place;
        const double qn = std::sqrt((double)pl.rotation[0] * pl.rotation[0] + (double)pl.rotation[1] * pl.rotation[1] +
                                    (double)pl.rotation[2] * pl.rotation[2] + (double)pl.rotation[3] * pl.rotation[3]);
        if (!(qn > 0.0) || !std::isfinite(qn) || !(pl.scale > 0.0f) || !std::isfinite(pl.scale)) return G4D_EINVAL;
        for (int k = 0; k < 3; ++k)
            if (!std::isfinite(pl.translation[k])) return G4D_EINVAL;
        for (int k = 0; k < 4; ++k) J.place_q[k] = (float)(pl.rotation[k] / qn);
        J.place_s = pl.scale;
        for (int k = 0; k < 3; ++k) J.place_t[k] = pl.translation[k];
        J.placed = !(J.place_q[0] == 1.0f && J.place_q[1] == 0.0f && J.place_q[2] == 0.0f && J.place_q[3] == 0.0f &&
                     pl.scale == 1.0f && pl.translation[0] == 0.0f && pl.translation[1] == 0.0f &&
                     pl.translation[2] == 0.0f);
        const int rows = J.n_sh_head + (it.M->wa ? 11 : 10);
        const KernelEntry *e = find_kernel(it.P->feat, it.P->n_scales, it.M->hidden,
                                           it.M->precision == G4D_MLP_BF16 ? 1 : 0, rows <= 16 ? 1 : 4);
        if (!e || (it.M->precision != G4D_MLP_F32 && it.M->precision != G4D_MLP_BF16)) return G4D_EUNSUPPORTED;
        kern[(size_t)i] = e;
        offset += G->n;
    }
    DeformBatch B{};
    const KernelEntry *ke = nullptr;
    for (int i = 0; i <= n_items; ++i) {
        const bool flush = B.n_jobs > 0 && (i == n_items || kern[(size_t)i] != ke || B.n_jobs == G4D_MAX_BATCH_JOBS);
        if (flush) {
            g4d_status st = launch(B, ke, s);
            if (st != G4D_OK) return st;
            B = DeformBatch{};
        }
        if (i == n_items) break;
        B.job[B.n_jobs++] = jobs[(size_t)i];
        ke = kern[(size_t)i];
    }
    return G4D_OK;
}

}  // namespace g4d

extern "C" g4d_status g4d_deform_compose(const g4d_compose_item *items, int32_t n_items, g4d_splats *out,
                                         void *stream) {
    return g4d::deform_compose(items, n_items, out, reinterpret_cast<hipStream_t>(stream));
}

extern "C" g4d_status g4d_deform(const g4d_gaussians *G, const g4d_planes *P, const g4d_mlp *M,
                                 float t, g4d_splats *out, void *stream) {
    g4d_deform_job j{G, P, M, t, out};
    return g4d::deform_batched(&j, 1, reinterpret_cast<hipStream_t>(stream));
}

extern "C" g4d_status g4d_deform_batched(const g4d_deform_job *jobs, int32_t n_jobs, void *stream) {
    return g4d::deform_batched(jobs, n_jobs, reinterpret_cast<hipStream_t>(stream));
}

extern "C" g4d_status g4d_deform_features(const g4d_gaussians *G, const g4d_planes *P, float t,
                                          float *features, void *stream) {
    return g4d::deform_features(G, P, t, features, reinterpret_cast<hipStream_t>(stream));
}
