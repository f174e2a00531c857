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
// W1 is read from global memory (L1/L2-resident: every block reads it); the
// head weights, their biases and the per-row gradient pointers are staged in
// LDS once per block (the heads are selected by a runtime row index, which
// in the inner loops would be a dependent kernel-argument load per step);
// f_h, h, the deltas and dz live in LDS.
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
    constexpr int FH = K + 1, HH = HID + 1, DS = 65;
    extern __shared__ __attribute__((aligned(16))) float smem[];
    float *s_fh = smem;                  // [GB][K+1]: f_h, later df_h
    float *s_dm = s_fh + GB * FH;       // [GB][3]: dL/d canonical mean
    float *s_h = s_dm + GB * 3;         // [GB][HID+1]: h (after ReLU)
    float *s_dz = s_h + GB * HH;        // [GB][HID+1]: dL/d(pre-activation)
    float *s_dd = s_dz + GB * HH;       // [GB][65]: head outputs, then their gradients
    float *s_w2 = s_dd + GB * DS;       // [rows][HID+1]: head weights
    float *s_b2 = s_w2 + rows * HH;      // [rows]
    // the plane-cell windows of the encoder backward reuse everything from
    // s_h on (dead once df_h is computed)
    float *s_win = s_h;
    const int win_cap = 2 * GB * HH + GB * DS + rows * HH + rows;
    __shared__ float *s_dw[64];          // gradient row of head row r (null: padding)
    __shared__ float *s_db[64];
    const int tid = threadIdx.x;
    const int g0 = blockIdx.x * GB;
    const int n = J.n;
    if (tid < rows) {
        int hq, k;
        if (head_of(J, tid, hq, k)) {
            s_dw[tid] = J.d_hw[hq] + (size_t)k * HID;
            s_db[tid] = J.d_hb[hq] + k;
            s_b2[tid] = J.hb[hq][k];
        } else {
            s_dw[tid] = nullptr;
            s_db[tid] = nullptr;
            s_b2[tid] = 0.0f;
        }
    }
    for (int idx = tid; idx < rows * HID; idx += kThreads) {
        const int r = idx / HID, j = idx - r * HID;
        int hq, k;
        s_w2[r * HH + j] = head_of(J, r, hq, k) ? J.hw[hq][(size_t)k * HID + j] : 0.0f;
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
    // ---- B. h = ReLU(W1 f_h + b1).  With 64 Gaussians per block a wave owns
    // whole rows of W1 (lane = Gaussian), so a row is wave-uniform and its
    // weights come through scalar loads; with fewer, Gaussian fastest (a
    // weight is one broadcast vector load)
    const int wave_u = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
    if constexpr (GB == 64) {
        for (int j = wave_u; j < HID; j += kThreads / 64) {
            const float *w = J.w1 + (size_t)j * K;
            float acc = J.b1[j];
            for (int i = 0; i < K; ++i) acc += w[i] * s_fh[lane * FH + i];
            s_h[lane * HH + j] = fmaxf(acc, 0.0f);
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
    __syncthreads();
    // ---- C. head outputs delta = W2 h + b2 (padding rows: zero weights)
    for (int idx = tid; idx < GB * rows; idx += kThreads) {
        const int g = idx % GB, r = idx / GB;
        float acc = s_b2[r];
        const float *w = s_w2 + r * HH;
        for (int j = 0; j < HID; ++j) acc += w[j] * s_h[g * HH + j];
        s_dd[g * DS + r] = acc;
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
            for (int r = 10 + nc + J.hrows[4]; r < rows; ++r) dd[r] = 0.0f;
        } else {
            for (int r = 0; r < rows; ++r) dd[r] = 0.0f;
            for (int k = 0; k < 3; ++k) s_dm[gl * 3 + k] = 0.0f;
        }
    } else if (J.d_sh) {
        for (int idx = tid - GB; idx < GB * J.n_sh_rows; idx += kThreads - GB) {
            const int gl = idx % GB, r = idx / GB, g = g0 + gl;
            if (g < n) J.d_sh[(size_t)r * n + g] = J.g_sh[(size_t)r * n + g];
        }
    }
    __syncthreads();
    // ---- heads backward: dz = (W2^T ddelta) * [h > 0]
    for (int idx = tid; idx < GB * HID; idx += kThreads) {
        const int g = idx % GB, j = idx / GB;
        float acc = 0.0f;
        for (int r = 0; r < rows; ++r) acc += s_w2[r * HH + j] * s_dd[g * DS + r];
        s_dz[g * HH + j] = s_h[g * HH + j] > 0.0f ? acc : 0.0f;
    }
    // dW2 += ddelta h^T, db2 += ddelta (sums over the block's Gaussians)
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
    __syncthreads();
    // ---- feature merger: dW1 += dz f_h^T, db1 += dz
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
    __syncthreads();
    // df_h = W1^T dz (overwrites f_h); column i of W1 wave-uniform as above
    if constexpr (GB == 64) {
        for (int i = wave_u; i < K; i += kThreads / 64) {
            float acc = 0.0f;
            for (int j = 0; j < HID; ++j) acc += J.w1[(size_t)j * K + i] * s_dz[lane * HH + j];
            s_fh[lane * FH + i] = acc;
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
    // spans that range plus one (the upper corners)
    __shared__ int s_lo[kMaxScalesB * 3], s_hi[kMaxScalesB * 3];
    __shared__ int s_woff[kMaxScalesB * 6], s_wa0[kMaxScalesB * 6], s_wb0[kMaxScalesB * 6];
    __shared__ int s_wn[kMaxScalesB * 6], s_wm[kMaxScalesB * 6];
    __shared__ int s_wtotal;
    if (tid < 3 * L) {
        s_lo[tid] = 0x7fffffff;
        s_hi[tid] = -1;
    }
    __syncthreads();
    if (tid < GB && g0 + tid < n) {
        const int g = g0 + tid;
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            const float xk = J.means[(size_t)k * n + g] - J.bmin[k];
#pragma unroll
            for (int l = 0; l < L; ++l) {
                int i0;
                float w;
                grid_coord(xk, J.gscale[l][k], J.res[l][k], i0, w);
                atomicMin(&s_lo[l * 3 + k], i0);
                atomicMax(&s_hi[l * 3 + k], i0);
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
                const int need = wn * wm * F;
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
    // ---- encoder backward (Eq. 7)
#pragma unroll
    for (int pass = 0; pass < NPASS; ++pass) {
        const int gl = pass * GPP + tid / LPG, c4 = tid % LPG, g = g0 + gl;
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
                        const int wrow = s_wn[q] * F;
                        float *lb = s_win + wo + ((ib_[p] - s_wb0[q]) * s_wn[q] + (ia_[p] - s_wa0[q])) * F + 4 * c4;
#pragma unroll
                        for (int c = 0; c < 4; ++c) {
                            if (dvv[c] == 0.0f) continue;
                            if (w00 != 0.0f) atomicAdd(lb + c, w00 * dvv[c]);
                            if (w10 != 0.0f) atomicAdd(lb + F + c, w10 * dvv[c]);
                            if (w01 != 0.0f) atomicAdd(lb + wrow + c, w01 * dvv[c]);
                            if (w11 != 0.0f) atomicAdd(lb + wrow + F + c, w11 * dvv[c]);
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
            const float v = s_win[wo + i];
            if (v == 0.0f) continue;
            const int cell = i / F, f = i - cell * F;
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

size_t bwd_smem(int gb, int K, int HID, int rows) {
    return ((size_t)gb * (K + 1) + 2 * (size_t)gb * (HID + 1) + (size_t)gb * 65 + (size_t)gb * 3 +
            (size_t)rows * (HID + 1) + rows) * 4;
}

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
