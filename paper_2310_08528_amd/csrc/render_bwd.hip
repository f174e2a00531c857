// Backward of the splat render on gfx950 (Sec. 3.1, Eq. 1-4; Eq. 2-3).
//
//   k_blend_bwd       one 256-thread block per tile, one wave per 8x8
//                     quadrant as in the forward.  Each pixel starts from its
//                     final transmittance and the list position of its last
//                     contributing Gaussian (both written by the forward), and
//                     walks its tile's list back to front, recomputing alpha
//                     with the forward's exact binary32 expressions (so the
//                     skip decisions are the forward's) and undoing the
//                     transmittance, T_i = T_(i+1) / (1 - alpha_i).  No
//                     per-pixel lists are stored.  A wave takes 64 entries at
//                     a time, keeps those that can reach its quadrant (the
//                     forward's conservative cull), and for each kept entry
//                     sums the 64 pixels' contributions across the wave.  The
//                     four waves walk the same 64-entry chunks: their sums
//                     meet in an LDS accumulator (LDS atomics), and the block
//                     then adds each entry's 2D gradient (u, v, conic, colour,
//                     opacity) to the Gaussian with one global atomic per
//                     component, spread over all 256 threads.  The wave sums
//                     are DPP butterflies inside each 16-lane row, whose four
//                     row sums go to the accumulator by LDS atomics (lane
//                     shuffles through the LDS crossbar cost twice as much,
//                     and readlanes across the rows about as much again).
//   k_preprocess_bwd  per Gaussian: the 2D gradient back through the conic
//                     inverse, Sigma' = J W Sigma W^T J^T (with J's
//                     dependence on the camera-space mean and the frustum
//                     clamp), Sigma = R S S^T R^T, the projection and the SH
//                     colour (coefficients and view direction).
//
// Derivatives of the compositing sum C = sum_i c_i alpha_i T_i + T_N bg:
//   dC/dc_i     = alpha_i T_i
//   dC/dalpha_i = T_i (c_i - S_i) - T_N bg / (1 - alpha_i),
// S_i the colour composited behind entry i (S <- alpha c + (1 - alpha) S
// walking back).  alpha = min(0.99, o exp(power)): a clamped alpha passes no
// gradient to o or power.
#include "g4d_internal.h"

namespace g4d {
namespace {

struct BwdCam {
    float v[12];
    float fx, fy, cx, cy, limx, limy;
    float campos[3];
    float bg[3];
};

__device__ __forceinline__ uint64_t lanemask_lt() {
    const uint32_t lo = __builtin_amdgcn_mbcnt_lo(0xffffffffu, 0u);
    const uint32_t l = __builtin_amdgcn_mbcnt_hi(0xffffffffu, lo);
    return (l == 0) ? 0ull : (~0ull >> (64 - l));
}

__device__ __forceinline__ float quad_form(float A, float B, float C, float dx, float dy) {
    return (A * dx) * dx + (2.0f * B * dx) * dy + (C * dy) * dy;
}

// The forward's per-quadrant cull: can the Gaussian reach alpha >= 1/255
// anywhere in [x_lo, x_hi] x [y_lo, y_hi]?  Conservative (see the forward).
__device__ __forceinline__ bool may_reach(float u, float v, float A, float B, float C, float iA, float iC,
                                          float thr, float x_lo, float x_hi, float y_lo, float y_hi) {
    if (x_hi < x_lo || y_hi < y_lo) return false;
    const float dxl = u - x_hi, dxh = u - x_lo;
    const float dyl = v - y_hi, dyh = v - y_lo;
    if (dxl <= 0.0f && dxh >= 0.0f && dyl <= 0.0f && dyh >= 0.0f) return true;
    const float ea = fminf(fmaxf(-(B * dxl) * iC, dyl), dyh);
    const float eb = fminf(fmaxf(-(B * dxh) * iC, dyl), dyh);
    const float ec = fminf(fmaxf(-(B * dyl) * iA, dxl), dxh);
    const float ed = fminf(fmaxf(-(B * dyh) * iA, dxl), dxh);
    const float qmin = fminf(fminf(quad_form(A, B, C, dxl, ea), quad_form(A, B, C, dxh, eb)),
                             fminf(quad_form(A, B, C, ec, dyl), quad_form(A, B, C, ed, dyh)));
    const float d2 = fmaxf(dxl * dxl, dxh * dxh) + fmaxf(dyl * dyl, dyh * dyh);
    return !(qmin > thr + 1e-3f * (1.0f + fabsf(thr)) + 2e-6f * (A + C) * d2);
}

__global__ void k_fill_zero(float *__restrict__ p, size_t n) {
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
        p[i] = 0.0f;
}

constexpr int kG2 = 9;   // 2D gradient components per Gaussian
constexpr int kBlendBwdWideN = 16384;   // up to this many Gaussians: eight entries per group

// Sum over the 64 lanes of a wave (every lane active): butterflies inside
// each row of 16 lanes with DPP (quad permutes, half-row and row mirrors,
// all on the VALU), then the four row sums read into scalars.
template <int CTRL>
__device__ __forceinline__ float dpp(float v) {
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
// Sum over each row of 16 lanes; every lane of the row receives it.  The
// adds stay adds (no contraction with a product that feeds them, which would
// split each DPP add into a move and an FMA).
__device__ __forceinline__ float row_sum(float v) {
#pragma clang fp contract(off)
    v += dpp<0xb1>(v);    // quad_perm [1, 0, 3, 2]: lane ^ 1
    v += dpp<0x4e>(v);    // quad_perm [2, 3, 0, 1]: lane ^ 2
    v += dpp<0x141>(v);   // row_half_mirror: the other quad of the half-row
    v += dpp<0x140>(v);   // row_mirror: the other half of the row
    return v;
}

template <int GRP>
__global__ __launch_bounds__(256) void k_blend_bwd(const uint4 *__restrict__ order, const uint32_t *__restrict__ gids,
                                                   uint32_t gmask, const float4 *__restrict__ recA,
                                                   const float4 *__restrict__ recB, const float4 *__restrict__ recC,
                                                   int width, int height, int tiles_x, int n_tiles, BwdCam cam,
                                                   const float *__restrict__ final_T,
                                                   const int32_t *__restrict__ n_contrib,
                                                   const float *__restrict__ grad_image, float *__restrict__ g2d,
                                                   int n) {
    constexpr int NW = 4;
    __shared__ float4 sR[NW][64 * 3];
    __shared__ uint32_t sSlot[NW][64];     // chunk index of each packed entry
    __shared__ float sAcc[64 * kG2];       // the chunk's entries: the four quadrants' sums
    __shared__ uint32_t sGid[64];
    __shared__ int sMax[NW];
    const int b = (int)blockIdx.x;
    if (b >= n_tiles) return;
    const uint4 ord = order[b];
    const int tile = (int)ord.x;
    const int tx = tile % tiles_x, ty = tile / tiles_x;
    const int tid = threadIdx.x, wave = tid >> 6, lane = tid & 63;
    const int qx0 = tx * kTile + (wave & 1) * 8, qy0 = ty * kTile + (wave >> 1) * 8;
    const int px = qx0 + (lane & 7), py = qy0 + (lane >> 3);
    const bool inside = px < width && py < height;
    const size_t plane = (size_t)width * height;
    const size_t pix = inside ? (size_t)py * width + px : 0;
    const int start = (int)ord.y;
    const float fpx = (float)px, fpy = (float)py;
    const float x_lo = (float)qx0, y_lo = (float)qy0;
    const float x_hi = fminf(x_lo + 7.0f, (float)(width - 1));
    const float y_hi = fminf(y_lo + 7.0f, (float)(height - 1));
    float T = inside ? final_T[pix] : 1.0f;
    const int last = inside ? n_contrib[pix] : 0;
    const float g0 = inside ? grad_image[pix] : 0.0f;
    const float g1 = inside ? grad_image[plane + pix] : 0.0f;
    const float g2 = inside ? grad_image[2 * plane + pix] : 0.0f;
    const float tnbg = T * ((cam.bg[0] * g0 + cam.bg[1] * g1) + cam.bg[2] * g2);
    float S0 = 0.0f, S1 = 0.0f, S2 = 0.0f;
    // the tile's highest contributing position (all waves walk the same chunks)
    int pmax = last;
#pragma unroll
    for (int o = 32; o >= 1; o >>= 1) pmax = max(pmax, __shfl_xor(pmax, o, 64));
    if (lane == 0) sMax[wave] = pmax;
    for (int i = tid; i < 64 * kG2; i += 256) sAcc[i] = 0.0f;
    __syncthreads();
    pmax = max(max(sMax[0], sMax[1]), max(sMax[2], sMax[3]));
    const float a_min = 1.0f / 255.0f;
    const uint64_t lt = lanemask_lt();
    float4 *__restrict__ R = sR[wave];
    uint32_t *__restrict__ Sl = sSlot[wave];
    for (int hi = pmax; hi >= 1; hi -= 64) {
        // every wave loads the chunk's 64 entries (lane 0: the highest position)
        // and keeps those that can reach its quadrant
        const int pos1 = hi - lane;
        bool keep = false;
        float4 A4 = make_float4(0.f, 0.f, 0.f, 0.f), B4 = A4;
        float C1 = 0.0f;
        uint32_t gid = 0;
        if (pos1 >= 1) {
            gid = gids[start + pos1 - 1] & gmask;
            if (gid >= (uint32_t)n) gid = 0;
            A4 = recA[gid];
            B4 = recB[gid];
            C1 = recC[gid].x;
            const float A = -2.0f * A4.z, C = -2.0f * A4.w, Bc = -B4.x;
            const float iA = __builtin_amdgcn_rcpf(A), iC = __builtin_amdgcn_rcpf(C);
            const float thr = 2.0f * (__logf(B4.y) + 5.541263545158426f);
            keep = may_reach(A4.x, A4.y, A, Bc, C, iA, iC, thr, x_lo, x_hi, y_lo, y_hi);
        }
        if (wave == 0) sGid[lane] = gid;
        const uint64_t km = __builtin_amdgcn_ballot_w64(keep);
        if (keep) {
            const int slot = (int)__popcll(km & lt);
            R[3 * slot] = A4;
            R[3 * slot + 1] = make_float4(B4.x, __log2f(B4.y), B4.z, B4.w);
            // 1/o by the hardware reciprocal and one Newton step (o in (0, 1))
            float io = __builtin_amdgcn_rcpf(B4.y);
            io = __builtin_fmaf(__builtin_fmaf(-B4.y, io, 1.0f), io, io);
            R[3 * slot + 2] = make_float4(C1, __int_as_float(pos1), io, 0.0f);
            Sl[slot] = (uint32_t)lane;
        }
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        const int cnt = (int)__popcll(km);
        // Entries in groups of GRP, in decreasing list position: the
        // transmittance and colour recursions stay in order, while the
        // entries' gradient terms and row sums are independent work for the
        // scheduler.
        struct Ent {
            float4 R0, R1, R2;
            float dx, dy, raw, alpha;
            bool act;
        };
        auto load_ent = [&](int e) -> Ent {
            Ent q;
            q.R0 = R[3 * e];
            q.R1 = R[3 * e + 1];
            q.R2 = R[3 * e + 2];
            const int pos = __float_as_int(q.R2.y);
            q.dx = q.R0.x - fpx;
            q.dy = q.R0.y - fpy;
            // the forward's expressions, so that the skip decisions are its own
            const float power = __builtin_fmaf(q.dx, __builtin_fmaf(q.R0.z, q.dx, q.R1.x * q.dy), (q.R0.w * q.dy) * q.dy);
            const float pw = power > 0.0f ? -INFINITY : power;
            q.raw = __builtin_amdgcn_exp2f(__builtin_fmaf(pw, 1.44269504f, q.R1.y));
            float alpha = fminf(0.99f, q.raw);
            q.alpha = alpha < a_min ? 0.0f : alpha;
            q.act = inside && pos <= last && q.alpha > 0.0f;
            return q;
        };
        // branch-free body: a lane that does not composite the entry takes
        // alpha = 0, for which 1/(1 - alpha) = 1 exactly and T, S and every
        // gradient term stay unchanged (zero)
        auto grad_of = [&](const Ent &q, float (&v)[kG2]) {
            const float al = q.act ? q.alpha : 0.0f;
            const float om = 1.0f - al;
            // 1/(1 - alpha): hardware reciprocal and one Newton step
            float r = __builtin_amdgcn_rcpf(om);
            r = __builtin_fmaf(__builtin_fmaf(-om, r, 1.0f), r, r);
            const float Ti = T * r;
            const float aT = al * Ti;
            v[5] = aT * g0;
            v[6] = aT * g1;
            v[7] = aT * g2;
            const float cg = (q.R1.z * g0 + q.R1.w * g1) + q.R2.x * g2;
            const float sg = (S0 * g0 + S1 * g1) + S2 * g2;
            const float dal = Ti * (cg - sg) - tnbg * r;
            S0 = al * q.R1.z + om * S0;
            S1 = al * q.R1.w + om * S1;
            S2 = al * q.R2.x + om * S2;
            T = Ti;
            // a clamped alpha passes nothing to o or the power
            const float dpw = q.raw > 0.99f ? 0.0f : dal * al;
            v[8] = dpw * q.R2.z;                                          // dalpha/do = alpha/o
            v[0] = dpw * __builtin_fmaf(2.0f * q.R0.z, q.dx, q.R1.x * q.dy);   // d power / du = -A dx - B dy
            v[1] = dpw * __builtin_fmaf(2.0f * q.R0.w, q.dy, q.R1.x * q.dx);   // d power / dv = -C dy - B dx
            const float hd = -0.5f * dpw, hx = hd * q.dx;
            v[2] = hx * q.dx;                                             // d power / dA
            v[3] = (hx + hx) * q.dy;                                      // d power / dB
            v[4] = (hd * q.dy) * q.dy;                                    // d power / dC
        };
        // lane k of each row adds component k of its row's sum into the chunk
        // accumulator (LDS atomics: the rows and the four quadrants meet there)
        auto add_sums = [&](const float (&v)[kG2], int e) {
            float sum[kG2];
#pragma unroll
            for (int k = 0; k < kG2; ++k) sum[k] = row_sum(v[k]);
            const int rk = lane & 15;
            float mine = sum[0];
#pragma unroll
            for (int k = 1; k < kG2; ++k) mine = rk == k ? sum[k] : mine;
            if (rk < kG2 && mine != 0.0f) atomicAdd(&sAcc[Sl[e] * kG2 + rk], mine);
        };
        constexpr int kGrp = GRP;   // entries per group
        int j = 0;
        for (; j + kGrp <= cnt; j += kGrp) {
            Ent q[kGrp];
            bool u[kGrp];
            bool any = false;
#pragma unroll
            for (int e = 0; e < kGrp; ++e) {
                q[e] = load_ent(j + e);
                // an entry no pixel of the quadrant composites changes nothing
                u[e] = __builtin_amdgcn_ballot_w64(q[e].act) != 0;
                any = any || u[e];
            }
            if (!any) continue;
            float v[kGrp][kG2];
#pragma unroll
            for (int e = 0; e < kGrp; ++e) grad_of(q[e], v[e]);
#pragma unroll
            for (int e = 0; e < kGrp; ++e)
                if (u[e]) add_sums(v[e], j + e);
        }
        for (; j < cnt; ++j) {
            const Ent qa = load_ent(j);
            if (__builtin_amdgcn_ballot_w64(qa.act) != 0) {
                float va[kG2];
                grad_of(qa, va);
                add_sums(va, j);
            }
        }
        __syncthreads();
        // one global atomic per (entry, component) of the tile, all threads
        for (int i = tid; i < 64 * kG2; i += 256) {
            const float val = sAcc[i];
            if (val != 0.0f) {
                const int e = i / kG2, k = i - e * kG2;
                atomicAdd(&g2d[(size_t)k * n + sGid[e]], val);
                sAcc[i] = 0.0f;
            }
        }
        __syncthreads();
    }
}

// Real SH basis (degree <= 3) on a unit direction, and its gradient with
// respect to the direction (of the Cartesian polynomials; the normalisation
// Jacobian removes the radial part).
__device__ __forceinline__ void sh_eval(int deg, float x, float y, float z, float (&Y)[16], float (&Dx)[16],
                                        float (&Dy)[16], float (&Dz)[16]) {
    const float C0 = 0.28209479177387814f, C1 = 0.4886025119029199f;
    const float K1 = 1.0925484305920792f, K2 = 0.31539156525252005f, K3 = 0.5462742152960396f;
    const float a = 0.5900435899266435f, bq = 2.890611442640554f, c = 0.4570457994644658f;
    const float d = 0.3731763325901154f, e = 1.445305721320277f;
#pragma unroll
    for (int k = 0; k < 16; ++k) Y[k] = Dx[k] = Dy[k] = Dz[k] = 0.0f;
    Y[0] = C0;
    if (deg >= 1) {
        Y[1] = -C1 * y; Dy[1] = -C1;
        Y[2] = C1 * z;  Dz[2] = C1;
        Y[3] = -C1 * x; Dx[3] = -C1;
    }
    if (deg >= 2) {
        const float xx = x * x, yy = y * y, zz = z * z;
        Y[4] = K1 * x * y;                 Dx[4] = K1 * y;  Dy[4] = K1 * x;
        Y[5] = -K1 * y * z;                Dy[5] = -K1 * z; Dz[5] = -K1 * y;
        Y[6] = K2 * (2.0f * zz - xx - yy); Dx[6] = -2.0f * K2 * x; Dy[6] = -2.0f * K2 * y; Dz[6] = 4.0f * K2 * z;
        Y[7] = -K1 * x * z;                Dx[7] = -K1 * z; Dz[7] = -K1 * x;
        Y[8] = K3 * (xx - yy);             Dx[8] = 2.0f * K3 * x; Dy[8] = -2.0f * K3 * y;
        if (deg >= 3) {
            Y[9] = -a * y * (3.0f * xx - yy);
            Dx[9] = -6.0f * a * x * y; Dy[9] = -3.0f * a * (xx - yy);
            Y[10] = bq * x * y * z;
            Dx[10] = bq * y * z; Dy[10] = bq * x * z; Dz[10] = bq * x * y;
            Y[11] = -c * y * (4.0f * zz - xx - yy);
            Dx[11] = 2.0f * c * x * y; Dy[11] = -c * (4.0f * zz - xx - 3.0f * yy); Dz[11] = -8.0f * c * y * z;
            Y[12] = d * z * (2.0f * zz - 3.0f * xx - 3.0f * yy);
            Dx[12] = -6.0f * d * x * z; Dy[12] = -6.0f * d * y * z; Dz[12] = d * (6.0f * zz - 3.0f * xx - 3.0f * yy);
            Y[13] = -c * x * (4.0f * zz - xx - yy);
            Dx[13] = -c * (4.0f * zz - 3.0f * xx - yy); Dy[13] = 2.0f * c * x * y; Dz[13] = -8.0f * c * x * z;
            Y[14] = e * z * (xx - yy);
            Dx[14] = 2.0f * e * x * z; Dy[14] = -2.0f * e * y * z; Dz[14] = e * (xx - yy);
            Y[15] = -a * x * (xx - 3.0f * yy);
            Dx[15] = -3.0f * a * (xx - yy); Dy[15] = 6.0f * a * x * y;
        }
    }
}

__global__ __launch_bounds__(256) void k_preprocess_bwd(int n, int sh_degree, const float *__restrict__ means,
                                                        const float *__restrict__ scales,
                                                        const float *__restrict__ quats,
                                                        const float *__restrict__ sh, BwdCam cam,
                                                        const float *__restrict__ g2d, float *__restrict__ d_means,
                                                        float *__restrict__ d_scales, float *__restrict__ d_quats,
                                                        float *__restrict__ d_opac, float *__restrict__ d_sh) {
    const int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    float G[kG2];
    bool any = false;
#pragma unroll
    for (int k = 0; k < kG2; ++k) {
        G[k] = g2d[(size_t)k * n + g];
        any = any || G[k] != 0.0f;
    }
    const int ncoef = (sh_degree + 1) * (sh_degree + 1);
    float dm[3] = {0.f, 0.f, 0.f}, ds[3] = {0.f, 0.f, 0.f}, dq[4] = {0.f, 0.f, 0.f, 0.f};
    if (!any) {
        for (int k = 0; k < 3; ++k) { d_means[(size_t)k * n + g] = 0.0f; d_scales[(size_t)k * n + g] = 0.0f; }
        for (int k = 0; k < 4; ++k) d_quats[(size_t)k * n + g] = 0.0f;
        d_opac[g] = 0.0f;
        for (int k = 0; k < ncoef * 3; ++k) d_sh[(size_t)k * n + g] = 0.0f;
        return;
    }
    const float du = G[0], dv = G[1], dA = G[2], dB = G[3], dC = G[4];
    float dcol[3] = {G[5], G[6], G[7]};
    const float m[3] = {means[g], means[(size_t)n + g], means[2 * (size_t)n + g]};
    const float s[3] = {scales[g], scales[(size_t)n + g], scales[2 * (size_t)n + g]};
    const float qw = quats[g], qx = quats[(size_t)n + g], qy = quats[2 * (size_t)n + g], qz = quats[3 * (size_t)n + g];
    const float *V = cam.v;
    const float px = ((V[0] * m[0] + V[1] * m[1]) + V[2] * m[2]) + V[3];
    const float py = ((V[4] * m[0] + V[5] * m[1]) + V[6] * m[2]) + V[7];
    const float pz = ((V[8] * m[0] + V[9] * m[1]) + V[10] * m[2]) + V[11];

    // ---- colour: SH coefficients and view direction
    {
        float dir[3] = {m[0] - cam.campos[0], m[1] - cam.campos[1], m[2] - cam.campos[2]};
        const float len = sqrtf(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
        const float il = 1.0f / len;
        dir[0] *= il; dir[1] *= il; dir[2] *= il;
        float Y[16], Dx[16], Dy[16], Dz[16];
        sh_eval(sh_degree, dir[0], dir[1], dir[2], Y, Dx, Dy, Dz);
        float ddir[3] = {0.f, 0.f, 0.f};
        for (int ch = 0; ch < 3; ++ch) {
            float col = 0.0f;
            for (int k = 0; k < ncoef; ++k) col += Y[k] * sh[((size_t)k * 3 + ch) * n + g];
            if (col + 0.5f < 0.0f) dcol[ch] = 0.0f;   // clamped at 0: no gradient
            for (int k = 0; k < ncoef; ++k) {
                const float c = sh[((size_t)k * 3 + ch) * n + g];
                d_sh[((size_t)k * 3 + ch) * n + g] = Y[k] * dcol[ch];
                ddir[0] += dcol[ch] * c * Dx[k];
                ddir[1] += dcol[ch] * c * Dy[k];
                ddir[2] += dcol[ch] * c * Dz[k];
            }
        }
        const float dd = ddir[0] * dir[0] + ddir[1] * dir[1] + ddir[2] * dir[2];
#pragma unroll
        for (int k = 0; k < 3; ++k) dm[k] += (ddir[k] - dir[k] * dd) * il;
    }

    // ---- forward quantities of Eq. 2-3
    const float xx = qx * qx, yy = qy * qy, zz = qz * qz;
    const float xy = qx * qy, xz = qx * qz, yz = qy * qz;
    const float wx = qw * qx, wy = qw * qy, wz = qw * qz;
    const float Rm[3][3] = {{1.0f - 2.0f * (yy + zz), 2.0f * (xy - wz), 2.0f * (xz + wy)},
                            {2.0f * (xy + wz), 1.0f - 2.0f * (xx + zz), 2.0f * (yz - wx)},
                            {2.0f * (xz - wy), 2.0f * (yz + wx), 1.0f - 2.0f * (xx + yy)}};
    float M[3][3], Sg[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) M[i][j] = Rm[i][j] * s[j];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) Sg[i][j] = M[i][0] * M[j][0] + M[i][1] * M[j][1] + M[i][2] * M[j][2];
    const float rx = px / pz, ry = py / pz;
    const bool clx = rx < -cam.limx || rx > cam.limx;
    const bool cly = ry < -cam.limy || ry > cam.limy;
    const float tx = fminf(cam.limx, fmaxf(-cam.limx, rx)) * pz;
    const float ty = fminf(cam.limy, fmaxf(-cam.limy, ry)) * pz;
    const float iz = 1.0f / pz, iz2 = iz * iz;
    const float j00 = cam.fx * iz, j02 = -cam.fx * tx * iz2;
    const float j11 = cam.fy * iz, j12 = -cam.fy * ty * iz2;
    const float W0[3] = {V[0], V[1], V[2]}, W1[3] = {V[4], V[5], V[6]}, W2[3] = {V[8], V[9], V[10]};
    float T0[3], T1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        T0[k] = j00 * W0[k] + j02 * W2[k];
        T1[k] = j11 * W1[k] + j12 * W2[k];
    }
    float ST0[3], ST1[3];   // Sigma T0, Sigma T1
#pragma unroll
    for (int i = 0; i < 3; ++i) {
        ST0[i] = Sg[i][0] * T0[0] + Sg[i][1] * T0[1] + Sg[i][2] * T0[2];
        ST1[i] = Sg[i][0] * T1[0] + Sg[i][1] * T1[1] + Sg[i][2] * T1[2];
    }
    const float a = (T0[0] * ST0[0] + T0[1] * ST0[1] + T0[2] * ST0[2]) + 0.3f;
    const float b = T0[0] * ST1[0] + T0[1] * ST1[1] + T0[2] * ST1[2];
    const float c = (T1[0] * ST1[0] + T1[1] * ST1[1] + T1[2] * ST1[2]) + 0.3f;
    const float det = a * c - b * b;
    const float id2 = 1.0f / (det * det);

    // ---- conic = inverse of (a b; b c): d(a, b, c)
    const float da = (-c * c * dA + b * c * dB - b * b * dC) * id2;
    const float db = (2.0f * b * c * dA - (det + 2.0f * b * b) * dB + 2.0f * a * b * dC) * id2;
    const float dc = (-b * b * dA + a * b * dB - a * a * dC) * id2;

    // ---- (a, b, c) = (T0 Sigma T0, T0 Sigma T1, T1 Sigma T1)
    float dSg[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) dSg[i][j] = da * T0[i] * T0[j] + db * T0[i] * T1[j] + dc * T1[i] * T1[j];
    float dT0[3], dT1[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        dT0[k] = 2.0f * da * ST0[k] + db * ST1[k];
        dT1[k] = db * ST0[k] + 2.0f * dc * ST1[k];
    }
    // ---- T = J W
    const float dj00 = dT0[0] * W0[0] + dT0[1] * W0[1] + dT0[2] * W0[2];
    const float dj02 = dT0[0] * W2[0] + dT0[1] * W2[1] + dT0[2] * W2[2];
    const float dj11 = dT1[0] * W1[0] + dT1[1] * W1[1] + dT1[2] * W1[2];
    const float dj12 = dT1[0] * W2[0] + dT1[1] * W2[1] + dT1[2] * W2[2];
    // ---- J(t) and the projection (u, v) = (fx x / z + cx, fy y / z + cy)
    float dpx = cam.fx * iz * du, dpy = cam.fy * iz * dv;
    float dpz = -cam.fx * px * iz2 * du - cam.fy * py * iz2 * dv;
    dpz += -cam.fx * iz2 * dj00 - cam.fy * iz2 * dj11;
    const float dtx = -cam.fx * iz2 * dj02, dty = -cam.fy * iz2 * dj12;
    dpz += 2.0f * cam.fx * tx * iz2 * iz * dj02 + 2.0f * cam.fy * ty * iz2 * iz * dj12;
    if (clx) dpz += (rx > 0.0f ? cam.limx : -cam.limx) * dtx;
    else dpx += dtx;
    if (cly) dpz += (ry > 0.0f ? cam.limy : -cam.limy) * dty;
    else dpy += dty;
    // camera-space mean p = W m + t
#pragma unroll
    for (int k = 0; k < 3; ++k) dm[k] += W0[k] * dpx + W1[k] * dpy + W2[k] * dpz;

    // ---- Sigma = M M^T, M = R diag(s)
    float dM[3][3];
#pragma unroll
    for (int i = 0; i < 3; ++i)
#pragma unroll
        for (int j = 0; j < 3; ++j) {
            float acc = 0.0f;
#pragma unroll
            for (int k = 0; k < 3; ++k) acc += (dSg[i][k] + dSg[k][i]) * M[k][j];
            dM[i][j] = acc;
        }
    float dR[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j) {
        ds[j] = dM[0][j] * Rm[0][j] + dM[1][j] * Rm[1][j] + dM[2][j] * Rm[2][j];
#pragma unroll
        for (int i = 0; i < 3; ++i) dR[i][j] = dM[i][j] * s[j];
    }
    dq[0] = 2.0f * (-qz * dR[0][1] + qy * dR[0][2] + qz * dR[1][0] - qx * dR[1][2] - qy * dR[2][0] + qx * dR[2][1]);
    dq[1] = 2.0f * (qy * dR[0][1] + qz * dR[0][2] + qy * dR[1][0] - 2.0f * qx * dR[1][1] - qw * dR[1][2] +
                    qz * dR[2][0] + qw * dR[2][1] - 2.0f * qx * dR[2][2]);
    dq[2] = 2.0f * (-2.0f * qy * dR[0][0] + qx * dR[0][1] + qw * dR[0][2] + qx * dR[1][0] + qz * dR[1][2] -
                    qw * dR[2][0] + qz * dR[2][1] - 2.0f * qy * dR[2][2]);
    dq[3] = 2.0f * (-2.0f * qz * dR[0][0] - qw * dR[0][1] + qx * dR[0][2] + qw * dR[1][0] - 2.0f * qz * dR[1][1] +
                    qy * dR[1][2] + qx * dR[2][0] + qy * dR[2][1]);
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        d_means[(size_t)k * n + g] = dm[k];
        d_scales[(size_t)k * n + g] = ds[k];
    }
#pragma unroll
    for (int k = 0; k < 4; ++k) d_quats[(size_t)k * n + g] = dq[k];
    d_opac[g] = G[8];
}

template <typename T>
T *ws_at(const g4d_workspace *ws, size_t off) {
    return reinterpret_cast<T *>(static_cast<char *>(ws->ptr) + off);
}

}  // namespace

g4d_status render_backward(const g4d_splats *G, const g4d_camera *C, const g4d_workspace *ws,
                           const float *final_T, const int32_t *n_contrib, const float *grad_image,
                           const g4d_splats_grad *out, hipStream_t s) {
    if (!G || !C || !ws || !final_T || !n_contrib || !grad_image || !out) return G4D_EINVAL;
    WsLayout L;
    if (!ws->ptr || (reinterpret_cast<uintptr_t>(ws->ptr) & 255) ||
        !make_layout(ws->n_max, ws->width_max, ws->height_max, ws->instance_capacity, &L) || ws->bytes < L.total)
        return G4D_EINVAL;
    const int n = G->n;
    if (n < 0 || n > L.n_max || G->sh_degree < 0 || G->sh_degree > 3) return G4D_EINVAL;
    if (C->width < 1 || C->height < 1 || C->width > L.w_max || C->height > L.h_max) return G4D_EINVAL;
    if (n == 0) return G4D_OK;
    if (!G->means || !G->scales || !G->quats || !G->opacity || !G->sh) return G4D_EINVAL;
    if (!out->means || !out->scales || !out->quats || !out->opacity || !out->sh) return G4D_EINVAL;
    BwdCam cam{};
    for (int i = 0; i < 12; ++i) cam.v[i] = C->viewmat[i];
    cam.fx = C->fx; cam.fy = C->fy; cam.cx = C->cx; cam.cy = C->cy;
    cam.limx = 1.3f * C->tan_half_fov_x;
    cam.limy = 1.3f * C->tan_half_fov_y;
    for (int i = 0; i < 3; ++i) { cam.campos[i] = C->campos[i]; cam.bg[i] = C->bg[i]; }
    const int tiles_x = (C->width + kTile - 1) / kTile, tiles_y = (C->height + kTile - 1) / kTile;
    const int tiles = tiles_x * tiles_y;
    // the forward's instance layout: packed words (tile << gbits) | index, or two arrays
    int gbits = 1, tbits = 0;
    while (gbits < 32 && (1u << gbits) < (uint32_t)n) ++gbits;
    while ((1 << tbits) < tiles) ++tbits;
    const bool packed = gbits + tbits <= 32;
    const uint32_t *gids = packed ? ws_at<uint32_t>(ws, L.tk0) : ws_at<uint32_t>(ws, L.tv0);
    const uint32_t gmask = packed ? (1u << gbits) - 1u : 0xffffffffu;
    float *g2d = ws_at<float>(ws, L.grad2d);
    hipLaunchKernelGGL(k_fill_zero, dim3((unsigned)std::min<size_t>(((size_t)kG2 * n + 255) / 256, 4096)), dim3(256),
                       0, s, g2d, (size_t)kG2 * n);
    // entries per group: eight (130 VGPRs, three waves per SIMD) where few
    // Gaussians leave the kernel latency-bound, four (82 VGPRs) where many
    // tiles keep the chip busy and occupancy pays (measured at 2000 and at
    // 100k Gaussians, 800x800)
    auto blend_bwd = n <= kBlendBwdWideN ? k_blend_bwd<8> : k_blend_bwd<4>;
    hipLaunchKernelGGL(blend_bwd, dim3(tiles), dim3(256), 0, s, ws_at<uint4>(ws, L.order), gids, gmask,
                       ws_at<float4>(ws, L.recA), ws_at<float4>(ws, L.recB), ws_at<float4>(ws, L.recC), C->width,
                       C->height, tiles_x, tiles, cam, final_T, n_contrib, grad_image, g2d, n);
    hipLaunchKernelGGL(k_preprocess_bwd, dim3((n + 255) / 256), dim3(256), 0, s, n, G->sh_degree, G->means,
                       G->scales, G->quats, G->sh, cam, g2d, out->means, out->scales, out->quats, out->opacity,
                       out->sh);
    G4D_HIP_CHECK(hipGetLastError());
    return G4D_OK;
}

}  // namespace g4d

extern "C" g4d_status g4d_render_backward(const g4d_splats *G, const g4d_camera *C, const g4d_workspace *ws,
                                          const float *final_T, const int32_t *n_contrib, const float *grad_image,
                                          const g4d_splats_grad *grad, void *stream) {
    return g4d::render_backward(G, C, ws, final_T, n_contrib, grad_image, grad, reinterpret_cast<hipStream_t>(stream));
}
