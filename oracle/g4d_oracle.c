/*
 * CPU oracle for the 4D-GS deform-then-splat render.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path may link, load or
 * call this file; it exists so that tests, the smoke check and the CPU
 * baseline of the benchmark can compare the HIP path against a plain,
 * slow, obviously correct implementation.  It shares no code with the HIP
 * path.
 *
 * Precision policy
 *   - Continuous values (deformation field, MLP, covariance inverse,
 *     colour, compositing weights and colours) are computed in FP64.
 *   - The discrete structure of the splat rasterizer (culling, screen-space
 *     radius, tile rectangle, and the depth key, which embeds the bits of a
 *     binary32 depth) is a binary32 object by definition, so it is computed
 *     in binary32 with a fixed operation order, no FMA contraction and
 *     correctly rounded division and square root.
 *   - The per-pixel skip/stop decisions of the compositing loop are taken in
 *     binary32 (the precision the kernel works in), alongside the FP64
 *     accumulation of colour; pixels whose binary32 decisions lie within a
 *     small relative margin of a threshold are flagged.
 *
 * Method sources (paper: "4D Gaussian Splatting for Real-Time Dynamic Scene
 * Rendering"):
 *   - HexPlane encoder: Sec. 4.2, Eq. 7 (bilinear queries of six planes per
 *     scale, element-wise product over planes, concatenation over scales).
 *   - Decoder: Sec. 4.2 (feature merger phi_d, heads phi_x, phi_r, phi_s)
 *     and Eq. 8 (X' = X + dX, r' = r + dr, s' = s + ds).
 *   - Splatting: Sec. 3.1, Eq. 1 (Gaussian), Eq. 2 (Sigma = R S S^T R^T),
 *     Eq. 3 (Sigma' = J W Sigma W^T J^T), Eq. 4 (front-to-back compositing
 *     of depth-ordered points), and the tile rasterizer of 3D-GS that the
 *     paper renders with (Sec. 4.1).
 *
 * Build: gcc -O2 -fopenmp -ffp-contract=off -fno-fast-math -shared -fPIC
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define ORC_TILE 16

/* ------------------------------------------------------------------ */
/* Sec. 4.2, Eq. 7: bilinear interpolation on one feature plane.        */
/* Plane layout [nb][na][F].  Coordinates (ua, ub) are in [-1, 1];      */
/* the corners of the plane sit at -1 and +1 (align-corners), and       */
/* queries outside are clamped to the border.                           */
/* ------------------------------------------------------------------ */
static void bilinear(const float *plane, int na, int nb, int F, double ua, double ub,
                     double *out /* F */)
{
    double ga = (ua + 1.0) * 0.5 * (double)(na - 1);
    double gb = (ub + 1.0) * 0.5 * (double)(nb - 1);
    if (ga < 0.0) ga = 0.0;
    if (ga > (double)(na - 1)) ga = (double)(na - 1);
    if (gb < 0.0) gb = 0.0;
    if (gb > (double)(nb - 1)) gb = (double)(nb - 1);
    int ia = (int)floor(ga), ib = (int)floor(gb);
    if (ia > na - 2) ia = na - 2;
    if (ib > nb - 2) ib = nb - 2;
    if (ia < 0) ia = 0;
    if (ib < 0) ib = 0;
    double wa = ga - (double)ia, wb = gb - (double)ib;
    const float *p00 = plane + ((size_t)ib * na + ia) * F;
    const float *p10 = plane + ((size_t)ib * na + ia + 1) * F;
    const float *p01 = plane + ((size_t)(ib + 1) * na + ia) * F;
    const float *p11 = plane + ((size_t)(ib + 1) * na + ia + 1) * F;
    for (int f = 0; f < F; ++f) {
        out[f] = (1.0 - wa) * (1.0 - wb) * (double)p00[f]
               + wa * (1.0 - wb) * (double)p10[f]
               + (1.0 - wa) * wb * (double)p01[f]
               + wa * wb * (double)p11[f];
    }
}

/* Exported for tests: one bilinear query. */
void orc_bilinear(const float *plane, int na, int nb, int F, double ua, double ub, double *out)
{
    bilinear(plane, na, nb, F, ua, ub, out);
}

/* Round to bfloat16 (round to nearest, ties to even), returned as a
 * double.  The argument is first rounded to binary32: the emulation models
 * a decoder that holds f_h and h as binary32 values (its own FP32
 * arithmetic) and rounds those to bfloat16 for the matrix products.
 * Infinities and NaN pass through.  Used only by the BF16-emulation mode. */
static double to_bf16(double x)
{
    float f = (float)x;
    uint32_t u;
    memcpy(&u, &f, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (double)f;
    uint32_t lsb = (u >> 16) & 1u;
    u = (u + 0x7fffu + lsb) & 0xffff0000u;
    memcpy(&f, &u, 4);
    return (double)f;
}

/* Exported for tests: to_bf16 over an array. */
void orc_to_bf16(int64_t n, const double *x, double *out)
{
    for (int64_t i = 0; i < n; ++i) out[i] = to_bf16(x[i]);
}

/* ------------------------------------------------------------------ */
/* Sec. 4.2 + Eq. 7 + Eq. 8: FP64 deformation of n canonical Gaussians. */
/*                                                                      */
/* Plane axes per scale, in order: (x,y), (x,z), (y,z), (x,t), (y,t),   */
/* (z,t); axis a is the fast (column) index of plane [n_b][n_a][F].     */
/* res[4*l + k] = resolution of axis k (x, y, z, t) at scale l.         */
/* Coordinates: u_k = 2 (mu_k - bmin_k) / (bmax_k - bmin_k) - 1 and     */
/* u_t = 2 t - 1, queried at the canonical mean.                        */
/* Decoder: h = ReLU(W1 f_h + b1); dx = Wx h + bx; dr = Wr h + br;      */
/* ds = Ws h + bs.  Outputs are render-ready: mean' = mean + dx;         */
/* scale' = exp(log_scale + ds); quat' = normalise(quat + dr) (zero     */
/* norm -> identity); opacity = sigmoid(logit).                         */
/* bf16_emulate != 0 rounds f_h, W1, h and the head weights to bf16      */
/* before the FP64 products (biases stay binary32).                     */
/* Appendix (colour and opacity deformation), optional: with wc, the    */
/* colour head dC = Wc h + bc gives one offset per SH coefficient       */
/* (n_sh = 3 (d+1)^2 rows, in the order of the colour array) and        */
/* out_sh = sh_in + dC; with wa, dalpha = Wa h + ba shifts the opacity  */
/* logit: opacity = sigmoid(logit + dalpha).                            */
/* ------------------------------------------------------------------ */
void orc_deform(int n, const float *means, const float *log_scales, const float *quats,
                const float *opacity_logits,
                int n_scales, int F, const float *bmin, const float *bmax, const int *res,
                const float *const *planes /* [n_scales*6] */,
                int in_dim, int hidden, const float *w1, const float *b1,
                const float *wx, const float *bx, const float *wr, const float *br,
                const float *ws, const float *bs, double t, int bf16_emulate,
                double *out_means, double *out_scales, double *out_quats, double *out_opacity,
                double *out_fh /* nullable [n][in_dim] */, double *out_delta /* nullable [n][10] */,
                int n_sh, const float *wc /* nullable [n_sh][hidden] */, const float *bc,
                const float *wa /* nullable [1][hidden] */, const float *ba,
                const float *sh_in /* [n_sh][n], read with wc */, double *out_sh /* [n_sh][n] */)
{
    static const int axes[6][2] = {{0, 1}, {0, 2}, {1, 2}, {0, 3}, {1, 3}, {2, 3}};
    const float *heads_w[3] = {wx, wr, ws};
    const float *heads_b[3] = {bx, br, bs};
    const int heads_n[3] = {3, 4, 3};

#pragma omp parallel for schedule(dynamic, 256)
    for (int g = 0; g < n; ++g) {
        double u[4];
        for (int k = 0; k < 3; ++k) {
            double m = (double)means[(size_t)k * n + g];
            u[k] = 2.0 * (m - (double)bmin[k]) / ((double)bmax[k] - (double)bmin[k]) - 1.0;
        }
        u[3] = 2.0 * t - 1.0;

        double fh[4 * 64];
        double tmp[64];
        for (int l = 0; l < n_scales; ++l) {
            double *fl = fh + l * F;
            for (int f = 0; f < F; ++f) fl[f] = 1.0;
            for (int p = 0; p < 6; ++p) {
                int a = axes[p][0], b = axes[p][1];
                int na = res[4 * l + a], nb = res[4 * l + b];
                bilinear(planes[6 * l + p], na, nb, F, u[a], u[b], tmp);
                for (int f = 0; f < F; ++f) fl[f] *= tmp[f];
            }
        }
        if (out_fh)
            for (int i = 0; i < in_dim; ++i) out_fh[(size_t)g * in_dim + i] = fh[i];

        double hbuf[512];
        for (int j = 0; j < hidden; ++j) {
            double acc = 0.0;
            for (int i = 0; i < in_dim; ++i) {
                double wv = (double)w1[(size_t)j * in_dim + i];
                double fv = fh[i];
                if (bf16_emulate) { wv = to_bf16(wv); fv = to_bf16(fv); }
                acc += wv * fv;
            }
            acc += (double)b1[j];
            hbuf[j] = acc > 0.0 ? acc : 0.0;
        }
        double delta[10];
        int o = 0;
        for (int hd = 0; hd < 3; ++hd) {
            for (int r = 0; r < heads_n[hd]; ++r) {
                double acc = 0.0;
                for (int j = 0; j < hidden; ++j) {
                    double wv = (double)heads_w[hd][(size_t)r * hidden + j];
                    double hv = hbuf[j];
                    if (bf16_emulate) { wv = to_bf16(wv); hv = to_bf16(hv); }
                    acc += wv * hv;
                }
                delta[o++] = acc + (double)heads_b[hd][r];
            }
        }
        if (out_delta)
            for (int i = 0; i < 10; ++i) out_delta[(size_t)g * 10 + i] = delta[i];

        /* appendix heads: phi_C and phi_alpha on the same h */
        double dalpha = 0.0;
        if (wa) {
            double acc = 0.0;
            for (int j = 0; j < hidden; ++j) {
                double wv = (double)wa[j], hv = hbuf[j];
                if (bf16_emulate) { wv = to_bf16(wv); hv = to_bf16(hv); }
                acc += wv * hv;
            }
            dalpha = acc + (double)ba[0];
        }
        if (wc) {
            for (int r = 0; r < n_sh; ++r) {
                double acc = 0.0;
                for (int j = 0; j < hidden; ++j) {
                    double wv = (double)wc[(size_t)r * hidden + j], hv = hbuf[j];
                    if (bf16_emulate) { wv = to_bf16(wv); hv = to_bf16(hv); }
                    acc += wv * hv;
                }
                out_sh[(size_t)r * n + g] = (double)sh_in[(size_t)r * n + g] + acc + (double)bc[r];
            }
        }

        /* Eq. 8 and activations */
        for (int k = 0; k < 3; ++k)
            out_means[(size_t)k * n + g] = (double)means[(size_t)k * n + g] + delta[k];
        double q[4], qn = 0.0;
        for (int k = 0; k < 4; ++k) {
            q[k] = (double)quats[(size_t)k * n + g] + delta[3 + k];
            qn += q[k] * q[k];
        }
        qn = sqrt(qn);
        for (int k = 0; k < 4; ++k)
            out_quats[(size_t)k * n + g] = qn > 0.0 ? q[k] / qn : (k == 0 ? 1.0 : 0.0);
        for (int k = 0; k < 3; ++k)
            out_scales[(size_t)k * n + g] = exp((double)log_scales[(size_t)k * n + g] + delta[7 + k]);
        out_opacity[g] = 1.0 / (1.0 + exp(-((double)opacity_logits[g] + dalpha)));
    }
}

/* ------------------------------------------------------------------ */
/* Real spherical harmonics, degree <= 3, from the closed form          */
/*   Y_l^0 = K_l^0 P_l^0(cos th)                                        */
/*   Y_l^m = sqrt2 K_l^m cos(m ph) P_l^m(cos th)   (m > 0)              */
/*   Y_l^m = sqrt2 K_l^|m| sin(|m| ph) P_l^|m|(cos th)   (m < 0)        */
/* with K_l^m = sqrt((2l+1)/(4 pi) (l-m)!/(l+m)!) and associated        */
/* Legendre functions carrying the Condon-Shortley phase.  Coefficient  */
/* index l*l + l + m.  (Sec. 3.1: colour from k SH functions.)          */
/* ------------------------------------------------------------------ */
static double factorial(int k)
{
    double r = 1.0;
    for (int i = 2; i <= k; ++i) r *= (double)i;
    return r;
}

static double assoc_legendre(int l, int m, double x)
{
    /* P_m^m = (-1)^m (2m-1)!! (1-x^2)^(m/2) */
    double pmm = 1.0;
    double s = sqrt(fmax(0.0, 1.0 - x * x));
    for (int i = 1; i <= m; ++i) pmm *= -(2.0 * i - 1.0) * s;
    if (l == m) return pmm;
    double pmm1 = x * (2.0 * m + 1.0) * pmm;
    if (l == m + 1) return pmm1;
    double pll = 0.0;
    for (int ll = m + 2; ll <= l; ++ll) {
        pll = ((2.0 * ll - 1.0) * x * pmm1 - (ll + m - 1.0) * pmm) / (double)(ll - m);
        pmm = pmm1;
        pmm1 = pll;
    }
    return pll;
}

double orc_sh_basis(int l, int m, double x, double y, double z)
{
    const double PI = 3.14159265358979323846;
    int am = m < 0 ? -m : m;
    double K = sqrt((2.0 * l + 1.0) / (4.0 * PI) * factorial(l - am) / factorial(l + am));
    double ph = atan2(y, x);
    double P = assoc_legendre(l, am, z);
    if (m == 0) return K * P;
    if (m > 0) return sqrt(2.0) * K * cos(am * ph) * P;
    return sqrt(2.0) * K * sin(am * ph) * P;
}

/* ------------------------------------------------------------------ */
/* Projection (Sec. 3.1, Eq. 2-3) for render-ready Gaussians.           */
/*                                                                      */
/* Camera: view[12] row-major 3x4 world->camera (W = its 3x3 block);    */
/* intr = {fx, fy, cx, cy, tan_half_fov_x, tan_half_fov_y, near};       */
/* campos[3]; image width x height; 16x16 tiles, tiles_x = ceil(W/16).  */
/*                                                                      */
/* Binary32 part (exact replica of the discrete structure):             */
/*   p = W mu + t; culled unless p.z > near;                            */
/*   R(q) from the unit quaternion (w,x,y,z); M = R diag(s);            */
/*   Sigma = M M^T; clamped x/z, y/z at +-1.3 tan_half_fov;             */
/*   J = [[fx/z, 0, -fx x/z^2], [0, fy/z, -fy y/z^2]]; T = J W;          */
/*   Sigma' = T Sigma T^T, +0.3 on the diagonal; culled unless det > 0;  */
/*   lambda_max = mid + sqrt(max(0.1, mid^2 - det)); r = ceil(3 sqrt l); */
/*   (u, v) = (fx x/z + cx, fy y/z + cy) with the unclamped ratios;      */
/*   tile rectangle [floor((u-r)/16), floor((u+r)/16)+1) clamped to the  */
/*   grid, same in y; culled if empty.  Depth key = bits of p.z.         */
/*   Conic (for the blend decisions): inverse of Sigma' in binary32.     */
/* FP64 part: u, v, conic and colour from the same binary32 inputs.      */
/* Colour = sum_k sh_k Y_k(dir) + 0.5, clamped at 0, with dir the unit   */
/* vector from the camera centre to the (deformed) mean.                 */
/* ------------------------------------------------------------------ */
void orc_project(int n, int sh_degree, const float *means, const float *scales,
                 const float *quats, const float *sh,
                 const float *view, const float *intr, const float *campos, int width, int height,
                 int32_t *rect /* [n][4] x0,y0,x1,y1 */, uint32_t *depth_bits, int32_t *radius,
                 float *f32_out /* [n][8]: u, v, a, b, c, conic_a, conic_b, conic_c */,
                 double *f64_out /* [n][8]: u, v, conic_a, conic_b, conic_c, r, g, b */)
{
    const int tiles_x = (width + ORC_TILE - 1) / ORC_TILE;
    const int tiles_y = (height + ORC_TILE - 1) / ORC_TILE;
    const int nsh = (sh_degree + 1) * (sh_degree + 1);

#pragma omp parallel for schedule(static)
    for (int g = 0; g < n; ++g) {
        int32_t *rc = rect + 4 * (size_t)g;
        rc[0] = rc[1] = rc[2] = rc[3] = 0;
        radius[g] = 0;
        depth_bits[g] = 0xffffffffu;
        for (int k = 0; k < 8; ++k) { f32_out[8 * (size_t)g + k] = 0.0f; f64_out[8 * (size_t)g + k] = 0.0; }

        const float mx = means[g], my = means[(size_t)n + g], mz = means[2 * (size_t)n + g];
        const float sx = scales[g], sy = scales[(size_t)n + g], sz = scales[2 * (size_t)n + g];
        const float qw = quats[g], qx = quats[(size_t)n + g], qy = quats[2 * (size_t)n + g],
                    qz = quats[3 * (size_t)n + g];
        if (!(isfinite(mx) && isfinite(my) && isfinite(mz) && isfinite(sx) && isfinite(sy) &&
              isfinite(sz) && isfinite(qw) && isfinite(qx) && isfinite(qy) && isfinite(qz)))
            continue;

        /* ---------------- binary32 key path ---------------- */
        float px = ((view[0] * mx + view[1] * my) + view[2] * mz) + view[3];
        float py = ((view[4] * mx + view[5] * my) + view[6] * mz) + view[7];
        float pz = ((view[8] * mx + view[9] * my) + view[10] * mz) + view[11];
        if (!(pz > intr[6])) continue;

        float xx = qx * qx, yy = qy * qy, zz = qz * qz;
        float xy = qx * qy, xz = qx * qz, yz = qy * qz;
        float wx = qw * qx, wy = qw * qy, wz = qw * qz;
        float R[3][3];
        R[0][0] = 1.0f - 2.0f * (yy + zz);
        R[0][1] = 2.0f * (xy - wz);
        R[0][2] = 2.0f * (xz + wy);
        R[1][0] = 2.0f * (xy + wz);
        R[1][1] = 1.0f - 2.0f * (xx + zz);
        R[1][2] = 2.0f * (yz - wx);
        R[2][0] = 2.0f * (xz - wy);
        R[2][1] = 2.0f * (yz + wx);
        R[2][2] = 1.0f - 2.0f * (xx + yy);
        float s3[3] = {sx, sy, sz};
        float M[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) M[i][j] = R[i][j] * s3[j];
        float S[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = i; j < 3; ++j) {
                S[i][j] = (M[i][0] * M[j][0] + M[i][1] * M[j][1]) + M[i][2] * M[j][2];
                S[j][i] = S[i][j];
            }

        const float fx = intr[0], fy = intr[1], cx = intr[2], cy = intr[3];
        const float limx = 1.3f * intr[4], limy = 1.3f * intr[5];
        float rx = px / pz, ry = py / pz;
        float crx = fminf(limx, fmaxf(-limx, rx));
        float cry = fminf(limy, fmaxf(-limy, ry));
        float tx = crx * pz, ty = cry * pz;
        float zz2 = pz * pz;
        float j00 = fx / pz, j02 = -((fx * tx) / zz2);
        float j11 = fy / pz, j12 = -((fy * ty) / zz2);
        float T[2][3];
        for (int k = 0; k < 3; ++k) {
            T[0][k] = j00 * view[k] + j02 * view[8 + k];
            T[1][k] = j11 * view[4 + k] + j12 * view[8 + k];
        }
        float U[2][3];
        for (int i = 0; i < 2; ++i)
            for (int k = 0; k < 3; ++k)
                U[i][k] = (T[i][0] * S[0][k] + T[i][1] * S[1][k]) + T[i][2] * S[2][k];
        float ca = (U[0][0] * T[0][0] + U[0][1] * T[0][1]) + U[0][2] * T[0][2];
        float cb = (U[0][0] * T[1][0] + U[0][1] * T[1][1]) + U[0][2] * T[1][2];
        float cc = (U[1][0] * T[1][0] + U[1][1] * T[1][1]) + U[1][2] * T[1][2];
        ca = ca + 0.3f;
        cc = cc + 0.3f;
        float det = ca * cc - cb * cb;
        if (!(det > 0.0f)) continue;
        float mid = 0.5f * (ca + cc);
        float disc = fmaxf(0.1f, mid * mid - det);
        float lam = mid + sqrtf(disc);
        float rad = ceilf(3.0f * sqrtf(lam));
        float u = fx * rx + cx;
        float v = fy * ry + cy;
        if (!(isfinite(u) && isfinite(v) && isfinite(rad))) continue;
        float fx0 = floorf((u - rad) * 0.0625f);
        float fx1 = floorf((u + rad) * 0.0625f) + 1.0f;
        float fy0 = floorf((v - rad) * 0.0625f);
        float fy1 = floorf((v + rad) * 0.0625f) + 1.0f;
        int x0 = (int)fminf(fmaxf(fx0, 0.0f), (float)tiles_x);
        int x1 = (int)fminf(fmaxf(fx1, 0.0f), (float)tiles_x);
        int y0 = (int)fminf(fmaxf(fy0, 0.0f), (float)tiles_y);
        int y1 = (int)fminf(fmaxf(fy1, 0.0f), (float)tiles_y);
        if (x1 <= x0 || y1 <= y0) continue;
        rc[0] = x0; rc[1] = y0; rc[2] = x1; rc[3] = y1;
        radius[g] = (int32_t)rad;
        uint32_t bits;
        memcpy(&bits, &pz, 4);
        depth_bits[g] = bits;
        float inv = 1.0f / det;
        float *o32 = f32_out + 8 * (size_t)g;
        o32[0] = u; o32[1] = v; o32[2] = ca; o32[3] = cb; o32[4] = cc;
        o32[5] = cc * inv; o32[6] = -(cb * inv); o32[7] = ca * inv;

        /* ---------------- FP64 continuous values ---------------- */
        double dm[3] = {mx, my, mz};
        double dp[3];
        for (int i = 0; i < 3; ++i)
            dp[i] = (double)view[4 * i] * dm[0] + (double)view[4 * i + 1] * dm[1] +
                    (double)view[4 * i + 2] * dm[2] + (double)view[4 * i + 3];
        double dq[4] = {qw, qx, qy, qz};
        double R64[3][3];
        R64[0][0] = 1 - 2 * (dq[2] * dq[2] + dq[3] * dq[3]);
        R64[0][1] = 2 * (dq[1] * dq[2] - dq[0] * dq[3]);
        R64[0][2] = 2 * (dq[1] * dq[3] + dq[0] * dq[2]);
        R64[1][0] = 2 * (dq[1] * dq[2] + dq[0] * dq[3]);
        R64[1][1] = 1 - 2 * (dq[1] * dq[1] + dq[3] * dq[3]);
        R64[1][2] = 2 * (dq[2] * dq[3] - dq[0] * dq[1]);
        R64[2][0] = 2 * (dq[1] * dq[3] - dq[0] * dq[2]);
        R64[2][1] = 2 * (dq[2] * dq[3] + dq[0] * dq[1]);
        R64[2][2] = 1 - 2 * (dq[1] * dq[1] + dq[2] * dq[2]);
        double ds[3] = {sx, sy, sz};
        double Sg[3][3];
        for (int i = 0; i < 3; ++i)
            for (int j = 0; j < 3; ++j) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k) acc += R64[i][k] * ds[k] * ds[k] * R64[j][k];
                Sg[i][j] = acc;
            }
        double drx = dp[0] / dp[2], dry = dp[1] / dp[2];
        double dlimx = 1.3 * (double)intr[4], dlimy = 1.3 * (double)intr[5];
        double dtx = fmin(dlimx, fmax(-dlimx, drx)) * dp[2];
        double dty = fmin(dlimy, fmax(-dlimy, dry)) * dp[2];
        double J[2][3] = {{(double)fx / dp[2], 0.0, -(double)fx * dtx / (dp[2] * dp[2])},
                          {0.0, (double)fy / dp[2], -(double)fy * dty / (dp[2] * dp[2])}};
        double Tm[2][3];
        for (int i = 0; i < 2; ++i)
            for (int k = 0; k < 3; ++k) {
                double acc = 0.0;
                for (int j = 0; j < 3; ++j) acc += J[i][j] * (double)view[4 * j + k];
                Tm[i][k] = acc;
            }
        double C2[2][2];
        for (int i = 0; i < 2; ++i)
            for (int j = 0; j < 2; ++j) {
                double acc = 0.0;
                for (int k = 0; k < 3; ++k)
                    for (int l = 0; l < 3; ++l) acc += Tm[i][k] * Sg[k][l] * Tm[j][l];
                C2[i][j] = acc;
            }
        C2[0][0] += 0.3;
        C2[1][1] += 0.3;
        double ddet = C2[0][0] * C2[1][1] - C2[0][1] * C2[1][0];
        double *o64 = f64_out + 8 * (size_t)g;
        o64[0] = (double)fx * drx + (double)cx;
        o64[1] = (double)fy * dry + (double)cy;
        o64[2] = C2[1][1] / ddet;
        o64[3] = -C2[0][1] / ddet;
        o64[4] = C2[0][0] / ddet;

        double dir[3] = {dm[0] - (double)campos[0], dm[1] - (double)campos[1],
                         dm[2] - (double)campos[2]};
        double dn = sqrt(dir[0] * dir[0] + dir[1] * dir[1] + dir[2] * dir[2]);
        for (int i = 0; i < 3; ++i) dir[i] /= dn;
        for (int ch = 0; ch < 3; ++ch) {
            double acc = 0.0;
            for (int l = 0; l <= sh_degree; ++l)
                for (int m = -l; m <= l; ++m) {
                    int k = l * l + l + m;
                    acc += (double)sh[((size_t)k * 3 + ch) * n + g] *
                           orc_sh_basis(l, m, dir[0], dir[1], dir[2]);
                }
            acc += 0.5;
            o64[5 + ch] = acc > 0.0 ? acc : 0.0;
        }
        (void)nsh;
    }
}

/* ------------------------------------------------------------------ */
/* Tile instances: one (key, gid) per Gaussian and touched tile.        */
/* key = (tile_id << 32) | depth_bits, tile_id = ty * tiles_x + tx.     */
/* Emission order is gid-major, tiles row-major; the list is then       */
/* ordered by (key, gid), which is the stable order of the keys.        */
/* ------------------------------------------------------------------ */
int64_t orc_count_instances(int n, const int32_t *rect)
{
    int64_t k = 0;
    for (int g = 0; g < n; ++g)
        k += (int64_t)(rect[4 * g + 2] - rect[4 * g + 0]) * (rect[4 * g + 3] - rect[4 * g + 1]);
    return k;
}

typedef struct { uint64_t key; uint32_t val; } kv_t;

static int kv_cmp(const void *a, const void *b)
{
    const kv_t *x = (const kv_t *)a, *y = (const kv_t *)b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->val != y->val) return x->val < y->val ? -1 : 1;
    return 0;
}

void orc_emit_instances(int n, const int32_t *rect, const uint32_t *depth_bits, int tiles_x,
                        uint64_t *keys, uint32_t *vals)
{
    int64_t o = 0;
    for (int g = 0; g < n; ++g) {
        const int32_t *rc = rect + 4 * (size_t)g;
        for (int ty = rc[1]; ty < rc[3]; ++ty)
            for (int tx = rc[0]; tx < rc[2]; ++tx) {
                keys[o] = ((uint64_t)(uint32_t)(ty * tiles_x + tx) << 32) | (uint64_t)depth_bits[g];
                vals[o] = (uint32_t)g;
                ++o;
            }
    }
}

void orc_sort_instances(int64_t k, uint64_t *keys, uint32_t *vals)
{
    kv_t *tmp = (kv_t *)malloc((size_t)(k > 0 ? k : 1) * sizeof(kv_t));
    for (int64_t i = 0; i < k; ++i) { tmp[i].key = keys[i]; tmp[i].val = vals[i]; }
    qsort(tmp, (size_t)k, sizeof(kv_t), kv_cmp);
    for (int64_t i = 0; i < k; ++i) { keys[i] = tmp[i].key; vals[i] = tmp[i].val; }
    free(tmp);
}

/* ranges[2*t], ranges[2*t+1] = [first, last+1) of tile t in the sorted list */
void orc_tile_ranges(int64_t k, const uint64_t *keys, int n_tiles, int64_t *ranges)
{
    for (int t = 0; t < 2 * n_tiles; ++t) ranges[t] = 0;
    for (int64_t i = 0; i < k; ++i) {
        int t = (int)(keys[i] >> 32);
        if (i == 0 || (int)(keys[i - 1] >> 32) != t) ranges[2 * t] = i;
        if (i == k - 1 || (int)(keys[i + 1] >> 32) != t) ranges[2 * t + 1] = i + 1;
    }
}

/* ------------------------------------------------------------------ */
/* Eq. 1 + Eq. 4: front-to-back compositing per pixel.                  */
/* For each Gaussian of the pixel's tile list, in order:               */
/*   d = (u - px, v - py); power = -1/2 (A dx^2 + C dy^2) - B dx dy     */
/*   skip if power > 0; alpha = min(0.99, o exp(power));                */
/*   skip if alpha < 1/255; stop (without adding) if T (1 - alpha) <    */
/*   1e-4; otherwise colour += c alpha T and T *= (1 - alpha).           */
/* Output colour + T * bg, the final T, the number of list entries      */
/* visited up to the last contributor, and (if evals is not null) the   */
/* number of list entries the pixel evaluates: up to and including the  */
/* entry that stops it, else the whole list.  If used is not null, the  */
/* pixel's decision signature is written there: used[2p] = number of     */
/* Gaussians composited, used[2p+1] = a polynomial hash of their indices */
/* in compositing order; two renders whose signatures agree composited  */
/* the same Gaussians in the same order at that pixel (a test aid: the  */
/* hash takes no part in the image).                                    */
/* Decisions are taken in binary32 (values f32 from orc_project); the   */
/* colour and T are accumulated in FP64 from the FP64 values.  flag[p]  */
/* counts binary32 decisions within `margin` (relative) of their        */
/* threshold (for the sign of power: relative to the magnitude of its   */
/* terms); such pixels are excluded from element-wise comparison.       */
/* ------------------------------------------------------------------ */
void orc_blend(int width, int height, const int64_t *ranges, const uint32_t *vals,
               const float *opacity, const float *f32v /* [n][8] */, const double *f64v /* [n][8] */,
               const float *bg, double margin,
               double *image /* [3][H][W] */, double *final_T /* [H][W] */,
               int32_t *n_contrib /* [H][W] */, int32_t *flag /* [H][W] */, int32_t *evals /* [H][W] or NULL */,
               int64_t *used /* [H][W][2] or NULL */)
{
    const int tiles_x = (width + ORC_TILE - 1) / ORC_TILE;
    const float a_min = 1.0f / 255.0f;
    const float t_min = 0.0001f;

#pragma omp parallel for schedule(dynamic, 1)
    for (int py = 0; py < height; ++py) {
        for (int px = 0; px < width; ++px) {
            int tile = (py / ORC_TILE) * tiles_x + (px / ORC_TILE);
            int64_t b = ranges[2 * tile], e = ranges[2 * tile + 1];
            double T = 1.0, C[3] = {0.0, 0.0, 0.0};
            float T32 = 1.0f;
            int last = 0, fl = 0;
            int64_t n_used = 0;
            uint64_t seq_hash = 0;
            int ev = (int)(e - b);
            const float fpx = (float)px, fpy = (float)py;
            for (int64_t i = b; i < e; ++i) {
                const uint32_t g = vals[i];
                const float *v32 = f32v + 8 * (size_t)g;
                const double *v64 = f64v + 8 * (size_t)g;
                /* binary32 decision track */
                float dx = v32[0] - fpx, dy = v32[1] - fpy;
                float p1 = (v32[5] * dx) * dx;
                float p2 = (v32[7] * dy) * dy;
                float p3 = (v32[6] * dx) * dy;
                float power32 = -0.5f * (p1 + p2) - p3;
                /* the form is positive definite, so power <= 0 exactly; its   */
                /* sign test only resolves rounding: flag when it is that close */
                float mag = 0.5f * (fabsf(p1) + fabsf(p2)) + fabsf(p3);
                if (fabsf(power32) < (float)margin * mag) ++fl;
                if (power32 > 0.0f) continue;
                float alpha32 = fminf(0.99f, opacity[g] * expf(power32));
                if (fabsf(alpha32 - a_min) <= (float)margin * a_min) ++fl;
                if (alpha32 < a_min) continue;
                float test32 = T32 * (1.0f - alpha32);
                if (fabsf(test32 - t_min) <= (float)(10.0 * margin) * t_min) ++fl;
                if (test32 < t_min) {
                    ev = (int)(i - b) + 1;
                    break;
                }
                /* FP64 values */
                double ddx = v64[0] - (double)px, ddy = v64[1] - (double)py;
                double power = -0.5 * (v64[2] * ddx * ddx + v64[4] * ddy * ddy) - v64[3] * ddx * ddy;
                double alpha = fmin(0.99, (double)opacity[g] * exp(power));
                for (int ch = 0; ch < 3; ++ch) C[ch] += v64[5 + ch] * alpha * T;
                T *= (1.0 - alpha);
                T32 = test32;
                last = (int)(i - b) + 1;
                ++n_used;
                seq_hash = seq_hash * 1000003u + (uint64_t)g + 1u;
            }
            size_t pix = (size_t)py * width + px;
            for (int ch = 0; ch < 3; ++ch)
                image[(size_t)ch * width * height + pix] = C[ch] + T * (double)bg[ch];
            final_T[pix] = T;
            n_contrib[pix] = last;
            flag[pix] = fl;
            if (evals) evals[pix] = ev;
            if (used) {
                used[2 * pix] = n_used;
                used[2 * pix + 1] = (int64_t)seq_hash;
            }
        }
    }
}
