// Device helpers shared by the path stage and the backward pass.
#pragma once

#include "sbr_internal.h"
#include "nu_weights.h"

namespace sbr {

// ------------------------------------------------------------------ helpers
struct cd {
    double re, im;
};
__device__ __forceinline__ cd cmul(cd a, cd b) { return {a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re}; }
__device__ __forceinline__ cd cdivz(cd a, cd b) {
    double q = b.re * b.re + b.im * b.im;
    return {(a.re * b.re + a.im * b.im) / q, (a.im * b.re - a.re * b.im) / q};
}
__device__ __forceinline__ cd csqrtp(cd z) {   // principal branch
    double r = sqrt(z.re * z.re + z.im * z.im);
    double x = sqrt(0.5 * (r + fabs(z.re)));
    if (x == 0.0) return {0.0, 0.0};
    double y = 0.5 * z.im / x;
    if (z.re >= 0.0) return {x, y};
    return {fabs(y), z.im >= 0.0 ? x : -x};
}

// Reflection coefficient (Eqs. 9-10 with n = sqrt(eps_c), Snell
// sin(dt) = sin(di)/n) and its derivative with respect to cos(di).
__device__ inline void reflect_coef(const MatTable &mt, int mi, double fc, double ci, cd &r, cd &dr) {
    int mode = (mt.n > 0 && mi < mt.n) ? mt.mode[mi] : 0;
    if (mode == 0) {
        r = {-1.0, 0.0};
        dr = {0.0, 0.0};
        return;
    }
    cd eps = {mt.eps_r[mi], -mt.sigma[mi] / (2.0 * kPi * fc * kEps0)};
    cd n = csqrtp(eps);
    // cos(dt) = sqrt(1 - (1 - ci^2) / eps)
    cd s2 = cdivz({1.0 - ci * ci, 0.0}, eps);
    cd ct = csqrtp({1.0 - s2.re, -s2.im});
    // d ct / d ci = (ci / eps) / ct
    cd dct = cdivz(cdivz({ci, 0.0}, eps), ct);
    if (mode == 1) {
        cd nct = cmul(n, ct), ndct = cmul(n, dct);
        cd num = {ci - nct.re, -nct.im}, den = {ci + nct.re, nct.im};
        r = cdivz(num, den);
        // d/dci (ci - n ct)/(ci + n ct) = 2 n (ct - ci dct) / den^2
        cd t = {ct.re - ci * dct.re, ct.im - ci * dct.im};
        cd top = cmul({2.0 * n.re, 2.0 * n.im}, t);
        dr = cdivz(top, cmul(den, den));
    } else {
        cd nci = {n.re * ci, n.im * ci};
        cd num = {nci.re - ct.re, nci.im - ct.im}, den = {nci.re + ct.re, nci.im + ct.im};
        r = cdivz(num, den);
        // d/dci (n ci - ct)/(n ci + ct) = 2 n (ct - ci dct) / den^2
        cd t = {ct.re - ci * dct.re, ct.im - ci * dct.im};
        cd top = cmul({2.0 * n.re, 2.0 * n.im}, t);
        dr = cdivz(top, cmul(den, den));
    }
}

// d r / d eps_c of the reflection coefficient above (holomorphic in eps_c);
// zero for the conductor.
__device__ inline cd reflect_deps(const MatTable &mt, int mi, double fc, double ci) {
    int mode = (mt.n > 0 && mi < mt.n) ? mt.mode[mi] : 0;
    if (mode == 0) return {0.0, 0.0};
    cd eps = {mt.eps_r[mi], -mt.sigma[mi] / (2.0 * kPi * fc * kEps0)};
    cd n = csqrtp(eps);
    cd s2 = cdivz({1.0 - ci * ci, 0.0}, eps);
    cd ct = csqrtp({1.0 - s2.re, -s2.im});
    cd dn = cdivz({0.5, 0.0}, n);                                   // 1 / (2 n)
    cd dct = cdivz(cdivz(s2, eps), {2.0 * ct.re, 2.0 * ct.im});     // (s^2 / eps^2) / (2 ct)
    if (mode == 1) {
        // r = (ci - K)/(ci + K), K = n ct
        cd K = cmul(n, ct);
        cd dK = {dn.re * ct.re - dn.im * ct.im + (n.re * dct.re - n.im * dct.im),
                 dn.re * ct.im + dn.im * ct.re + (n.re * dct.im + n.im * dct.re)};
        cd den = {ci + K.re, K.im};
        cd drdK = cdivz({-2.0 * ci, 0.0}, cmul(den, den));
        return cmul(drdK, dK);
    }
    // r = (a - b)/(a + b), a = n ci, b = ct:  dr = 2 (a' b - a b') / (a + b)^2
    cd a = {n.re * ci, n.im * ci}, b = ct;
    cd da = {dn.re * ci, dn.im * ci};
    cd t1 = cmul(da, b), t2 = cmul(a, dct);
    cd num = {2.0 * (t1.re - t2.re), 2.0 * (t1.im - t2.im)};
    cd den = {a.re + b.re, a.im + b.im};
    return cdivz(num, cmul(den, den));
}

// Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011): ten rounds of two
// 32 x 32 -> 64-bit products with the published multipliers, the key bumped by
// the Weyl constants after each round.  Words 0 and 1 of the output.
__device__ __forceinline__ void philox2(uint32_t c0, uint32_t c1, uint32_t c2, uint32_t c3, uint32_t k0, uint32_t k1,
                                        uint32_t *w0, uint32_t *w1) {
#pragma unroll
    for (int r = 0; r < 10; r++) {
        const uint32_t h0 = __umulhi(0xD2511F53u, c0), l0 = 0xD2511F53u * c0;
        const uint32_t h1 = __umulhi(0xCD9E8D57u, c2), l1 = 0xCD9E8D57u * c2;
        const uint32_t n0 = h1 ^ c1 ^ k0, n2 = h0 ^ c3 ^ k1;
        c0 = n0;
        c1 = l1;
        c2 = n2;
        c3 = l0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    *w0 = c0;
    *w1 = c1;
}

// Unit direction of grid cell (ix, iy) in the radar frame and its solid angle:
// at the cell centre, or with SBR_RAYS_JITTER at a Philox-drawn point of it.
__device__ __forceinline__ void grid_dir_local(const GridDev &g, int ix, int iy, double dr[3], double *dw) {
    double jx = 0.5, jy = 0.5;
    if (g.options & SBR_RAYS_JITTER) {
        uint32_t w0, w1;
        philox2((uint32_t)(iy * g.nx + ix), 0u, 0u, 0u, g.seed_lo, g.seed_hi, &w0, &w1);
        jx = (double)(w0 >> 8) * (1.0 / 16777216.0);
        jy = (double)(w1 >> 8) * (1.0 / 16777216.0);
    }
    double u = g.thx * (2.0 * (ix + jx) / g.nx - 1.0);
    double v = g.thy * (2.0 * (iy + jy) / g.ny - 1.0);
    double q = 1.0 + u * u + v * v;
    double s = 1.0 / sqrt(q);
    dr[0] = u * s;
    dr[1] = v * s;
    dr[2] = s;
    *dw = (2.0 * g.thx / g.nx) * (2.0 * g.thy / g.ny) / (q * sqrt(q));
}

__device__ __forceinline__ void grid_ray(const GridDev &g, const RadarDev &rd, int ix, int iy,
                                         double d[3], double *dw) {
    double dr[3];
    grid_dir_local(g, ix, iy, dr, dw);
    for (int i = 0; i < 3; i++) d[i] = rd.rot[3 * i] * dr[0] + rd.rot[3 * i + 1] * dr[1] + rd.rot[3 * i + 2] * dr[2];
}


// Bounces of ray r that return a path: a hit that is not occluded, not cut
// by SBR_DROP_FLAGGED (a flag other than SBR_HIT_OCCLUDED ends the ray's
// paths), and with SBR_EXIT_ONLY only the ray's last hit.  Bit k = bounce k;
// *nb = highest returning bounce + 1 (0 when none).  A face id outside
// [0, nf) ends the ray like a miss, so no face outside the mesh is read.
__device__ __forceinline__ uint32_t ray_path_mask(const int32_t *tri, const uint8_t *flags, size_t R, size_t r,
                                                  int K, int nf, bool drop, bool exit_only, int *nb) {
    uint32_t mask = 0;
    int nh = 0;
    bool cut = false;
    for (int k = 0; k < K; k++) {
        const size_t slot = (size_t)k * R + r;
        if ((unsigned)tri[slot] >= (unsigned)nf) break;
        nh = k + 1;
        const uint8_t fl = flags[slot];
        if (drop && (fl & ~SBR_HIT_OCCLUDED)) cut = true;
        if (!cut && !(fl & SBR_HIT_OCCLUDED)) mask |= 1u << k;
    }
    if (exit_only) mask &= nh > 0 ? (1u << (nh - 1)) : 0u;
    *nb = mask ? 32 - __clz((int)mask) : 0;
    return mask;
}


// Deconvolution of the non-uniform FFT forms: 1 / Psi((s - S/2) / 2S) for
// mode s < S, with Psi(xi) = int psi(z) e^{-2 pi j xi z} dz by the trapezoid
// rule at kNuSteps points per grid unit (psi vanishes with all its
// derivatives up to the order of e^{-beta} at the ends of its support):
// Psi = h (psi(0) + 2 sum_n psi(nh) cos(2 pi xi n h)), h = 1/kNuSteps, the
// cosines by the three-term recurrence, all in FP64.  kn holds the kernel
// samples psi(n h), n < kNuTaps (nu_kernel_sample).
constexpr int kNuSteps = 16;
constexpr int kNuTaps = kNuW * kNuSteps / 2;   // n h < W/2
__device__ inline double nu_kernel_sample(int n) {
    const double x = 2.0 * n / (double)(kNuW * kNuSteps);
    return exp(kNuBeta * (sqrt(1.0 - x * x) - 1.0));
}
__device__ inline float nu_corr_value(int S, int s, const double *kn) {
    const int M = 2 * S;
    const double c1 = cospi(2.0 * (double)(s - S / 2) / (double)(M * kNuSteps));
    double cp = 1.0, cc = c1, acc = kn[0] + 2.0 * kn[1] * c1;
    for (int n = 2; n < kNuTaps; n++) {
        const double cn = 2.0 * c1 * cc - cp;
        cp = cc;
        cc = cn;
        acc += 2.0 * kn[n] * cn;
    }
    return (float)((double)kNuSteps / acc);
}

// The kNuW tap weights of the non-uniform FFT kernel for a point at grid
// coordinate x = rint(x) + u, u in [-1/2, 1/2]: w[t] = psi(u + 3 - t) for the
// taps l = rint(x) - 3 + t, from the polynomial forms of nu_weights.h (even
// and odd parts in u, so that mirrored taps share them); no transcendentals.
__device__ __forceinline__ void nu_weights(float u, float w[kNuW]) {
    const float u2 = u * u;
#pragma unroll
    for (int t = 0; t <= kNuHalf; t++) {
        float e = kNuPolyE[t][kNuPolyNE - 1];
#pragma unroll
        for (int k = kNuPolyNE - 2; k >= 0; k--) e = fmaf(e, u2, kNuPolyE[t][k]);
        if (t == kNuHalf) {
            w[t] = e;
        } else {
            float o = kNuPolyO[t][kNuPolyNO - 1];
#pragma unroll
            for (int k = kNuPolyNO - 2; k >= 0; k--) o = fmaf(o, u2, kNuPolyO[t][k]);
            w[t] = fmaf(u, o, e);
            w[kNuW - 1 - t] = fmaf(-u, o, e);
        }
    }
}

}  // namespace sbr
