// Backpropagation: adjoint of the IF synthesis (Eqs. 11-12) per path, then
// the reverse sweep through the ray geometry of every ray (Eq. 13 chain rule)
// with per-bounce recomputation, scattering dL/dverts.
#include <vector>

#include "sbr_internal.h"
#include "sbr_device.h"

namespace sbr {

namespace {

struct AdjArgs {
    const int32_t *count;
    PathSoA rec;
    const float2 *G;       // [V][C][S]
    int32_t V, C, S;
    int32_t rows;          // G rows per LDS stage (direct form)
    int32_t Sp;            // S rounded up to a multiple of 8
    int32_t v_per;         // antennas per y-block
    int32_t nvs;           // y-blocks
    int32_t ppl;           // paths per lane of the kernel that runs this request
    float fcf, sl_fs, tc;  // fc, slope / fs, chirp period
    float *tau_bar;        // [V][cap]
    float2 *abar_part;     // [nvs][cap]
    float *tdb_part;       // [nvs][cap] dL/d taudot partials
    const float4 *nu_rows; // [V][C][2S + 8] non-uniform FFT rows (NULL: direct form)
    float *nu_corr;        // [S] its 1/Psi table
};

constexpr int kAdjRowsMax = 8;   // G rows staged in LDS at a time
constexpr int kAdjPPL = 2;       // paths per lane, direct form
constexpr int kNuPPL = 4;        // paths per lane, non-uniform FFT form
constexpr int kAdjQueueDirect = 32;   // work counter of the direct form (queue[0]: the other)

// ---- Eqs. 11-12 by a type-2 non-uniform FFT -------------------------------
// For each (v, c) the two sums of the adjoint are finite Fourier series of one
// G row evaluated at a path's beat frequency g (cycles per sample, reduced to
// [-1/2, 1/2]):
//   P(g) = sum_s h1_s e^{2 pi j s g},  h1_s = conj(G_s)
//   Q(g) = sum_s h2_s e^{2 pi j s g},  h2_s = conj(G_s) (fc + (slope/fs) s)
// (Q = fc P + (slope/fs) x P'(x) of the direct form).  By the identity of the
// non-uniform FFT forms (sbr_internal.h),
//   P(g) = e^{2 pi j g S/2} sum_l u_l psi(gM - l),
//   u_l  = sum_s' (h_{s'+S/2} / Psi(s'/M)) e^{2 pi j s' l / M}:
// the rows u (one per (v, c), shared by every path) cost one dense DFT each,
// and a path then needs kNuW taps per (v, c) instead of S terms; the error
// stays below 1e-6 of sum_s |h_s| at every g (two orders of magnitude under
// the FP32 rounding of a 256-term direct sum).
// float4's layout for address-space-qualified 16-byte loads of the rows
struct alignas(16) F4 {
    float x, y, z, w;
};
__device__ __forceinline__ SBR_GLOBAL_AS const F4 *gmem4(const float4 *p) { return (SBR_GLOBAL_AS const F4 *)p; }

// Chirp rows per LDS stage of the non-uniform FFT adjoint: about 36 KiB
// (4 rows at S = 256), 1 .. 8 rows.
__host__ __device__ inline int nu_stage(int S) { return max(1, min(8, 36864 / (nu_row_len(S) * 16))); }

// frac(n f) for an integer-valued n < 2^24: the product is exact inside the fma
__device__ __forceinline__ float frac_of_product(float n, float f) { return fmaf(n, f, -rintf(n * f)); }

// 1 / Psi((s - S/2) / 2S) for s < S (nu_corr_value) of request blockIdx.y of an
// adjoint batch, blocks of 256 modes.
__global__ __launch_bounds__(256) void k_nu_corr_adj(const AdjArgs *__restrict__ args) {
    __shared__ double kn[kNuTaps];
    if (threadIdx.x < kNuTaps) kn[threadIdx.x] = nu_kernel_sample((int)threadIdx.x);
    __syncthreads();
    const AdjArgs &a = args[blockIdx.y];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < a.S) a.nu_corr[s] = nu_corr_value(a.S, s, kn);
}


// Gradient row (v, c) of a request of the batch (blocks [first[j], first[j + 1])
// are request j's rows, v major): u1_l, u2_l (float4: u1.re, u1.im, u2.re, u2.im)
// for l = -M/2 - 3 .. M/2 + 3 at index l + M/2 + 3, the DFT of the S
// deconvolved modes (mode s' = s - S/2 at position s' mod M of an M-point
// sequence, zero elsewhere) with twiddles e^{2 pi j k / M} from an
// exact-index LDS table: for M a power of two an in-place radix-2 FFT in LDS
// (both sequences in the same butterflies), otherwise a direct sum per
// output; the last entry of the row is zero padding.
__global__ __launch_bounds__(256) void k_nu_rows(const AdjArgs *__restrict__ args, const int32_t *__restrict__ first,
                                                 int m) {
    extern __shared__ float4 nsh[];
    // request j of the batch owns blocks (rows) [first[j], first[j + 1])
    int j = 0, hi = m;
    while (hi - j > 1) {
        const int mid = (j + hi) >> 1;
        if (first[mid] <= (int)blockIdx.x) j = mid;
        else hi = mid;
    }
    const AdjArgs &a = args[j];
    const float2 *__restrict__ G = a.G;
    const float *__restrict__ corr = a.nu_corr;
    float4 *__restrict__ rows = const_cast<float4 *>(a.nu_rows);
    const int S = a.S;
    const float fcf = a.fcf, sl_fs = a.sl_fs;
    const int M = 2 * S, RL = nu_row_len(S);
    float2 *tw = reinterpret_cast<float2 *>(nsh + M);        // [M], after the M-point sequence
    const size_t row = (size_t)((int)blockIdx.x - first[j]);
    for (int k = threadIdx.x; k < M; k += blockDim.x) {
        double sn, cs;
        sincospi(2.0 * k / M, &sn, &cs);
        tw[k] = make_float2((float)cs, (float)sn);
    }
    const float2 *g = G + row * S;
    float4 *out = rows + row * RL;
    if ((M & (M - 1)) == 0) {
        // a[n] = h_{s}, n = (s - S/2) mod M (zero for the other half), stored
        // at bit-reversed positions; X[l] = sum_n a[n] e^{2 pi j n l / M}
        float4 *a4 = nsh;   // [M]
        const int lg = 31 - __clz(M);
        for (int n = threadIdx.x; n < M; n += blockDim.x) {
            const int s = (n + S / 2) % M;
            float4 h = make_float4(0.f, 0.f, 0.f, 0.f);
            if (s < S) {
                const float2 v = g[s];
                const float r = corr[s];
                const float w2 = fmaf(sl_fs, (float)s, fcf);
                const float hr = v.x * r, hi = -v.y * r;   // conj(G_s) / Psi
                h = make_float4(hr, hi, hr * w2, hi * w2);
            }
            a4[__brev((uint32_t)n) >> (32 - lg)] = h;
        }
        __syncthreads();
        for (int half = 1; half < M; half <<= 1) {
            const int tstep = M / (2 * half);
            for (int i = threadIdx.x; i < M / 2; i += blockDim.x) {
                const int pos = i & (half - 1), j0 = ((i - pos) << 1) + pos, j1 = j0 + half;
                const float2 w = tw[pos * tstep];
                const float4 u = a4[j0], v = a4[j1];
                const float4 vw = make_float4(v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x,
                                              v.z * w.x - v.w * w.y, v.z * w.y + v.w * w.x);
                a4[j0] = make_float4(u.x + vw.x, u.y + vw.y, u.z + vw.z, u.w + vw.w);
                a4[j1] = make_float4(u.x - vw.x, u.y - vw.y, u.z - vw.z, u.w - vw.w);
            }
            __syncthreads();
        }
        for (int i = threadIdx.x; i < RL; i += blockDim.x) {
            if (i < RL - 1) {
                int lm = (i - (M / 2 + kNuHalf)) % M;   // l mod M
                if (lm < 0) lm += M;
                out[i] = a4[lm];
            } else {
                out[i] = make_float4(0.f, 0.f, 0.f, 0.f);
            }
        }
        return;
    }
    float4 *hb = nsh;   // [S] h1, h2 over Psi
    for (int s = threadIdx.x; s < S; s += blockDim.x) {
        const float2 v = g[s];
        const float r = corr[s];
        const float w2 = fmaf(sl_fs, (float)s, fcf);
        const float hr = v.x * r, hi = -v.y * r;   // conj(G_s) / Psi
        hb[s] = make_float4(hr, hi, hr * w2, hi * w2);
    }
    __syncthreads();
    for (int i = threadIdx.x; i < RL; i += blockDim.x) {
        float ar = 0.f, ai = 0.f, br = 0.f, bi = 0.f;
        if (i < RL - 1) {
            int lm = (i - (M / 2 + kNuHalf)) % M;   // l mod M
            if (lm < 0) lm += M;
            int k = (int)(((long long)(M - S / 2) * lm) % M);   // (s - S/2) l mod M at s = 0
            for (int s = 0; s < S; s++) {
                const float2 t = tw[k];
                const float4 h = hb[s];
                ar = fmaf(h.x, t.x, fmaf(-h.y, t.y, ar));
                ai = fmaf(h.x, t.y, fmaf(h.y, t.x, ai));
                br = fmaf(h.z, t.x, fmaf(-h.w, t.y, br));
                bi = fmaf(h.z, t.y, fmaf(h.w, t.x, bi));
                k += lm;
                if (k >= M) k -= M;
            }
        }
        out[i] = make_float4(ar, ai, br, bi);
    }
}

// One work item of the non-uniform FFT form: per path and (v, c) the taps
// l0 .. l0 + 6 around x = gM (l0 = rint(x) - 3) of both rows, kernel weights
// from their polynomial forms (nu_weights), and the same accumulation as the
// direct form with z0 e^{2 pi j g S/2} as the phase factor.  That phase is
// alpha + c beta + (S/2) g = alpha + (S/2) gamma + c (beta + (S/2) eps) up to
// an integer ((S/2) times the integer that reduces g), so from one chirp to
// the next the factor turns by r = e^{2 pi j (beta + (S/2) eps)}: it is
// computed exactly at the first chirp of each stage and rotated by r for the
// others (at most 7 rotations).  The rows of `stage` chirps at a time are
// copied to LDS by the whole block (coalesced 16-byte loads), so that each
// row read from L2 serves the item's 256 PPL paths, and paths of similar beat
// frequency read the same LDS words.
template <int PPL>
__device__ __forceinline__ void adj_item_nu(const AdjArgs &a, float4 *rsh, const int stage, const int P,
                                            const int grp, const int blk_p0) {
    const auto amp = gmem(a.rec.amp);
    const auto bet = gmem(a.rec.beta);
    const auto eps = gmem(a.rec.epsd);
    const auto alp = gmem(a.rec.alpha);
    const auto gam = gmem(a.rec.gamma);
    const auto tbar = gmem(a.tau_bar);
    int pp[PPL];
    bool act[PPL];
    float Ax[PPL], Ay[PPL], beta[PPL], epsd[PPL], abr[PPL], abi[PPL], tdb[PPL], rc[PPL], rs[PPL];
    const int S = a.S, M = 2 * S, RL = nu_row_len(S);
    const float Mf = (float)M, halfS = (float)(S / 2);
#pragma unroll
    for (int i = 0; i < PPL; i++) {
        pp[i] = blk_p0 + i * 256 + threadIdx.x;
        act[i] = pp[i] < P;
        const int pc = act[i] ? pp[i] : blk_p0;
        const F2 A = amp[pc];
        Ax[i] = A.x;
        Ay[i] = A.y;
        beta[i] = bet[pc];
        epsd[i] = eps[pc];
        abr[i] = abi[i] = tdb[i] = 0.0f;
        pp[i] = pc;
        float rt = beta[i] + frac_of_product(halfS, epsd[i]);   // turn per chirp
        rt -= rintf(rt);
        rs[i] = __builtin_amdgcn_sinf(rt);
        rc[i] = __builtin_amdgcn_cosf(rt);
    }
    const int v0 = grp * a.v_per, v1 = min(a.V, v0 + a.v_per);
    for (int v = v0; v < v1; v++) {
        float alpha[PPL], gamma[PPL], tb[PPL];
#pragma unroll
        for (int i = 0; i < PPL; i++) {
            alpha[i] = alp[(size_t)v * a.rec.cap + pp[i]];
            gamma[i] = gam[(size_t)v * a.rec.cap + pp[i]];
            tb[i] = 0.0f;
        }
        const auto rows_v = gmem4(a.nu_rows) + (size_t)v * a.C * RL;
        for (int c0 = 0; c0 < a.C; c0 += stage) {
            const int nr = min(stage, a.C - c0);
            __syncthreads();   // the previous stage has been read
            for (int i = threadIdx.x; i < nr * RL; i += 256) {
                const F4 u = rows_v[(size_t)c0 * RL + i];
                rsh[i] = make_float4(u.x, u.y, u.z, u.w);
            }
            __syncthreads();
            float zc[PPL], zs[PPL];   // phase factor of the current chirp
            for (int cc = 0; cc < nr; cc++) {
                const float cf = (float)(c0 + cc);
                const float4 *row = rsh + cc * RL;
#pragma unroll
                for (int i = 0; i < PPL; i++) {
                    const float f = fmaf(cf, epsd[i], gamma[i]);
                    const float g = f - rintf(f);   // [-1/2, 1/2]
                    const float x = g * Mf;         // exact
                    const float xr = rintf(x);
                    const int i0 = min(max((int)xr + M / 2, 0), M);   // row index of l0 = xr - 3 (clamped: NaN-safe)
                    float w[kNuW];
                    nu_weights(x - xr, w);
                    float pr = 0.f, pi = 0.f, qr = 0.f, qi = 0.f;
#pragma unroll
                    for (int t = 0; t < kNuW; t++) {
                        const float4 u = row[i0 + t];
                        pr = fmaf(w[t], u.x, pr);
                        pi = fmaf(w[t], u.y, pi);
                        qr = fmaf(w[t], u.z, qr);
                        qi = fmaf(w[t], u.w, qi);
                    }
                    if (cc == 0) {   // block-uniform
                        float th = alpha[i] + frac_of_product(cf, beta[i]) + frac_of_product(halfS, g);
                        th -= rintf(th);
                        zs[i] = __builtin_amdgcn_sinf(th);
                        zc[i] = __builtin_amdgcn_cosf(th);
                    } else {
                        const float tc = zc[i] * rc[i] - zs[i] * rs[i];
                        zs[i] = zc[i] * rs[i] + zs[i] * rc[i];
                        zc[i] = tc;
                    }
                    // Q0 = z0 P, m = z0 Q (z0 including e^{2 pi j g S/2})
                    const float q0r = zc[i] * pr - zs[i] * pi, q0i = zc[i] * pi + zs[i] * pr;
                    const float mr = zc[i] * qr - zs[i] * qi, mi = zc[i] * qi + zs[i] * qr;
                    abr[i] += q0r;
                    abi[i] -= q0i;
                    const float dq = -2.0f * (float)kPi * (Ax[i] * mi + Ay[i] * mr);
                    tb[i] += dq;
                    tdb[i] = fmaf(dq, cf * a.tc, tdb[i]);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < PPL; i++)
            if (act[i]) tbar[(size_t)v * a.rec.cap + pp[i]] = tb[i];
    }
#pragma unroll
    for (int i = 0; i < PPL; i++)
        if (act[i]) {
            gmem(a.abar_part)[(size_t)grp * a.rec.cap + pp[i]] = F2{abr[i], abi[i]};
            gmem(a.tdb_part)[(size_t)grp * a.rec.cap + pp[i]] = tdb[i];
        }
}

// Path-stationary adjoint of Eq. (8).  For each (path, v, c) the sums
//   P(x) = sum_s conj(G_s) x^s,  P'(x)   with x = e^{2 pi j delta}
// run by Horner's rule; with z0 = e^{2 pi j phi0}:
//   sum_s w_s = z0 P(x),  sum_s s w_s = z0 x P'(x),  w_s = conj(G_s) e^{j phi_s}
//   dL/dA    += conj(z0 P(x))                                  (Eq. 12)
//   dL/dtau  += -2 pi Im(A (fc z0 P + (slope/fs) z0 x P'))       (Eq. 11)
// Each lane carries PPL paths (256 apart) so every G sample read from LDS
// feeds 8 * PPL fused multiply-adds.
//
// Work items are (antenna group, tile of 256 * PPL paths) pairs, antenna group
// major; the number of live paths is only known on the device, so a grid of
// about one device-full of blocks takes items from an atomic counter until
// they run out (no blocks are launched for the empty path slots).
template <int PPL>
__device__ __forceinline__ void adj_item(const AdjArgs &a, float2 *gsh, const int P, const int grp,
                                         const int blk_p0) {
    const auto amp = gmem(a.rec.amp);
    const auto bet = gmem(a.rec.beta);
    const auto eps = gmem(a.rec.epsd);
    const auto alp = gmem(a.rec.alpha);
    const auto gam = gmem(a.rec.gamma);
    const auto tbar = gmem(a.tau_bar);
    int pp[PPL];
    bool act[PPL];
    float2 A[PPL];
    float beta[PPL], epsd[PPL], abr[PPL], abi[PPL], tdb[PPL];
#pragma unroll
    for (int i = 0; i < PPL; i++) {
        pp[i] = blk_p0 + i * 256 + threadIdx.x;
        act[i] = pp[i] < P;
        const int pc = act[i] ? pp[i] : blk_p0;
        A[i] = make_float2(amp[pc].x, amp[pc].y);
        beta[i] = bet[pc];
        epsd[i] = eps[pc];
        abr[i] = 0.0f;
        abi[i] = 0.0f;
        tdb[i] = 0.0f;
        pp[i] = pc;
    }
    const int v0 = grp * a.v_per, v1 = min(a.V, v0 + a.v_per);
    const int S = a.S;
    for (int v = v0; v < v1; v++) {
        float alpha[PPL], gamma[PPL], tb[PPL];
#pragma unroll
        for (int i = 0; i < PPL; i++) {
            alpha[i] = alp[(size_t)v * a.rec.cap + pp[i]];
            gamma[i] = gam[(size_t)v * a.rec.cap + pp[i]];
            tb[i] = 0.0f;
        }
        for (int c0 = 0; c0 < a.C; c0 += a.rows) {
            const int nr = min(a.rows, a.C - c0);
            __syncthreads();
            // rows padded with zeros to Sp = S rounded up to 8: leading zero
            // coefficients leave Horner's recurrences unchanged
            const auto src = gmem(a.G) + ((size_t)v * a.C + c0) * S;
            for (int i = threadIdx.x; i < nr * a.Sp; i += 256) {
                const int rr = i / a.Sp, ss = i - rr * a.Sp;
                if (ss < S) {
                    const F2 g = src[(size_t)rr * S + ss];
                    gsh[i] = make_float2(g.x, g.y);
                } else {
                    gsh[i] = make_float2(0.0f, 0.0f);
                }
            }
            __syncthreads();
            for (int cc = 0; cc < nr; cc++) {
                const int c = c0 + cc;
                const float cf = (float)c;
                float zs[PPL], zc[PPL], xs[PPL], xc[PPL], pr[PPL], pi[PPL], qr[PPL], qi[PPL];
#pragma unroll
                for (int i = 0; i < PPL; i++) {
                    const float delta = fmaf(cf, epsd[i], gamma[i]);
                    const float cb = cf * beta[i];
                    float ph = alpha[i] + fmaf(cf, beta[i], -rintf(cb));
                    ph -= rintf(ph);
                    zs[i] = __builtin_amdgcn_sinf(ph);
                    zc[i] = __builtin_amdgcn_cosf(ph);
                    const float dd = delta - rintf(delta);
                    xs[i] = __builtin_amdgcn_sinf(dd);
                    xc[i] = __builtin_amdgcn_cosf(dd);
                    pr[i] = pi[i] = qr[i] = qi[i] = 0.0f;
                }
                const float4 *g4 = reinterpret_cast<const float4 *>(gsh + cc * a.Sp);
                // q = q x + p ;  p = p x + conj(g_s), s descending
#define SBR_HORNER_STEP(GR, GI)                                                 \
    _Pragma("unroll") for (int i = 0; i < PPL; i++) {                          \
        float nqr = fmaf(qr[i], xc[i], fmaf(-qi[i], xs[i], pr[i]));            \
        float nqi = fmaf(qr[i], xs[i], fmaf(qi[i], xc[i], pi[i]));             \
        float npr = fmaf(pr[i], xc[i], fmaf(-pi[i], xs[i], (GR)));             \
        float npi = fmaf(pr[i], xs[i], fmaf(pi[i], xc[i], -(GI)));             \
        qr[i] = nqr;                                                           \
        qi[i] = nqi;                                                           \
        pr[i] = npr;                                                           \
        pi[i] = npi;                                                           \
    }
                for (int j = a.Sp / 2 - 4; j >= 0; j -= 4) {
                    const float4 h3 = g4[j + 3], h2 = g4[j + 2], h1 = g4[j + 1], h0 = g4[j];
                    SBR_HORNER_STEP(h3.z, h3.w)
                    SBR_HORNER_STEP(h3.x, h3.y)
                    SBR_HORNER_STEP(h2.z, h2.w)
                    SBR_HORNER_STEP(h2.x, h2.y)
                    SBR_HORNER_STEP(h1.z, h1.w)
                    SBR_HORNER_STEP(h1.x, h1.y)
                    SBR_HORNER_STEP(h0.z, h0.w)
                    SBR_HORNER_STEP(h0.x, h0.y)
                }
#undef SBR_HORNER_STEP
#pragma unroll
                for (int i = 0; i < PPL; i++) {
                    // Q0 = z0 P, Q1 = z0 x P'
                    const float q0r = zc[i] * pr[i] - zs[i] * pi[i], q0i = zc[i] * pi[i] + zs[i] * pr[i];
                    const float xqr = xc[i] * qr[i] - xs[i] * qi[i], xqi = xc[i] * qi[i] + xs[i] * qr[i];
                    const float q1r = zc[i] * xqr - zs[i] * xqi, q1i = zc[i] * xqi + zs[i] * xqr;
                    abr[i] += q0r;
                    abi[i] -= q0i;
                    const float mr = a.fcf * q0r + a.sl_fs * q1r;
                    const float mi = a.fcf * q0i + a.sl_fs * q1i;
                    const float dq = -2.0f * (float)kPi * (A[i].x * mi + A[i].y * mr);
                    tb[i] += dq;
                    tdb[i] += dq * (cf * a.tc);   // tau(c) = tau + c t_chirp taudot
                }
            }
        }
#pragma unroll
        for (int i = 0; i < PPL; i++)
            if (act[i]) tbar[(size_t)v * a.rec.cap + pp[i]] = tb[i];
    }
#pragma unroll
    for (int i = 0; i < PPL; i++)
        if (act[i]) {
            gmem(a.abar_part)[(size_t)grp * a.rec.cap + pp[i]] = F2{abr[i], abi[i]};
            gmem(a.tdb_part)[(size_t)grp * a.rec.cap + pp[i]] = tdb[i];
        }
}

// Work items of each request of a batch: (antenna groups) x (path tiles of
// 256 x args[i].ppl paths) for its device-side path count; item_first[i] =
// first item of request i, item_first[n] = total.  Also clears the work
// counters of both adjoint forms.  One block.
__global__ __launch_bounds__(1024) void k_adj_items(const AdjArgs *args, int n, uint32_t *item_first,
                                                    uint32_t *queue) {
    __shared__ uint32_t part[1024];
    const int t = threadIdx.x;
    const int chunk = (n + 1023) / 1024;
    const int b = t * chunk, e = min(n, b + chunk);
    uint32_t sum = 0;
    for (int i = b; i < e; i++) {
        const uint32_t P = (uint32_t)args[i].count[0], tile = 256u * (uint32_t)args[i].ppl;
        sum += (P + tile - 1u) / tile * (uint32_t)args[i].nvs;
    }
    part[t] = sum;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        const uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - sum;
    for (int i = b; i < e; i++) {
        item_first[i] = run;
        const uint32_t P = (uint32_t)args[i].count[0], tile = 256u * (uint32_t)args[i].ppl;
        run += (P + tile - 1u) / tile * (uint32_t)args[i].nvs;
    }
    if (t == 1023) item_first[n] = part[1023];
    if (t == 0) {
        queue[0] = 0u;
        queue[kAdjQueueDirect] = 0u;
    }
}

// Request of a work item: binary search over item_first[lo .. hi).
__device__ __forceinline__ int adj_request(const uint32_t *item_first, int lo, int hi, uint32_t item) {
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (item_first[mid] <= item) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Work items of requests [r0, r1) of a batch (one request for sbr_backward)
// are taken from one atomic counter by about one device-full of blocks; an
// item is mapped to its request by binary search over item_first, then to
// (antenna group, path tile) exactly as in a launch of its own.  `slot` is
// the LDS float2 offset of the work-item word (after the largest G-row stage).
template <int PPL>
__global__ __launch_bounds__(256) void k_synth_adj(const AdjArgs *__restrict__ args,
                                                   const uint32_t *__restrict__ item_first, int r0, int r1,
                                                   uint32_t *queue, int slot) {
    // [rows][Sp] G rows, then the current work item.  No static LDS: it would
    // shift the dynamic area off the 16-byte alignment of the row reads.
    extern __shared__ float2 gsh[];
    uint32_t &s_item = *reinterpret_cast<uint32_t *>(gsh + slot);
    const uint32_t first = item_first[r0], total = item_first[r1];
    for (;;) {
        __syncthreads();   // the previous item is done with s_item and gsh
        if (threadIdx.x == 0) s_item = first + atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= total) break;   // uniform over the block
        const int lo = adj_request(item_first, r0, r1, item);
        const AdjArgs &a = args[lo];
        const int P = __builtin_amdgcn_readfirstlane(*gmem(a.count));
        const uint32_t tiles = (uint32_t)((P + 256 * PPL - 1) / (256 * PPL));
        const uint32_t local = item - item_first[lo];
        adj_item<PPL>(a, gsh, P, (int)(local / tiles), (int)(local % tiles) * 256 * PPL);
    }
}

// The same work queue over requests [r0, r1) for the non-uniform FFT form;
// `stage` rows of nu_row_len(S) float4 per LDS stage, the work-item word
// after the largest stage (float4 offset `slot`).
template <int PPL>
__global__ __launch_bounds__(256) void k_synth_adj_nu(const AdjArgs *__restrict__ args,
                                                      const uint32_t *__restrict__ item_first, int r0, int r1,
                                                      uint32_t *queue, int slot) {
    extern __shared__ float4 rsh[];
    uint32_t &s_item = *reinterpret_cast<uint32_t *>(rsh + slot);
    const uint32_t first = item_first[r0], total = item_first[r1];
    for (;;) {
        __syncthreads();   // the previous item is done with s_item and the rows
        if (threadIdx.x == 0) s_item = first + atomicAdd(queue, 1u);
        __syncthreads();
        const uint32_t item = __builtin_amdgcn_readfirstlane(s_item);
        if (item >= total) break;   // uniform over the block
        const int lo = adj_request(item_first, r0, r1, item);
        const AdjArgs &a = args[lo];
        const int P = __builtin_amdgcn_readfirstlane(*gmem(a.count));
        const uint32_t tiles = (uint32_t)((P + 256 * PPL - 1) / (256 * PPL));
        const uint32_t local = item - item_first[lo];
        adj_item_nu<PPL>(a, rsh, nu_stage(a.S), P, (int)(local / tiles), (int)(local % tiles) * 256 * PPL);
    }
}

__global__ void k_reduce_abar(const int32_t *count, const float2 *part, const float *tpart, int nvs, int cap,
                              float2 *abar, float *tdbar) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= count[0]) return;
    float r = 0.0f, i = 0.0f, t = 0.0f;
    for (int s = 0; s < nvs; s++) {
        float2 x = part[(size_t)s * cap + p];
        r += x.x;
        i += x.y;
        t += tpart[(size_t)s * cap + p];
    }
    abar[p] = make_float2(r, i);
    tdbar[p] = t;
}

struct GeomArgs {
    const float *verts;
    const int32_t *faces;
    const uint16_t *mat_id;
    const int32_t *tri;
    int32_t R;
    int32_t nf;
    MatTable mt;
    int32_t any_fresnel;
    RadarDev rd;
    GridDev g;
    ChirpDev ch;
    const int32_t *ray_first;
    const uint8_t *flags;
    int32_t drop, exit_only;
    const float2 *abar;
    const float *tau_bar;   // [V][cap]
    const float *tdbar;     // [cap] dL/d taudot
    int32_t cap;
    float *grad;            // [nv][3]
    float *g_mats;          // [n_mats][2] or NULL
    float *g_radar;         // [6] or NULL
    float *g_rot;           // [9] or NULL
    float *g_atten;         // [1] or NULL
    int32_t attached;       // 1: first hits follow their triangle (Eqs. 6-7)
    float txl[SBR_MAX_TX][3];   // antenna positions in the radar frame
    float rxl[SBR_MAX_RX][3];
};

__device__ __forceinline__ float3 f3(float x, float y, float z) { return make_float3(x, y, z); }
__device__ __forceinline__ float3 operator+(float3 a, float3 b) { return f3(a.x + b.x, a.y + b.y, a.z + b.z); }
__device__ __forceinline__ float3 operator-(float3 a, float3 b) { return f3(a.x - b.x, a.y - b.y, a.z - b.z); }
__device__ __forceinline__ float3 operator*(float s, float3 a) { return f3(s * a.x, s * a.y, s * a.z); }
__device__ __forceinline__ float dot3(float3 a, float3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ float3 cross3(float3 a, float3 b) {
    return f3(a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x);
}
__device__ __forceinline__ float len3(float3 a) { return sqrtf(dot3(a, a)); }
__device__ __forceinline__ float3 vload3(const float *v, int i) { return f3(v[3 * i], v[3 * i + 1], v[3 * i + 2]); }

__device__ __forceinline__ void atomic_add3(float *g, int vi, float3 x) {
    atomicAdd(&g[3 * vi], x.x);
    atomicAdd(&g[3 * vi + 1], x.y);
    atomicAdd(&g[3 * vi + 2], x.z);
}

// Sum of x over the run of consecutive lanes that share `key` (segmented
// inclusive scan, lanes in order); valid in the last lane of each run.
__device__ __forceinline__ float seg_sum(float x, int lane, int s0) {
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        float y = __shfl_up(x, off);
        if (lane - off >= s0) x += y;
    }
    return x;
}

// Per ray: single-precision forward recompute of its bounces from the face
// ids (nothing is stored per path), path adjoints -> dL/dx_j and dL/dcos_j,
// then one reverse sweep through x = o + t d, t = N.(a - o)/(N.d), the
// specular reflection, the normalisation and the cross product, Fresnel
// coefficients included.  Rays of a wavefront are consecutive in a grid row,
// so neighbouring lanes often hit the same face: their vertex gradients are
// summed over runs of equal face ids first and added by one atomic per run.
template <int K>
__global__ __launch_bounds__(256) void k_geom_adj(GeomArgs a) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    const int lane = threadIdx.x & 63;
    int first = 0, n = 0;               // n: bounces to recompute (last returning one + 1)
    uint32_t mask = 0;                  // bounces that return a path
    if (r < a.R) {
        first = a.ray_first[r];
        mask = ray_path_mask(a.tri, a.flags, (size_t)a.R, (size_t)r, a.g.K, a.nf, a.drop != 0, a.exit_only != 0, &n);
    }
    if (__ballot(n > 0) == 0) return;   // uniform over the wavefront
    const int ix = r % a.g.nx, iy = r / a.g.nx;
    double d0[3], dl[3], dwd;
    grid_dir_local(a.g, ix, iy, dl, &dwd);
    for (int i = 0; i < 3; i++) d0[i] = a.rd.rot[3 * i] * dl[0] + a.rd.rot[3 * i + 1] * dl[1] + a.rd.rot[3 * i + 2] * dl[2];
    const float dw = (float)dwd;
    const float3 O = f3((float)a.rd.o[0], (float)a.rd.o[1], (float)a.rd.o[2]);
    // ---- forward recompute, cached per bounce
    float3 X[K], D[K], VA[K], E1[K], E2[K];
    float T[K], CI[K], SG[K], LC[K];
    float2 RC[K], DRC[K], DEPS[K];
    int F[K], MAT[K];
    float3 dir = f3((float)d0[0], (float)d0[1], (float)d0[2]);
    float3 o = O;
    float L = 0.0f;
#pragma unroll
    for (int k = 0; k < K; k++) {
        F[k] = -1;
        MAT[k] = -1;
        if (k < n) {
            const int f = a.tri[(size_t)k * a.R + r];
            const float3 va = vload3(a.verts, a.faces[3 * f]);
            const float3 e1 = vload3(a.verts, a.faces[3 * f + 1]) - va;
            const float3 e2 = vload3(a.verts, a.faces[3 * f + 2]) - va;
            const float3 N = cross3(e1, e2);
            const float den = dot3(N, dir);
            const float t = dot3(N, va - o) / den;
            const float3 x = o + t * dir;
            L += len3(x - o);
            const float nl = len3(N);
            const float dn = den / nl;
            X[k] = x;
            D[k] = dir;
            VA[k] = va;
            E1[k] = e1;
            E2[k] = e2;
            T[k] = t;
            LC[k] = L;
            F[k] = f;
            CI[k] = fabsf(dn);
            SG[k] = dn >= 0.0f ? 1.0f : -1.0f;
            cd rc = {-1.0, 0.0}, drc = {0.0, 0.0}, de = {0.0, 0.0};
            const int mi = a.mat_id ? (int)a.mat_id[f] : 0;
            if (a.any_fresnel) {
                reflect_coef(a.mt, mi, a.ch.fc, (double)CI[k], rc, drc);
                if (a.g_mats) de = reflect_deps(a.mt, mi, a.ch.fc, (double)CI[k]);
                if (mi < a.mt.n && a.mt.mode[mi] != 0) MAT[k] = mi;
            }
            RC[k] = make_float2((float)rc.re, (float)rc.im);
            DRC[k] = make_float2((float)drc.re, (float)drc.im);
            DEPS[k] = make_float2((float)de.re, (float)de.im);
            dir = dir - (2.0f * dn / nl) * N;
            o = x;
        }
    }
    // ---- path adjoints -> dL/dx_j, dL/dcos_j
    float3 xb[K];
    float cib[K];
    float2 gm[K];                           // dL/d (eps_r, sigma) of the material at bounce j
    float3 go = f3(0.f, 0.f, 0.f);          // dL/d radar origin
    float3 gu = f3(0.f, 0.f, 0.f);          // dL/d scene velocity
    float3 gd0 = f3(0.f, 0.f, 0.f);         // dL/d first ray direction (Doppler part)
    float gR[9];                            // dL/d rot from the antenna positions
#pragma unroll
    for (int q = 0; q < 9; q++) gR[q] = 0.0f;
    const bool want_rot = a.g_rot != nullptr;
    float wJ = 0.0f;                        // sum over the ray's paths of Re(conj(Abar) A)
    const float atn = (float)a.rd.atten;
    float ga_atn = 0.0f;                    // dL/d attenuation
    // directional gains F(d_0) G(x_k - o) of Eq. 1, cos^n about the boresight zb
    const float ntg = (float)a.rd.n_tg, nrg = (float)a.rd.n_rg;
    const float3 ZB = f3((float)a.rd.rot[2], (float)a.rd.rot[5], (float)a.rd.rot[8]);
    const float3 D0 = f3((float)d0[0], (float)d0[1], (float)d0[2]);
    const float ctx = dot3(D0, ZB);
    const float Fg = ntg == 0.0f ? 1.0f : (ctx > 0.0f ? __powf(ctx, ntg) : 0.0f);
    float3 gZ = f3(0.f, 0.f, 0.f);          // dL/d boresight vector (world)
    const float3 U = f3((float)a.rd.vel[0], (float)a.rd.vel[1], (float)a.rd.vel[2]);
#pragma unroll
    for (int k = 0; k < K; k++) {
        xb[k] = f3(0.f, 0.f, 0.f);
        cib[k] = 0.0f;
        gm[k] = make_float2(0.f, 0.f);
    }
    const float inv_we0 = (float)(1.0 / (2.0 * kPi * a.ch.fc * kEps0));
    const int ntx = a.rd.n_tx, nrx = a.rd.n_rx;
    const float ic0 = (float)(1.0 / kC0);
#pragma unroll
    for (int k = 0; k < K; k++) {
        if ((mask >> k) & 1u) {
            const int p = first + __popc(mask & ((1u << k) - 1u));
            const float2 ab = a.abar[p];
            float2 prod = make_float2(1.0f, 0.0f);
#pragma unroll
            for (int j = 0; j <= k; j++)
                prod = make_float2(prod.x * RC[j].x - prod.y * RC[j].y, prod.x * RC[j].y + prod.y * RC[j].x);
            const float3 qk = X[k] - O;
            const float Rk = len3(qk);
            const float qz = dot3(qk, ZB);
            const float Gg = nrg == 0.0f ? 1.0f : (qz > 0.0f ? __powf(qz / Rk, nrg) : 0.0f);
            // A = dw prod ci_k exp(-a (L + R)) F G / (L R);  u = Re(conj(Abar) A / ci_k)
            const float sc = dw / (LC[k] * Rk) * __expf(-atn * (LC[k] + Rk)) * (Fg * Gg);
            const float u = sc * (ab.x * prod.x + ab.y * prod.y);
            const float gk = u * CI[k];
            wJ += gk;                               // Re(conj(Abar) A): dL/d log(cell weight)
            cib[k] += u;
            const float Lb = -gk / LC[k] - atn * gk, Rb = -gk / Rk - atn * gk;
            ga_atn -= gk * (LC[k] + Rk);            // d A / d a = -(L + R) A
            if (nrg != 0.0f && qz > 0.0f) {         // log G = n (log(q.zb) - log |q|)
                const float3 t = nrg * ((1.0f / qz) * ZB - (1.0f / (Rk * Rk)) * qk);
                xb[k] = xb[k] + gk * t;
                go = go - gk * t;
                gZ = gZ + (gk * nrg / qz) * qk;
            }
            if (ntg != 0.0f && ctx > 0.0f) {        // log F = n log(d_0.zb)
                gd0 = gd0 + (gk * ntg / ctx) * ZB;
                gZ = gZ + (gk * ntg / ctx) * D0;
            }
            if (a.any_fresnel) {
#pragma unroll
                for (int j = 0; j <= k; j++) {
                    float2 ex = make_float2(sc * CI[k], 0.0f);
#pragma unroll
                    for (int i = 0; i <= k; i++)
                        if (i != j) ex = make_float2(ex.x * RC[i].x - ex.y * RC[i].y, ex.x * RC[i].y + ex.y * RC[i].x);
                    const float2 dA = make_float2(ex.x * DRC[j].x - ex.y * DRC[j].y, ex.x * DRC[j].y + ex.y * DRC[j].x);
                    cib[j] += ab.x * dA.x + ab.y * dA.y;
                    if (a.g_mats) {
                        // eps_c = eps_r - j sigma / (omega eps_0): d/deps_r = d/deps_c,
                        // d/dsigma = -j / (omega eps_0) d/deps_c
                        const float2 W = make_float2(ex.x * DEPS[j].x - ex.y * DEPS[j].y,
                                                     ex.x * DEPS[j].y + ex.y * DEPS[j].x);
                        gm[j].x += ab.x * W.x + ab.y * W.y;
                        gm[j].y += (ab.x * W.y - ab.y * W.x) * inv_we0;
                    }
                }
            }
            float3 prv = O;
#pragma unroll
            for (int j = 0; j <= k; j++) {
                const float3 sg = X[j] - prv;
                const float3 uj = (Lb / len3(sg)) * sg;
                xb[j] = xb[j] + uj;
                if (j > 0) xb[j - 1] = xb[j - 1] - uj;
                else go = go - uj;                  // first segment starts at the origin
                prv = X[j];
            }
            xb[k] = xb[k] + (Rb / Rk) * (X[k] - O);
            // the TX leg of antenna (t, m) moves with the sum over m of its
            // delay adjoints, the RX leg with the sum over t; both sums are
            // formed inside their loops (no runtime-indexed arrays)
            const float *tbp = a.tau_bar + p;
            float Tt = 0.0f;
            for (int t = 0; t < ntx; t++) {
                float ts = 0.0f;
                for (int m = 0; m < nrx; m++) ts += tbp[(size_t)(t * nrx + m) * a.cap];
                Tt += ts;
                const float3 q = X[0] - f3((float)a.rd.tx[t][0], (float)a.rd.tx[t][1], (float)a.rd.tx[t][2]);
                const float3 gq = (ts * ic0 / len3(q)) * q;
                xb[0] = xb[0] + gq;
                go = go - gq;                       // TX positions move with the origin
                if (want_rot) {                     // tx_world = origin + rot tx_local
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        gR[c] -= gq.x * a.txl[t][c];
                        gR[3 + c] -= gq.y * a.txl[t][c];
                        gR[6 + c] -= gq.z * a.txl[t][c];
                    }
                }
            }
            for (int m = 0; m < nrx; m++) {
                float rs = 0.0f;
                for (int t = 0; t < ntx; t++) rs += tbp[(size_t)(t * nrx + m) * a.cap];
                const float3 q = X[k] - f3((float)a.rd.rx[m][0], (float)a.rd.rx[m][1], (float)a.rd.rx[m][2]);
                const float3 gq = (rs * ic0 / len3(q)) * q;
                xb[k] = xb[k] + gq;
                go = go - gq;                       // RX positions move with the origin
                if (want_rot) {
#pragma unroll
                    for (int c = 0; c < 3; c++) {
                        gR[c] -= gq.x * a.rxl[m][c];
                        gR[3 + c] -= gq.y * a.rxl[m][c];
                        gR[6 + c] -= gq.z * a.rxl[m][c];
                    }
                }
            }
            go = go - (Rb / Rk) * (X[k] - O);        // R_k = |x_k - origin|
            // taudot = 2 (u . d_1) / c
            const float tdq = a.tdbar[p] * 2.0f * ic0;
            gu = gu + tdq * f3((float)d0[0], (float)d0[1], (float)d0[2]);
            gd0 = gd0 + tdq * U;
#pragma unroll
            for (int j = 1; j <= k; j++) {
                const float3 sg = X[j] - X[j - 1];
                const float3 uj = (Tt * ic0 / len3(sg)) * sg;
                xb[j] = xb[j] + uj;
                xb[j - 1] = xb[j - 1] - uj;
            }
        }
    }
    // ---- reverse sweep over bounces
    float3 dnext = f3(0.f, 0.f, 0.f);   // dL/d d_{j+1}
#pragma unroll
    for (int j = K - 1; j >= 0; j--) {
        const bool act = j < n;
        float3 ga = f3(0.f, 0.f, 0.f), gb = ga, gc = ga;
        if (act && j == 0 && a.attached) {
            // Eqs. 6-7 with T attached to the first hit: x_0 = a + b1 e1 + b2 e2 at
            // fixed (b1, b2), d_0 = (x_0 - o) / |x_0 - o|, cell weight times
            // D / D_0 with D = |N . (x_0 - o)| / |x_0 - o|^3
            const float3 e1 = E1[0], e2 = E2[0];
            const float3 N = cross3(e1, e2);
            const float nl = len3(N);
            const float3 nh = (1.0f / nl) * N;
            const float3 d = D[0];
            const float dn = dot3(d, nh);
            const float3 q = X[0] - O;
            const float r0 = len3(q);
            const float nn = dot3(N, N);
            const float3 w0 = X[0] - VA[0];
            const float b1 = dot3(cross3(w0, e2), N) / nn, b2 = dot3(cross3(e1, w0), N) / nn;
            float3 db = (cib[0] * SG[0]) * nh + gd0;   // cos_0 = |d_0 . n|, Doppler 2 u.d_0 / c
            float3 nhb = (cib[0] * SG[0]) * d;
            const float ndn = dot3(nh, dnext);          // d_1 = d_0 - 2 (d_0.n) n
            db = db + dnext - (2.0f * ndn) * nh;
            nhb = nhb - 2.0f * (dn * dnext + ndn * d);
            const float3 dq = (1.0f / r0) * (db - dot3(db, d) * d);
            const float sN = dot3(N, q);
            const float3 lj = wJ * ((1.0f / sN) * N - (3.0f / (r0 * r0)) * q);
            const float3 xb0 = xb[0] + dq + lj;
            go = go - dq - lj;
            const float3 Nb = (wJ / sN) * q + (1.0f / nl) * (nhb - dot3(nhb, nh) * nh);
            const float3 gbN = cross3(e2, Nb), gcN = cross3(Nb, e1);
            ga = (1.0f - b1 - b2) * xb0 - gbN - gcN;
            gb = b1 * xb0 + gbN;
            gc = b2 * xb0 + gcN;
            dnext = f3(0.f, 0.f, 0.f);                  // d_0 no longer depends on the grid
            gd0 = f3(0.f, 0.f, 0.f);
        } else if (act) {
            const float3 e1 = E1[j], e2 = E2[j];
            const float3 N = cross3(e1, e2);
            const float nl = len3(N);
            const float3 nh = (1.0f / nl) * N;
            const float3 d = D[j];
            const float dn = dot3(d, nh);
            const float t = T[j];
            float3 ob = xb[j];                     // x = o + t d
            const float tbar = dot3(xb[j], d);
            float3 db = t * xb[j];
            float3 nhb = (cib[j] * SG[j]) * d;      // cos = |d . n|
            db = db + (cib[j] * SG[j]) * nh;
            const float ndn = dot3(nh, dnext);      // d_{j+1} = d - 2 (d.n) n
            db = db + dnext - (2.0f * ndn) * nh;
            nhb = nhb - 2.0f * (dn * dnext + ndn * d);
            const float den = dot3(N, d);           // t = N.(a - o) / (N.d)
            const float w = tbar / den;
            float3 Nb = w * (VA[j] - X[j]);
            ga = w * N;
            ob = ob - w * N;
            db = db - (w * t) * N;
            Nb = Nb + (1.0f / nl) * (nhb - dot3(nhb, nh) * nh);   // n = N / |N|
            gb = cross3(e2, Nb);                    // N = e1 x e2
            gc = cross3(Nb, e1);
            ga = ga - gb - gc;
            if (j > 0) xb[j - 1] = xb[j - 1] + ob;
            else go = go + ob;                      // rays start at the origin
            dnext = db;
        }
        // sum over runs of lanes that hit the same face, one atomic per run
        const int key = act ? F[j] : -1;
        const int kprev = __shfl_up(key, 1);
        int s0 = (lane == 0 || kprev != key) ? lane : 0;
#pragma unroll
        for (int off = 1; off < 64; off <<= 1) s0 = max(s0, __shfl_up(s0, off));
        const int knext = __shfl_down(key, 1);
        const bool tail = act && (lane == 63 || knext != key);
        float v9[9] = {ga.x, ga.y, ga.z, gb.x, gb.y, gb.z, gc.x, gc.y, gc.z};
#pragma unroll
        for (int q = 0; q < 9; q++) v9[q] = seg_sum(v9[q], lane, s0);
        if (tail) {
            const int f = F[j];
            atomic_add3(a.grad, a.faces[3 * f], f3(v9[0], v9[1], v9[2]));
            atomic_add3(a.grad, a.faces[3 * f + 1], f3(v9[3], v9[4], v9[5]));
            atomic_add3(a.grad, a.faces[3 * f + 2], f3(v9[6], v9[7], v9[8]));
        }
        if (a.g_mats) {
            // one wavefront sum per distinct material of this bounce
            const int km = act ? MAT[j] : -1;
            uint64_t pending = __ballot(km >= 0);
            while (pending) {
                const int leader = __ffsll((unsigned long long)pending) - 1;
                const int m = __shfl(km, leader);
                const bool mine = km == m;
                float e0 = mine ? gm[j].x : 0.0f, e1 = mine ? gm[j].y : 0.0f;
                for (int off = 32; off >= 1; off >>= 1) {
                    e0 += __shfl_xor(e0, off);
                    e1 += __shfl_xor(e1, off);
                }
                if (lane == leader) {
                    atomicAdd(&a.g_mats[2 * m], e0);
                    atomicAdd(&a.g_mats[2 * m + 1], e1);
                }
                pending &= ~__ballot(mine);
            }
        }
    }
    if (a.g_radar) {
        float v6[6] = {go.x, go.y, go.z, gu.x, gu.y, gu.z};
#pragma unroll
        for (int q = 0; q < 6; q++) {
            for (int off = 32; off >= 1; off >>= 1) v6[q] += __shfl_xor(v6[q], off);
            if (lane == 0) atomicAdd(&a.g_radar[q], v6[q]);
        }
    }
    if (a.g_atten) {
        float v = ga_atn;
        for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off);
        if (lane == 0) atomicAdd(a.g_atten, v);
    }
    if (want_rot) {
        // d_0 = rot d_local: dL/drot += (dL/dd_0) d_local^T, where dL/dd_0 is
        // what the reverse sweep left for the first segment plus the Doppler part
        const float3 g0 = dnext + gd0;
        const float l0 = (float)dl[0], l1 = (float)dl[1], l2 = (float)dl[2];
        // zb = rot e_z: the gains add dL/dzb to the third column
        float v9[9] = {gR[0] + g0.x * l0, gR[1] + g0.x * l1, gR[2] + g0.x * l2 + gZ.x,
                       gR[3] + g0.y * l0, gR[4] + g0.y * l1, gR[5] + g0.y * l2 + gZ.y,
                       gR[6] + g0.z * l0, gR[7] + g0.z * l1, gR[8] + g0.z * l2 + gZ.z};
#pragma unroll
        for (int q = 0; q < 9; q++) {
            for (int off = 32; off >= 1; off >>= 1) v9[q] += __shfl_xor(v9[q], off);
            if (lane == 0) atomicAdd(&a.g_rot[q], v9[q]);
        }
    }
}

}  // namespace

struct BackPlan {
    int nvs, v_per;
};

// One antenna per block row (grid.y) unless the per-row partial sums of Abar
// and taudot_bar (12 bytes per path and row) would pass 4 GiB: the number of
// live paths is only known on the device, and splitting over antennas keeps
// the launch full when few of the `cap` slots hold paths.
static BackPlan back_plan(long long cap, int V) {
    const long long budget = 4LL << 30;
    int v_per = 1;
    while (v_per < V && (long long)((V + v_per - 1) / v_per) * cap * 12 > budget) v_per++;
    const int nvs = (V + v_per - 1) / v_per;
    return {nvs, v_per};
}

// Whether a request's adjoint sums run as the non-uniform FFT form.
static bool use_nu(int32_t S, int32_t flags) { return nu_size(S) && !(flags & SBR_DIRECT_SUMS); }

// Adjoint buffers after the path stage: tau_bar, Abar and taudot_bar partials
// and sums, then (for chirps of kNuMinS .. kNuMaxS samples, whatever the
// flags) the 1/Psi table and the non-uniform FFT rows.
struct BackExtra {
    float *tau_bar;
    float2 *part, *abar;
    float *tpart, *tdbar;
    float *corr;
    float4 *rows;
    size_t bytes;
};

static BackExtra back_extra(void *buf, int32_t R, int32_t K, int32_t V, int32_t C, int32_t S) {
    const long long cap = (long long)R * K;
    const BackPlan bp = back_plan(cap, V);
    Carver cv(buf);
    BackExtra e;
    e.tau_bar = cv.take<float>((size_t)V * cap);
    e.part = cv.take<float2>((size_t)bp.nvs * cap);
    e.abar = cv.take<float2>(cap);
    e.tpart = cv.take<float>((size_t)bp.nvs * cap);
    e.tdbar = cv.take<float>(cap);
    e.corr = nullptr;
    e.rows = nullptr;
    if (nu_size(S)) {
        e.corr = cv.take<float>((size_t)S);
        e.rows = cv.take<float4>((size_t)V * C * nu_row_len(S));
    }
    e.bytes = align_up(cv.off, 256);
    return e;
}

size_t backward_extra_bytes(int32_t R, int32_t K, int32_t V, int32_t C, int32_t S) {
    return back_extra(nullptr, R, K, V, C, S).bytes;
}

// Device table of a batched adjoint: the requests' arguments, their first
// work items and the work counter.
struct AdjTable {
    AdjArgs *args;
    uint32_t *item_first;
    uint32_t *queue;
    int32_t *row_first;   // first G row of each request of the non-uniform FFT form
};

static AdjTable adj_table(void *buf, int n, size_t *bytes) {
    Carver cv(buf);
    AdjTable t;
    t.args = cv.take<AdjArgs>(n);
    t.item_first = cv.take<uint32_t>((size_t)n + 1);
    t.queue = cv.take<uint32_t>(64);
    t.row_first = cv.take<int32_t>((size_t)n + 1);
    if (bytes) *bytes = align_up(cv.off, 256);
    return t;
}

size_t adj_table_bytes(int n) {
    size_t b = 0;
    adj_table(nullptr, n, &b);
    return b;
}

// G rows per LDS stage of a request with S samples, with the 16-byte
// work-item slot after them, within 64 KiB of LDS per block.
static int adj_rows(int Sp) { return std::max(1, std::min<int>(kAdjRowsMax, (65536 - 16) / (int)(sizeof(float2) * Sp))); }

int launch_backward_batch(const BackwardReq *reqs, int n, void *table, hipStream_t s) {
    if (n <= 0) return SBR_OK;
    // requests of the non-uniform FFT form first, then those of the direct one
    std::vector<int> order;
    for (int r = 0; r < n; r++)
        if (use_nu(reqs[r].cd.S, reqs[r].flags)) order.push_back(r);
    const int n_nu = (int)order.size();
    for (int r = 0; r < n; r++)
        if (!use_nu(reqs[r].cd.S, reqs[r].flags)) order.push_back(r);
    std::vector<AdjArgs> aa(n);
    std::vector<GeomArgs> gg(n);
    size_t lds_f2 = 0;   // float2 words of the largest G-row stage
    long long items_nu = 0, items_direct = 0;
    for (int r = 0; r < n; r++) {
        const BackwardReq &q = reqs[order[r]];
        const RadarDev &rd = q.rd;
        const int V = rd.n_tx * rd.n_rx;
        const long long cap = q.st.rec.cap;
        const bool nu = r < n_nu;
        BackPlan bp = back_plan(cap, V);
        const BackExtra e = back_extra(q.extra, q.gd.nx * q.gd.ny, q.gd.K, V, q.cd.C, q.cd.S);
        AdjArgs &a = aa[r];
        a.count = q.st.count;
        a.rec = q.st.rec;
        a.G = q.G;
        a.V = V;
        a.C = q.cd.C;
        a.S = q.cd.S;
        a.v_per = bp.v_per;
        a.nvs = bp.nvs;
        a.ppl = nu ? kNuPPL : kAdjPPL;
        a.fcf = (float)q.cd.fc;
        a.sl_fs = (float)(q.cd.slope / q.cd.fs);
        a.tc = (float)q.cd.tc;
        a.tau_bar = e.tau_bar;
        a.abar_part = e.part;
        a.tdb_part = e.tpart;
        a.nu_rows = nu ? e.rows : nullptr;
        a.nu_corr = nu ? e.corr : nullptr;
        a.Sp = (q.cd.S + 7) / 8 * 8;
        a.rows = adj_rows(a.Sp);
        if (nu) {
            items_nu += (cap + 256 * kNuPPL - 1) / (256 * kNuPPL) * bp.nvs;
        } else {
            lds_f2 = std::max(lds_f2, (size_t)a.rows * a.Sp);
            items_direct += (cap + 256 * kAdjPPL - 1) / (256 * kAdjPPL) * bp.nvs;
        }
        GeomArgs &g = gg[r];
        const sbr_mesh *m = q.mesh;
        g.verts = m->verts;
        g.faces = m->faces;
        g.mat_id = m->mat_id;
        g.tri = q.hits->tri;
        g.R = q.gd.nx * q.gd.ny;
        g.nf = m->nf;
        g.mt = q.mt;
        g.any_fresnel = 0;
        for (int i = 0; i < q.mt.n; i++)
            if (q.mt.mode[i] != 0) g.any_fresnel = 1;
        g.rd = rd;
        g.g = q.gd;
        g.ch = q.cd;
        g.ray_first = q.st.ray_first;
        g.flags = q.hits->flags;
        g.drop = (q.flags & SBR_DROP_FLAGGED) ? 1 : 0;
        g.exit_only = (q.flags & SBR_EXIT_ONLY) ? 1 : 0;
        g.abar = e.abar;
        g.tau_bar = e.tau_bar;
        g.tdbar = e.tdbar;
        g.cap = (int32_t)cap;
        g.grad = q.grad;
        g.g_mats = q.params ? q.params->materials : nullptr;
        g.g_radar = q.params ? q.params->radar : nullptr;
        g.g_rot = q.params ? q.params->rot : nullptr;
        g.g_atten = q.params ? q.params->attenuation : nullptr;
        g.attached = (q.flags & SBR_ATTACHED) ? 1 : 0;
        for (int t = 0; t < SBR_MAX_TX; t++)
            for (int c = 0; c < 3; c++) g.txl[t][c] = t < q.radar->n_tx ? (float)q.radar->tx[t][c] : 0.0f;
        for (int k = 0; k < SBR_MAX_RX; k++)
            for (int c = 0; c < 3; c++) g.rxl[k][c] = k < q.radar->n_rx ? (float)q.radar->rx[k][c] : 0.0f;
    }
    AdjTable t = adj_table(table, n, nullptr);
    int rc = put_table(t.args, aa.data(), sizeof(AdjArgs) * n, s);
    if (rc) return rc;
    hipLaunchKernelGGL(k_adj_items, dim3(1), dim3(1024), 0, s, t.args, n, t.item_first, t.queue);
    SBR_LAUNCHED();
    if (n_nu > 0) {
        // all requests of this form: 1/Psi tables, then the row transforms
        std::vector<int32_t> row_first(1, 0);
        int max_s = 0;
        for (int r = 0; r < n_nu; r++) {
            const long long rows = (long long)aa[r].V * aa[r].C;
            if (row_first.back() + rows > 0x7fffffffLL) {
                set_error("batched backward: more than 2^31 gradient rows in one launch");
                return SBR_E_ARG;
            }
            row_first.push_back(row_first.back() + (int32_t)rows);
            max_s = std::max(max_s, (int)aa[r].S);
        }
        if ((rc = put_table(t.row_first, row_first.data(), sizeof(int32_t) * (n_nu + 1), s))) return rc;
        ProfScope ps(kProfSynthAdj, s);
        hipLaunchKernelGGL(k_nu_corr_adj, dim3((unsigned)((max_s + 255) / 256), (unsigned)n_nu), dim3(256), 0, s,
                           t.args);
        const size_t lds_rows = sizeof(float4) * 2 * max_s + sizeof(float2) * 2 * max_s;   // sequence + twiddles
        hipLaunchKernelGGL(k_nu_rows, dim3((unsigned)row_first.back()), dim3(256), lds_rows, s, t.args, t.row_first,
                           n_nu);
        SBR_LAUNCHED();
        size_t slot = 0;   // float4 words of the largest row stage
        for (int r = 0; r < n_nu; r++) slot = std::max(slot, (size_t)nu_stage(aa[r].S) * nu_row_len(aa[r].S));
        const size_t lds = sizeof(float4) * slot + 16;
        dim3 grid((unsigned)std::max(1LL, std::min<long long>(items_nu, resident_blocks((const void *)k_synth_adj_nu<kNuPPL>,
                                                                                         256, lds, 256 * 2))));
        ProfScope pk(kProfNuTaps, s);
        hipLaunchKernelGGL(k_synth_adj_nu<kNuPPL>, grid, dim3(256), lds, s, t.args, t.item_first, 0, n_nu, t.queue,
                           (int)slot);
    }
    SBR_LAUNCHED();
    if (n_nu < n) {
        const size_t lds = sizeof(float2) * lds_f2 + 16;
        // one device-full of blocks, or fewer if the path slots cannot fill it
        dim3 grid((unsigned)std::max(1LL, std::min<long long>(items_direct, resident_blocks((const void *)k_synth_adj<kAdjPPL>,
                                                                                             256, lds, 256 * 2))));
        ProfScope ps(kProfSynthAdj, s);
        hipLaunchKernelGGL(k_synth_adj<kAdjPPL>, grid, dim3(256), lds, s, t.args, t.item_first, n_nu, n,
                           t.queue + kAdjQueueDirect, (int)lds_f2);
    }
    SBR_LAUNCHED();
    for (int r = 0; r < n; r++) {
        const AdjArgs &a = aa[r];
        const GeomArgs &g = gg[r];
        const long long cap = a.rec.cap;
        hipLaunchKernelGGL(k_reduce_abar, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, a.count, a.abar_part,
                           a.tdb_part, a.nvs, (int)cap, const_cast<float2 *>(g.abar), const_cast<float *>(g.tdbar));
        SBR_LAUNCHED();
        if (g.R == 0 || g.nf == 0) continue;
        dim3 gb((unsigned)((g.R + 255) / 256));
        switch (g.g.K) {
        case 1: hipLaunchKernelGGL(k_geom_adj<1>, gb, dim3(256), 0, s, g); break;
        case 2: hipLaunchKernelGGL(k_geom_adj<2>, gb, dim3(256), 0, s, g); break;
        case 3: hipLaunchKernelGGL(k_geom_adj<3>, gb, dim3(256), 0, s, g); break;
        case 4: hipLaunchKernelGGL(k_geom_adj<4>, gb, dim3(256), 0, s, g); break;
        case 5: hipLaunchKernelGGL(k_geom_adj<5>, gb, dim3(256), 0, s, g); break;
        case 6: hipLaunchKernelGGL(k_geom_adj<6>, gb, dim3(256), 0, s, g); break;
        case 7: hipLaunchKernelGGL(k_geom_adj<7>, gb, dim3(256), 0, s, g); break;
        default: hipLaunchKernelGGL(k_geom_adj<8>, gb, dim3(256), 0, s, g); break;
        }
        SBR_LAUNCHED();
    }
    return SBR_OK;
}

}  // namespace sbr
