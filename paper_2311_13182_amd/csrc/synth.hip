// Path stage (FP64 refinement of every hit into I^t / I^s, compacted in
// ray-major order) and the IF synthesis of Eq. (8).
#include <cmath>
#include <utility>
#include <vector>

#include "sbr_internal.h"
#include "sbr_device.h"

namespace sbr {

namespace {

struct PathArgs {
    const float *verts;
    const int32_t *faces;
    const uint16_t *mat_id;
    const int32_t *tri;
    const uint8_t *flags;
    int32_t drop;
    int32_t exit_only;
    int32_t R;
    int32_t nf;
    MatTable mt;
    RadarDev rd;
    GridDev g;
    ChirpDev ch;
    PathStage st;
};

__device__ __forceinline__ uint32_t ray_mask(const PathArgs &a, size_t r, int *nb) {
    return ray_path_mask(a.tri, a.flags, (size_t)a.R, r, a.g.K, a.nf, a.drop != 0, a.exit_only != 0, nb);
}

__device__ __forceinline__ int block_sum(int x, int *sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int off = 32; off >= 1; off >>= 1) x += __shfl_xor(x, off);
    if (lane == 0) sh[w] = x;
    __syncthreads();
    int t = 0;
    for (int i = 0; i < (int)(blockDim.x >> 6); i++) t += sh[i];
    __syncthreads();
    return t;
}

// inclusive prefix within the block (wave scan + wave offsets)
__device__ __forceinline__ int block_incl_scan(int x, int *sh) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    for (int off = 1; off < 64; off <<= 1) {
        int y = __shfl_up(x, off);
        if (lane >= off) x += y;
    }
    if (lane == 63) sh[w] = x;
    __syncthreads();
    int add = 0;
    for (int i = 0; i < w; i++) add += sh[i];
    __syncthreads();
    return x + add;
}

__global__ __launch_bounds__(kPathBlock) void k_path_count(PathArgs a) {
    __shared__ int sh[kPathBlock / 64];
    size_t r = (size_t)blockIdx.x * kPathBlock + threadIdx.x;
    int nb;
    int n = r < (size_t)a.R ? __popc(ray_mask(a, r, &nb)) : 0;
    int t = block_sum(n, sh);
    if (threadIdx.x == 0) a.st.blk[blockIdx.x] = t;
}

__global__ __launch_bounds__(1024) void k_path_scan(PathArgs a) {
    __shared__ int part[1024];
    const int t = threadIdx.x, nb = a.st.nblk;
    int chunk = (nb + 1023) / 1024;
    int b = t * chunk, e = min(nb, b + chunk);
    int s = 0;
    for (int i = b; i < e; i++) s += a.st.blk[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        int v = t >= off ? part[t - off] : 0;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    int run = part[t] - s;
    for (int i = b; i < e; i++) {
        int x = a.st.blk[i];
        a.st.blk[i] = run;
        run += x;
    }
    if (t == 1023) {
        a.st.count[0] = part[1023];
        a.st.ray_first[a.R] = part[1023];
    }
}

__device__ __forceinline__ double frac_d(double x) { return x - floor(x); }

__global__ __launch_bounds__(kPathBlock) void k_path_refine(PathArgs a) {
    __shared__ int sh[kPathBlock / 64];
    const size_t r = (size_t)blockIdx.x * kPathBlock + threadIdx.x;
    const bool act = r < (size_t)a.R;
    int nb = 0;
    const uint32_t mask = act ? ray_mask(a, r, &nb) : 0u;
    const int n = __popc(mask);
    int incl = block_incl_scan(n, sh);
    if (!act) return;
    int p = a.st.blk[blockIdx.x] + incl - n;
    a.st.ray_first[r] = p;
    if (n == 0) return;
    const int ix = (int)(r % a.g.nx), iy = (int)(r / a.g.nx);
    double d[3], dw;
    grid_ray(a.g, a.rd, ix, iy, d, &dw);
    const double d0[3] = {d[0], d[1], d[2]};
    double o[3] = {a.rd.o[0], a.rd.o[1], a.rd.o[2]};
    const double taudot = 2.0 * (a.rd.vel[0] * d[0] + a.rd.vel[1] * d[1] + a.rd.vel[2] * d[2]) / kC0;
    const double beta = frac_d(a.ch.fc * a.ch.tc * taudot);
    const double epsd = a.ch.slope * a.ch.tc * taudot / a.ch.fs;
    double xp[3] = {o[0], o[1], o[2]}, x1[3] = {0, 0, 0};
    double L = 0.0, Lmid = 0.0;
    cd pr = {1.0, 0.0};
    const int cap = a.st.rec.cap;
    const int ntx = a.rd.n_tx, nrx = a.rd.n_rx;
    for (int k = 0; k < nb; k++) {
        const int f = a.tri[(size_t)k * a.R + r];
        double va[3], vb[3], vc[3];
        for (int i = 0; i < 3; i++) {
            va[i] = a.verts[3 * a.faces[3 * f] + i];
            vb[i] = a.verts[3 * a.faces[3 * f + 1] + i];
            vc[i] = a.verts[3 * a.faces[3 * f + 2] + i];
        }
        double e1[3] = {vb[0] - va[0], vb[1] - va[1], vb[2] - va[2]};
        double e2[3] = {vc[0] - va[0], vc[1] - va[1], vc[2] - va[2]};
        double N[3] = {e1[1] * e2[2] - e1[2] * e2[1], e1[2] * e2[0] - e1[0] * e2[2], e1[0] * e2[1] - e1[1] * e2[0]};
        double nd = N[0] * d[0] + N[1] * d[1] + N[2] * d[2];
        double th = (N[0] * (va[0] - o[0]) + N[1] * (va[1] - o[1]) + N[2] * (va[2] - o[2])) / nd;
        double x[3] = {o[0] + th * d[0], o[1] + th * d[1], o[2] + th * d[2]};
        double nl = sqrt(N[0] * N[0] + N[1] * N[1] + N[2] * N[2]);
        double dn = nd / nl;
        double ci = fabs(dn);
        cd rc, drc;
        reflect_coef(a.mt, a.mat_id ? (int)a.mat_id[f] : 0, a.ch.fc, ci, rc, drc);
        pr = cmul(pr, rc);
        double seg = sqrt((x[0] - xp[0]) * (x[0] - xp[0]) + (x[1] - xp[1]) * (x[1] - xp[1]) +
                          (x[2] - xp[2]) * (x[2] - xp[2]));
        L += seg;
        if (k == 0) {
            x1[0] = x[0];
            x1[1] = x[1];
            x1[2] = x[2];
        } else {
            Lmid += seg;
        }
        if (!((mask >> k) & 1u)) {            // this bounce returns no path
            for (int i = 0; i < 3; i++) {
                o[i] = x[i];
                xp[i] = x[i];
                d[i] = d[i] - 2.0 * dn * N[i] / nl;
            }
            continue;
        }
        double Rk = sqrt((x[0] - a.rd.o[0]) * (x[0] - a.rd.o[0]) + (x[1] - a.rd.o[1]) * (x[1] - a.rd.o[1]) +
                         (x[2] - a.rd.o[2]) * (x[2] - a.rd.o[2]));
        double sc = dw * ci / (L * Rk) * exp(-a.rd.atten * (L + Rk));
        if (a.rd.n_tg != 0.0 || a.rd.n_rg != 0.0) {   // F G of Eq. 1 about boresight
            const double zb[3] = {a.rd.rot[2], a.rd.rot[5], a.rd.rot[8]};
            const double ct = d0[0] * zb[0] + d0[1] * zb[1] + d0[2] * zb[2];
            const double cr = ((x[0] - a.rd.o[0]) * zb[0] + (x[1] - a.rd.o[1]) * zb[1] + (x[2] - a.rd.o[2]) * zb[2]) / Rk;
            sc *= pow(ct > 0.0 ? ct : 0.0, a.rd.n_tg) * pow(cr > 0.0 ? cr : 0.0, a.rd.n_rg);
        }
        a.st.rec.amp[p] = make_float2((float)(pr.re * sc), (float)(pr.im * sc));
        a.st.rec.beta[p] = (float)beta;
        a.st.rec.epsd[p] = (float)epsd;
        // one square root per (TX, RX) pair instead of per-antenna distance
        // arrays: a runtime-indexed array would live in per-thread stack memory
        for (int t = 0; t < ntx; t++) {
            const double dtx = sqrt((x1[0] - a.rd.tx[t][0]) * (x1[0] - a.rd.tx[t][0]) +
                                    (x1[1] - a.rd.tx[t][1]) * (x1[1] - a.rd.tx[t][1]) +
                                    (x1[2] - a.rd.tx[t][2]) * (x1[2] - a.rd.tx[t][2]));
            for (int m = 0; m < nrx; m++) {
                const double drx = sqrt((x[0] - a.rd.rx[m][0]) * (x[0] - a.rd.rx[m][0]) +
                                        (x[1] - a.rd.rx[m][1]) * (x[1] - a.rd.rx[m][1]) +
                                        (x[2] - a.rd.rx[m][2]) * (x[2] - a.rd.rx[m][2]));
                const double tau = (dtx + Lmid + drx) / kC0;
                const int v = t * nrx + m;
                a.st.rec.alpha[(size_t)v * cap + p] = (float)frac_d(a.ch.fc * tau);
                a.st.rec.gamma[(size_t)v * cap + p] = (float)(a.ch.slope * tau / a.ch.fs);
            }
        }
        p++;
        for (int i = 0; i < 3; i++) {
            o[i] = x[i];
            xp[i] = x[i];
            d[i] = d[i] - 2.0 * dn * N[i] / nl;
        }
    }
}

}  // namespace

PathStage carve_path_stage(Carver &cv, int32_t R, int32_t K, int32_t V) {
    PathStage st;
    st.nblk = (R + kPathBlock - 1) / kPathBlock;
    st.count = cv.take<int32_t>(64);
    st.ray_first = cv.take<int32_t>((size_t)R + 1);
    st.blk = cv.take<int32_t>(st.nblk);
    long long cap = (long long)R * K;
    st.rec.cap = (int32_t)cap;
    st.rec.V = V;
    st.rec.alpha = cv.take<float>((size_t)V * cap);
    st.rec.gamma = cv.take<float>((size_t)V * cap);
    st.rec.amp = cv.take<float2>(cap);
    st.rec.beta = cv.take<float>(cap);
    st.rec.epsd = cv.take<float>(cap);
    return st;
}

int launch_paths(const sbr_mesh *m, const MatTable &mt, const RadarDev &rd, const GridDev &gd,
                 const ChirpDev &cd, const sbr_hits *h, int32_t flags, const PathStage &st,
                 hipStream_t s) {
    PathArgs a;
    a.verts = m->verts;
    a.faces = m->faces;
    a.mat_id = m->mat_id;
    a.tri = h->tri;
    a.flags = h->flags;
    a.drop = (flags & SBR_DROP_FLAGGED) ? 1 : 0;
    a.exit_only = (flags & SBR_EXIT_ONLY) ? 1 : 0;
    a.R = gd.nx * gd.ny;
    a.nf = m->nf;
    a.mt = mt;
    a.rd = rd;
    a.g = gd;
    a.ch = cd;
    a.st = st;
    hipLaunchKernelGGL(k_path_count, dim3(st.nblk), dim3(kPathBlock), 0, s, a);
    hipLaunchKernelGGL(k_path_scan, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_path_refine, dim3(st.nblk), dim3(kPathBlock), 0, s, a);
    SBR_LAUNCHED();
    return SBR_OK;
}

// ------------------------------------------------------------------ Eq. (8)
namespace {


__device__ __forceinline__ float frac_f(float x) { return x - floorf(x); }

// exact fractional part of an integer n times f (n < 2^24): the product is
// formed exactly inside the fma before the nearest integer is removed
__device__ __forceinline__ float frac_mul(float n, float f) {
    float p = n * f;
    return fmaf(n, f, -rintf(p));
}

// A path's beat frequency delta (cycles per sample) is within 0.0403 of 0 or
// 1/2 -- |sin(2 pi delta)| < 1/4 -- on some lane of the wavefront.  Its lanes
// differ only in chirp, so in delta only by the tiny Doppler drift, and the
// choice is made once per wavefront.
__device__ __forceinline__ bool near_dc_or_nyquist(float dph) {
    const float m = fabsf(dph);
    return __any(m < 0.0403f || m > 0.4597f);
}

constexpr int kRotList = 512;   // paths per wavefront remembered for the rotation pass

// Accumulate one path into the lane's L samples.  ROT = false advances the
// phase with the real three-term recurrence z[s+1] = 2 cos(2 pi delta) z[s] -
// z[s-1] (2 FMA per sample), which loses about cot(2 pi delta) <= 4 ulps of
// frequency per step on the paths it is used for.  ROT = true advances by
// complex rotation z[s+1] = z[s] w (4 per sample), accurate at every
// frequency, for the paths near 0 or 1/2 cycle per sample.  Both restart the
// phase exactly (hardware sin/cos in revolutions).
template <int L, bool ROT>
__device__ __forceinline__ void add_path(float alpha, float delta, float dph, float beta, float2 A, float cf,
                                         float s0, float (&ar)[L], float (&ai)[L]) {
    float ph = alpha + frac_mul(cf, beta) + frac_mul(s0, delta);
    ph = ph - rintf(ph);
    const float sn = __builtin_amdgcn_sinf(ph), cs = __builtin_amdgcn_cosf(ph);
    const float ws = __builtin_amdgcn_sinf(dph), wc = __builtin_amdgcn_cosf(dph);
    float zr = A.x * cs - A.y * sn, zi = A.x * sn + A.y * cs;   // z[s0]
    float yr = zr * wc - zi * ws, yi = zr * ws + zi * wc;       // z[s0 + 1]
    ar[0] += zr;
    ai[0] += zi;
    if (L > 1) {
        ar[1] += yr;
        ai[1] += yi;
    }
    if (!ROT) {
        const float k2 = 2.0f * wc;
#pragma unroll
        for (int i = 2; i < L; i++) {
            float nr = fmaf(k2, yr, -zr);
            float ni = fmaf(k2, yi, -zi);
            zr = yr;
            zi = yi;
            yr = nr;
            yi = ni;
            ar[i] += nr;
            ai[i] += ni;
        }
    } else {
#pragma unroll
        for (int i = 2; i < L; i++) {
            float nr = fmaf(yr, wc, -yi * ws);
            float ni = fmaf(yr, ws, yi * wc);
            yr = nr;
            yi = ni;
            ar[i] += nr;
            ai[i] += ni;
        }
    }
}

// One wavefront owns 64 (chirp, sample-block) lanes of one antenna; each lane
// accumulates L consecutive samples over a chunk of paths.  The main pass
// takes the paths whose beat frequency is well away from 0 and 1/2 cycle per
// sample on every lane (recurrence) and remembers the others in LDS; a second
// pass adds those by rotation (it rescans the chunk if more than kRotList of
// them came up).  Path records are wavefront-uniform (scalar loads); the next
// one is fetched while the current one is accumulated.  (bx, chunk) is the
// block's place in the request's own (x, chunk) grid.
template <int L>
__device__ __forceinline__ void synth_block(const SynthArgs &a, const int bx, const int chunk,
                                            int (&rot_list)[4][kRotList]) {
    const int wv = __builtin_amdgcn_readfirstlane(bx * 4 + (int)(threadIdx.x >> 6));
    const int lane = threadIdx.x & 63, wl = threadIdx.x >> 6;
    const int v = __builtin_amdgcn_readfirstlane(wv / a.tiles_per_v);
    if (v >= a.V) return;   // wave-uniform; the kernel has no block barrier
    const int e = (wv % a.tiles_per_v) * 64 + lane;
    const int c = e / a.SB, b = e % a.SB;
    const int P = __builtin_amdgcn_readfirstlane(*gmem(a.count));
    const long long per = ((long long)P + a.n_chunks - 1) / a.n_chunks;
    const int p0 = (int)min((long long)P, per * chunk);
    const int p1 = (int)min((long long)P, per * (chunk + 1));
    const float cf = (float)c;
    const float s0 = (float)(b * L);
    float ar[L], ai[L];
#pragma unroll
    for (int i = 0; i < L; i++) {
        ar[i] = 0.0f;
        ai[i] = 0.0f;
    }
    const auto al = gmem(a.rec.alpha + (size_t)v * a.rec.cap);
    const auto ga = gmem(a.rec.gamma + (size_t)v * a.rec.cap);
    const auto amp = gmem(a.rec.amp);
    const auto bet = gmem(a.rec.beta);
    const auto eps = gmem(a.rec.epsd);
    int n_rot = 0;   // wave-uniform
    {
        float n_al = 0.f, n_ga = 0.f, n_be = 0.f, n_ep = 0.f;
        F2 n_A = {0.f, 0.f};
        if (p0 < p1) {
            n_al = al[p0];
            n_ga = ga[p0];
            n_A = amp[p0];
            n_be = bet[p0];
            n_ep = eps[p0];
        }
        for (int p = p0; p < p1; p++) {
            const float alpha = n_al, gamma = n_ga, beta = n_be, epsd = n_ep;
            const float2 A = make_float2(n_A.x, n_A.y);
            if (p + 1 < p1) {
                n_al = al[p + 1];
                n_ga = ga[p + 1];
                n_A = amp[p + 1];
                n_be = bet[p + 1];
                n_ep = eps[p + 1];
            }
            const float delta = fmaf(cf, epsd, gamma);   // cycles per sample
            const float dph = delta - rintf(delta);
            if (near_dc_or_nyquist(dph)) {
                if (n_rot < kRotList && lane == 0) rot_list[wl][n_rot] = p;
                n_rot++;
                continue;
            }
            add_path<L, false>(alpha, delta, dph, beta, A, cf, s0, ar, ai);
        }
    }
    // rotation pass: over the remembered paths, or the whole chunk again if
    // they did not fit (one loop body, so the accumulators are not doubled)
    const bool listed = n_rot <= kRotList;
    const int n_iter = n_rot == 0 ? 0 : (listed ? n_rot : p1 - p0);
    // the list was written by lane 0 of this wavefront; LDS operations of one
    // wavefront complete in order
    __builtin_amdgcn_fence(__ATOMIC_SEQ_CST, "wavefront");
    for (int i = 0; i < n_iter; i++) {
        const int p = listed ? __builtin_amdgcn_readfirstlane(rot_list[wl][i]) : p0 + i;
        const float delta = fmaf(cf, eps[p], ga[p]);
        const float dph = delta - rintf(delta);
        if (!listed && !near_dc_or_nyquist(dph)) continue;
        const F2 Ap = amp[p];
        add_path<L, true>(al[p], delta, dph, bet[p], make_float2(Ap.x, Ap.y), cf, s0, ar, ai);
    }
    if (c < a.C) {
        const auto out = gmem(a.partial) + ((size_t)chunk * a.V + v) * (size_t)a.C * a.S + (size_t)c * a.S;
        int sb = b * L;
#pragma unroll
        for (int i = 0; i < L; i++)
            if (sb + i < a.S) out[sb + i] = F2{ar[i], ai[i]};
    }
}

// One launch covers the requests of a batch that share L (one request for
// sbr_synth_if): request idx[i] owns blocks [first[i], first[i + 1]) of the
// grid, its own (x, chunk) grid laid out x fastest.  A block finds its
// request by binary search over `first` (uniform, scalar loads), so every
// request's waves do exactly the work they do in a launch of their own.
template <int L>
__global__ __launch_bounds__(256) void k_synth(const SynthArgs *__restrict__ args,
                                               const int32_t *__restrict__ first, const int32_t *__restrict__ idx,
                                               int n) {
    __shared__ int rot_list[4][kRotList];
    const int blk = (int)blockIdx.x;
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first[mid] <= blk) lo = mid;
        else hi = mid;
    }
    const SynthArgs &a = args[idx[lo]];
    const int local = blk - first[lo];
    synth_block<L>(a, local % a.gx, local / a.gx, rot_list);
}

// ---- Eq. (8) on the matrix cores ------------------------------------------
// For one antenna v and chirp c, a 256-sample run s = s_base + 16 s1 + s2
// (s1, s2 < 16) of the sum over paths factors into a complex matrix product
// with the paths as the contracted axis:
//   S[s1][s2] = sum_p U[s1][p] W[p][s2],
//   U[s1][p] = A_p e^{2 pi j (alpha_p + c beta_p + (s_base + 16 s1) delta_p)},
//   W[p][s2] = e^{2 pi j s2 delta_p},  delta_p = gamma_p + c eps_p,
// the first chirp's factors from exactly reduced phases, each later chirp's
// by one complex rotation of the previous one (no recurrence along samples,
// so accurate at every beat frequency).  Four paths at a time feed
// v_mfma_f32_16x16x4_f32 (three real products for the complex one): lane l
// supplies U[l % 16][l / 16] and W[l / 16][l % 16] and holds
// D[4 (l / 16) + j][l % 16].  The VALU only forms the 2 x 16 x 4 factors per
// path quadruple and chirp; the matrix cores do the 8 flops of every
// path-sample.  A wavefront owns one antenna, kMfmaChirps chirps and one
// 256-sample run, over a chunk of paths.
constexpr int kMfmaChirps = 8;
constexpr int kMfmaRun = 256;   // samples per run (16 x 16)

typedef float f32x4s __attribute__((ext_vector_type(4)));

__device__ __forceinline__ void synth_mfma_block(const SynthArgs &a, const int bx, const int chunk) {
    const int wv = __builtin_amdgcn_readfirstlane(bx * 4 + (int)(threadIdx.x >> 6));
    const int v = __builtin_amdgcn_readfirstlane(wv / a.tiles_per_v);
    if (v >= a.V) return;   // wave-uniform; the kernel has no block barrier
    const int rem = wv - v * a.tiles_per_v;
    const int cg = rem / a.SB, run = rem - cg * a.SB;
    const int c0 = cg * kMfmaChirps;
    const int lane = threadIdx.x & 63, k = lane >> 4, i = lane & 15;
    const int P = __builtin_amdgcn_readfirstlane(*gmem(a.count));
    const long long per = ((long long)P + a.n_chunks - 1) / a.n_chunks;
    const int p0 = (int)min((long long)P, per * chunk);
    const int p1 = (int)min((long long)P, per * (chunk + 1));
    const auto al = gmem(a.rec.alpha + (size_t)v * a.rec.cap);
    const auto ga = gmem(a.rec.gamma + (size_t)v * a.rec.cap);
    const auto amp = gmem(a.rec.amp);
    const auto bet = gmem(a.rec.beta);
    const auto eps = gmem(a.rec.epsd);
    const float su = (float)(run * kMfmaRun + 16 * i);   // first sample of this lane's U row
    const float sw = (float)i;                           // this lane's W column
    f32x4s k1[kMfmaChirps], k2[kMfmaChirps], k3[kMfmaChirps];
#pragma unroll
    for (int g = 0; g < kMfmaChirps; g++) {
        k1[g] = (f32x4s){0.f, 0.f, 0.f, 0.f};
        k2[g] = k1[g];
        k3[g] = k1[g];
    }
    const float c0f = (float)c0;
    // the records of the next path quadruple are fetched while the current
    // one is turned into factors and products
    float n_al = 0.f, n_ga = 0.f, n_be = 0.f, n_ep = 0.f;
    F2 n_A = {0.f, 0.f};
    if (p0 + k < p1) {
        n_al = al[p0 + k];
        n_ga = ga[p0 + k];
        n_be = bet[p0 + k];
        n_ep = eps[p0 + k];
        n_A = amp[p0 + k];
    }
    for (int p = p0; p < p1; p += 4) {
        const float alpha = n_al, gamma = n_ga, beta = n_be, epsd = n_ep;
        const float Ax = n_A.x, Ay = n_A.y;   // zero past the chunk's last path
        const int pn = p + 4 + k;
        n_al = n_ga = n_be = n_ep = 0.f;
        n_A = F2{0.f, 0.f};
        if (pn < p1) {
            n_al = al[pn];
            n_ga = ga[pn];
            n_be = bet[pn];
            n_ep = eps[pn];
            n_A = amp[pn];
        }
        // factors of the first chirp c0 from reduced phases; each later chirp
        // multiplies them by e^{2 pi j (beta + su eps)} (U) and
        // e^{2 pi j sw eps} (W), the change of their phases per chirp
        const float delta = fmaf(c0f, epsd, gamma);   // cycles per sample
        float ph = alpha + frac_mul(c0f, beta) + frac_mul(su, delta);
        ph = ph - rintf(ph);
        const float pw = frac_mul(sw, delta);
        float qu = beta + frac_mul(su, epsd);
        qu = qu - rintf(qu);
        const float qw = frac_mul(sw, epsd);
        const float s_u = __builtin_amdgcn_sinf(ph), c_u = __builtin_amdgcn_cosf(ph);
        const float s_w = __builtin_amdgcn_sinf(pw), c_w = __builtin_amdgcn_cosf(pw);
        const float s_ru = __builtin_amdgcn_sinf(qu), c_ru = __builtin_amdgcn_cosf(qu);
        const float s_rw = __builtin_amdgcn_sinf(qw), c_rw = __builtin_amdgcn_cosf(qw);
        float ur[kMfmaChirps], ui[kMfmaChirps], wr[kMfmaChirps], wi[kMfmaChirps];
        ur[0] = Ax * c_u - Ay * s_u;
        ui[0] = Ax * s_u + Ay * c_u;
        wr[0] = c_w;
        wi[0] = s_w;
#pragma unroll
        for (int g = 1; g < kMfmaChirps; g++) {
            ur[g] = fmaf(ur[g - 1], c_ru, -ui[g - 1] * s_ru);
            ui[g] = fmaf(ur[g - 1], s_ru, ui[g - 1] * c_ru);
            wr[g] = fmaf(wr[g - 1], c_rw, -wi[g - 1] * s_rw);
            wi[g] = fmaf(wr[g - 1], s_rw, wi[g - 1] * c_rw);
        }
        // three real products per chirp (Gauss): with U = a + jb, W = c + jd,
        // K1 += (a + b) c, K2 += a (d - c), K3 += b (c + d); then
        // Re = K1 - K3, Im = K1 + K2.  Ordered so that products into one
        // accumulator are kMfmaChirps instructions apart (a group's chirps
        // past C are computed too and never stored)
#pragma unroll
        for (int g = 0; g < kMfmaChirps; g++)
            k1[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(ur[g] + ui[g], wr[g], k1[g], 0, 0, 0);
#pragma unroll
        for (int g = 0; g < kMfmaChirps; g++)
            k2[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(ur[g], wi[g] - wr[g], k2[g], 0, 0, 0);
#pragma unroll
        for (int g = 0; g < kMfmaChirps; g++)
            k3[g] = __builtin_amdgcn_mfma_f32_16x16x4f32(ui[g], wr[g] + wi[g], k3[g], 0, 0, 0);
    }
    const size_t row0 = ((size_t)chunk * a.V + v) * (size_t)a.C;
    const auto out = gmem(a.partial);
#pragma unroll
    for (int g = 0; g < kMfmaChirps; g++) {
        const int c = c0 + g;
        if (c >= a.C) break;
#pragma unroll
        for (int j = 0; j < 4; j++) {
            const int s = run * kMfmaRun + 16 * (4 * k + j) + i;
            out[(row0 + c) * a.S + s] = F2{k1[g][j] - k3[g][j], k1[g][j] + k2[g][j]};
        }
    }
}

__global__ __launch_bounds__(256) void k_synth_mfma(const SynthArgs *__restrict__ args,
                                                    const int32_t *__restrict__ first,
                                                    const int32_t *__restrict__ idx, int n) {
    const int blk = (int)blockIdx.x;
    int lo = 0, hi = n;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first[mid] <= blk) lo = mid;
        else hi = mid;
    }
    const SynthArgs &a = args[idx[lo]];
    const int local = blk - first[lo];
    synth_mfma_block(a, local % a.gx, local / a.gx);
}

// Fixed-order sum of the chunk partials: four running sums over the chunks
// c = 0, 1, 2, 3 (mod 4), so that four loads are in flight, then
// (s0 + s1) + (s2 + s3).
__global__ void k_reduce_chunks(const float2 *partial, int n_chunks, size_t n, float2 *out) {
    size_t e = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= n) return;
    float2 s[4] = {make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f), make_float2(0.f, 0.f)};
    int c = 0;
    for (; c + 4 <= n_chunks; c += 4) {
#pragma unroll
        for (int q = 0; q < 4; q++) {
            const float2 x = partial[(size_t)(c + q) * n + e];
            s[q].x += x.x;
            s[q].y += x.y;
        }
    }
    for (int q = 0; c + q < n_chunks; q++) {
        const float2 x = partial[(size_t)(c + q) * n + e];
        s[q].x += x.x;
        s[q].y += x.y;
    }
    out[e] = make_float2((s[0].x + s[1].x) + (s[2].x + s[3].x), (s[0].y + s[1].y) + (s[2].y + s[3].y));
}

// ---- Eq. (8) by a type-1 non-uniform FFT ----------------------------------
// Row [v][c][.] of the cube is sum_p w_p e^{2 pi j s g_p}, g_p = gamma_p +
// c eps_p reduced to [-1/2, 1/2] and w_p = A_p e^{2 pi j (alpha_p + c beta_p)}.
// With centred modes s' = s - S/2 and w'_p = w_p e^{2 pi j g_p S/2}, the
// identity of the non-uniform FFT forms (sbr_internal.h) gives
//   row[s' + S/2] = (1 / Psi(s'/M)) sum_l b_l e^{2 pi j s' l / M},
//   b_l = sum_p w'_p psi(g_p M - l),
// so each path adds kNuW weighted copies of w'_p to a grid of M = 2S points
// (spreading), and one DFT per row and the deconvolution finish it.  The
// spreading rounds every contribution to an integer of the scale
// 2^(19 - e), max(|Re A|, |Im A|) < 2^e over the paths of its chunk (so below
// 2^19.5 in magnitude; a strong path costs precision only in its own chunk),
// and sums them as integers: integer addition is exact, so the grid and the
// cube do not depend on the order in which blocks, waves or lanes add.

// Request of a block of a batched launch: binary search over first[0..m]
// (request j owns blocks [first[j], first[j + 1])).
__device__ __forceinline__ int nu_request(const int32_t *first, int m, int blk) {
    int lo = 0, hi = m;
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (first[mid] <= blk) lo = mid;
        else hi = mid;
    }
    return lo;
}

// The per-chunk amplitude words of request nidx[blockIdx.x], cleared before
// k_nu_amax runs.
__global__ void k_nu_zero(const SynthArgs *__restrict__ args, const int32_t *__restrict__ nidx) {
    const SynthArgs &a = args[nidx[blockIdx.x]];
    for (int c = threadIdx.x; c < a.n_chunks; c += blockDim.x) a.amax[c] = 0u;
}

// Blocks per path chunk of k_nu_amax.
constexpr int kNuAmaxSub = 16;

// Request nidx[blockIdx.y], chunk blockIdx.x / kNuAmaxSub (the chunks of
// k_nu_spread): max over the chunk's live paths of max(|Re A|, |Im A|), as
// the bits of a non-negative float: an integer maximum, exact and
// order-independent.
__global__ __launch_bounds__(256) void k_nu_amax(const SynthArgs *__restrict__ args,
                                                 const int32_t *__restrict__ nidx) {
    const SynthArgs &a = args[nidx[blockIdx.y]];
    const int chunk = (int)blockIdx.x / kNuAmaxSub, sub = (int)blockIdx.x % kNuAmaxSub;
    if (chunk >= a.n_chunks) return;   // block-uniform
    const int P = *gmem(a.count);
    const long long per = ((long long)P + a.n_chunks - 1) / a.n_chunks;
    const int p0 = (int)min((long long)P, per * chunk);
    const int p1 = (int)min((long long)P, per * (chunk + 1));
    const auto amp = gmem(a.rec.amp);
    uint32_t m = 0;
    for (int p = p0 + sub * 256 + (int)threadIdx.x; p < p1; p += kNuAmaxSub * 256) {
        const F2 A = amp[p];
        m = max(m, __float_as_uint(fmaxf(fabsf(A.x), fabsf(A.y))));
    }
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) m = max(m, (uint32_t)__shfl_xor((int)m, off));
    if ((threadIdx.x & 63) == 0 && m != 0u) atomicMax(a.amax + chunk, m);
}

// Request nidx[blockIdx.y]: its 1/Psi table (nu_corr_value), 256 modes a block.
__global__ __launch_bounds__(256) void k_nu_corr_batch(const SynthArgs *__restrict__ args,
                                                       const int32_t *__restrict__ nidx) {
    __shared__ double kn[kNuTaps];
    if (threadIdx.x < kNuTaps) kn[threadIdx.x] = nu_kernel_sample((int)threadIdx.x);
    __syncthreads();
    const SynthArgs &a = args[nidx[blockIdx.y]];
    const int s = blockIdx.x * blockDim.x + threadIdx.x;
    if (s < a.S) a.corr[s] = nu_corr_value(a.S, s, kn);
}

// Fixed-point scale 2^(19 - e) with max(|Re A|, |Im A|) = amax < 2^e, so that
// |A psi| <= sqrt(2) amax stays below 2^19.5 after scaling (and 2048 such
// contributions below 2^31); e is held in [-100, 128] so that the scale is a
// finite normal float.
__device__ __forceinline__ float nu_scale(uint32_t amax_bits) {
    int e = 0;
    const float amax = __uint_as_float(amax_bits);
    if (amax > 0.0f && amax_bits < 0x7f800000u) (void)frexpf(amax, &e);
    return ldexpf(1.0f, 19 - max(e, -100));
}

// rint(a b) for |a b| < 2^22 as an integer: the fused a b + 1.5 2^23 is
// rounded once to a float of unit spacing whose low mantissa bits hold
// 2^22 + rint(a b).
__device__ __forceinline__ int rint_product(float a, float b) {
    return __float_as_int(fmaf(a, b, 12582912.0f)) - 0x4B400000;
}

constexpr int kNuSpreadThreads = 1024;

// Spreading: block = (path chunk, antenna v, group of cg chirps).  A
// contribution (re, im), both integers below 2^19.5 in magnitude, is added as
// the single 64-bit integer im 2^32 + re to a cell of the block's grid rows
// in LDS ([cg][nu_row_len(S) + 1]: one cell of padding makes the row stride
// odd, so that 32 consecutive rows start on 32 different bank pairs), halving
// the LDS atomics of separate real and imaginary cells.  A cell takes at most
// one contribution per path, so after 2048 paths its sum of real parts RE is
// below 2^31 in magnitude and (RE, IM) is recovered exactly from the low word
// (as a signed 32-bit value) and the rest; at that point every cell is moved
// into 64-bit accumulators held in registers (cell tid + 1024 k of thread
// tid) and cleared.  Paths of a radar scene share few beat frequencies
// (neighbouring paths come from neighbouring rays, and the scene fills few
// range bins), and additions to one cell, or to one bank, within an
// instruction serialise.  So the block takes its chunk 1024 paths at a time,
// lane l of wave w the path at 16 l + w (lanes of a wave 16 paths apart), and
// each lane walks the group's chirps from a starting row chosen so that its
// cell of the first chirp lies on bank pair l mod 32: row r of column j sits
// on bank pair (r (RLs mod 32) + j) mod 32, and RLs is odd, so the row is
// (l - j) times the inverse of RLs mod 32.  With 32 chirps every step of the
// walk then puts the 64 lanes of an instruction on all 32 bank pairs, two
// each, as long as the paths' columns stay put from chirp to chirp.  The
// phase factor e^{2 pi j (alpha + c beta + g S/2)} is computed exactly at
// every eighth chirp of the walk and turned in between (g S/2 changes by
// (S/2) eps from chirp to chirp, up to an integer).
constexpr int kNuCells = 17;   // grid cells per thread: cg (nu_row_len(S) + 1) <= 1024 kNuCells

__global__ __launch_bounds__(kNuSpreadThreads) void k_nu_spread(const SynthArgs *__restrict__ args,
                                                                 const int32_t *__restrict__ nidx,
                                                                 const int32_t *__restrict__ first, int m) {
    extern __shared__ unsigned long long nsp[];
    // blocks in hardware order (dealt to the 8 XCDs in turn, so every
    // request of a batch spreads over all of them): request, then chunk, v,
    // chirp group with the chirp group fastest
    const int j = nu_request(first, m, (int)blockIdx.x);
    const SynthArgs &a = args[nidx[j]];
    const int blk = (int)blockIdx.x - first[j];
    const int S = a.S, M = 2 * S, RL = nu_row_len(S), RLs = RL + 1;
    const int cgi = blk % a.ncg, rest = blk / a.ncg;
    const int v = rest % a.V, chunk = rest / a.V;
    const int c0 = cgi * a.cg, nc = min(a.cg, a.C - c0);
    const int ncell = nc * RLs, tid = (int)threadIdx.x;
    for (int i = tid; i < ncell; i += kNuSpreadThreads) nsp[i] = 0ull;
    long long acc_re[kNuCells], acc_im[kNuCells];
#pragma unroll
    for (int k = 0; k < kNuCells; k++) acc_re[k] = acc_im[k] = 0;
    __syncthreads();
    const int P = __builtin_amdgcn_readfirstlane(*gmem(a.count));
    const long long per = ((long long)P + a.n_chunks - 1) / a.n_chunks;
    const int p0 = (int)min((long long)P, per * chunk);
    const int p1 = (int)min((long long)P, per * (chunk + 1));
    const float sigma = nu_scale(gmem(a.amax)[chunk]);
    const auto al = gmem(a.rec.alpha + (size_t)v * a.rec.cap);
    const auto ga = gmem(a.rec.gamma + (size_t)v * a.rec.cap);
    const auto amp = gmem(a.rec.amp);
    const auto bet = gmem(a.rec.beta);
    const auto eps = gmem(a.rec.epsd);
    const float Mf = (float)M, halfS = (float)(S / 2);
    const int lane = tid & 63, wave = tid >> 6;
    // rows start (RLs mod 32) bank pairs apart; its inverse mod 32 (odd)
    const int rs32 = RLs & 31;
    int inv = rs32;
#pragma unroll
    for (int it = 0; it < 4; it++) inv = (inv * (2 - rs32 * inv)) & 31;
    int step = 0;
    for (int base = p0; base < p1; base += kNuSpreadThreads, step++) {   // block-uniform trip count
        const int p = base + 16 * lane + wave;
        if (p < p1) {
            const float alpha = al[p], gamma = ga[p], beta = bet[p], epsd = eps[p];
            const F2 A = amp[p];
            const float Ax = A.x * sigma, Ay = A.y * sigma;
            // the phase factor turns by r = e^{2 pi j (beta + (S/2) eps)} from one
            // chirp to the next, and by r^-(nc-1) from the group's last chirp to its first
            float rho = beta + frac_mul(halfS, epsd);
            rho -= rintf(rho);
            float rw = -(float)(nc - 1) * rho;
            rw = fmaf(-(float)(nc - 1), rho, -rintf(rw));   // frac(-(nc - 1) rho), exact product
            rw -= rintf(rw);
            const float rs = __builtin_amdgcn_sinf(rho), rc = __builtin_amdgcn_cosf(rho);
            const float ws = __builtin_amdgcn_sinf(rw), wc = __builtin_amdgcn_cosf(rw);
            float zs = 0.0f, zc = 1.0f;
            // starting row: bank pair of (row, j0) = lane mod 32 at the group's first
            // chirp, so the lanes of an instruction spread over all bank pairs
            int cl;
            {
                const float f0 = fmaf((float)c0, epsd, gamma);
                const float x0 = (f0 - rintf(f0)) * Mf;
                const int jj = min(max((int)rintf(x0) + M / 2, 0), M);
                cl = (((lane - jj) * inv) & 31) % nc;
            }
            for (int k = 0; k < nc; k++, cl = cl + 1 == nc ? 0 : cl + 1) {
                const float cf = (float)(c0 + cl);
                const float f = fmaf(cf, epsd, gamma);
                const float g = f - rintf(f);   // [-1/2, 1/2]
                const float x = g * Mf;         // exact
                const float xr = rintf(x);
                const int j0 = min(max((int)xr + M / 2, 0), M);   // cell of l0 = xr - 3 (clamped: NaN-safe)
                if ((k & 7) == 0) {   // wave-uniform: exact every 8 chirps
                    float th = alpha + frac_mul(cf, beta) + frac_mul(halfS, g);
                    th -= rintf(th);
                    zs = __builtin_amdgcn_sinf(th);
                    zc = __builtin_amdgcn_cosf(th);
                } else {
                    const float ms = cl == 0 ? ws : rs, mc = cl == 0 ? wc : rc;
                    const float tc = zc * mc - zs * ms;
                    zs = zc * ms + zs * mc;
                    zc = tc;
                }
                const float wr = Ax * zc - Ay * zs, wi = Ax * zs + Ay * zc;
                float w[kNuW];
                nu_weights(x - xr, w);
                unsigned long long *cell = nsp + (size_t)cl * RLs + j0;
#pragma unroll
                for (int t = 0; t < kNuW; t++) {
                    const int re = rint_product(wr, w[t]), im = rint_product(wi, w[t]);
                    // im 2^32 + re as one 64-bit two's-complement word
                    const unsigned long long word =
                        ((unsigned long long)(uint32_t)(im + (re >> 31)) << 32) | (uint32_t)re;
                    atomicAdd(cell + t, word);
                }
            }
        }
        if ((step & 1) == 1 || base + kNuSpreadThreads >= p1) {   // block-uniform: every 2048 paths
            __syncthreads();   // the steps' additions are done
#pragma unroll
            for (int k = 0; k < kNuCells; k++) {
                const int i = tid + k * kNuSpreadThreads;
                if (i < ncell) {
                    const unsigned long long word = nsp[i];
                    nsp[i] = 0ull;
                    const long long re = (int32_t)(uint32_t)word;
                    acc_re[k] += re;
                    acc_im[k] += ((long long)word - re) >> 32;
                }
            }
            __syncthreads();   // cleared before the next step adds
        }
    }
    // the chunk's rows [c][re, im][RL] of request j's partial
    long long *dst = a.grid + (((size_t)chunk * a.V + v) * a.C + c0) * (size_t)RL * 2;
#pragma unroll
    for (int k = 0; k < kNuCells; k++) {
        const int i = tid + k * kNuSpreadThreads;
        if (i < ncell) {
            const int row = i / RLs, jj = i - row * RLs;
            if (jj < RL) {
                dst[(size_t)(2 * row) * RL + jj] = acc_re[k];
                dst[(size_t)(2 * row + 1) * RL + jj] = acc_im[k];
            }
        }
    }
}

// Row (v, c) = blockIdx.x of the non-uniform FFT form: the chunks' integer
// cells summed and folded onto the periodic grid (cell l of l + M/2 + 3 and,
// for the first 2 kNuHalf + 1 positions, of l + 3M/2 + 3), scaled back to FP64,
// each chunk's cells scaled by its own fixed-point scale and summed in FP64
// in chunk order, then the DFT to the S centred modes and the deconvolution
// 1/Psi.  For M a
// power of two the DFT is an in-place radix-2 FFT in LDS (grid points stored
// at bit-reversed positions), otherwise a direct sum with exact-index
// twiddles.  A non-finite amplitude makes the row NaN, as the direct sum would.
__global__ __launch_bounds__(256) void k_nu_synth_rows(const SynthArgs *__restrict__ args,
                                                       const int32_t *__restrict__ nidx,
                                                       const int32_t *__restrict__ first, int m) {
    extern __shared__ double2 nrs[];
    const int j = nu_request(first, m, (int)blockIdx.x);
    const SynthArgs &a = args[nidx[j]];
    float2 *out = a.out;
    const int S = a.S, M = 2 * S, RL = nu_row_len(S);
    double2 *b = nrs;        // [M]
    double2 *tw = nrs + M;   // [M]
    const size_t row = (size_t)((int)blockIdx.x - first[j]);
    for (int k = threadIdx.x; k < M; k += blockDim.x) {
        double sn, cs;
        sincospi(2.0 * k / M, &sn, &cs);
        tw[k] = make_double2(cs, sn);
    }
    __shared__ double inv_s[kNuMaxChunks];   // 1 / scale of each chunk
    __shared__ int bad_s;
    if (threadIdx.x == 0) bad_s = 0;
    __syncthreads();
    for (int ch = threadIdx.x; ch < a.n_chunks; ch += blockDim.x) {
        const uint32_t ab = gmem(a.amax)[ch];
        inv_s[ch] = 1.0 / (double)nu_scale(ab);
        if (ab >= 0x7f800000u) bad_s = 1;
    }
    __syncthreads();
    const size_t chunk_stride = (size_t)a.V * a.C * RL * 2;
    const bool pow2 = (M & (M - 1)) == 0;
    const int lg = 31 - __clz(M);
    for (int l = threadIdx.x; l < M; l += blockDim.x) {
        const int j1 = (l + M / 2 + kNuHalf) % M;
        const bool wrap = j1 + M < RL - 1;
        double re = 0.0, im = 0.0;
        const long long *src = a.grid + row * RL * 2;   // real row, then imaginary row
        for (int ch = 0; ch < a.n_chunks; ch++, src += chunk_stride) {
            long long cr = src[j1], ci = src[RL + j1];
            if (wrap) {
                cr += src[j1 + M];
                ci += src[RL + j1 + M];
            }
            re = fma((double)cr, inv_s[ch], re);   // exact products (power-of-two scales)
            im = fma((double)ci, inv_s[ch], im);
        }
        b[pow2 ? (int)(__brev((uint32_t)l) >> (32 - lg)) : l] = make_double2(re, im);
    }
    __syncthreads();
    const bool bad = bad_s != 0;
    const auto corr = gmem(a.corr);
    if (pow2) {
        // X[k] = sum_l b_l e^{2 pi j k l / M}, decimation in time
        for (int half = 1; half < M; half <<= 1) {
            const int tstep = M / (2 * half);
            for (int i = threadIdx.x; i < M / 2; i += blockDim.x) {
                const int pos = i & (half - 1), j0 = ((i - pos) << 1) + pos, j1 = j0 + half;
                const double2 w = tw[pos * tstep], u = b[j0], v = b[j1];
                const double2 vw = make_double2(v.x * w.x - v.y * w.y, v.x * w.y + v.y * w.x);
                b[j0] = make_double2(u.x + vw.x, u.y + vw.y);
                b[j1] = make_double2(u.x - vw.x, u.y - vw.y);
            }
            __syncthreads();
        }
        for (int s = threadIdx.x; s < S; s += blockDim.x) {
            const double2 f = b[((s - S / 2) % M + M) % M];   // mode s' = s - S/2
            const double cr = corr[s];
            out[row * S + s] = bad ? make_float2(__int_as_float(0x7fc00000), __int_as_float(0x7fc00000))
                                   : make_float2((float)(f.x * cr), (float)(f.y * cr));
        }
        return;
    }
    for (int s = threadIdx.x; s < S; s += blockDim.x) {
        const int step = ((s - S / 2) % M + M) % M;   // s' mod M
        int k = 0;
        double fr = 0.0, fi = 0.0;
        for (int l = 0; l < M; l++) {
            const double2 t = tw[k], bb = b[l];
            fr = fma(bb.x, t.x, fma(-bb.y, t.y, fr));
            fi = fma(bb.x, t.y, fma(bb.y, t.x, fi));
            k += step;
            if (k >= M) k -= M;
        }
        const double cr = corr[s];
        out[row * S + s] = bad ? make_float2(__int_as_float(0x7fc00000), __int_as_float(0x7fc00000))
                               : make_float2((float)(fr * cr), (float)(fi * cr));
    }
}

}  // namespace

__global__ void k_zero_f32(float *p, size_t n) {
    size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = 0.0f;
}

int fill_zero_f32(float *p, size_t n, hipStream_t s) {
    if (n == 0) return SBR_OK;
    hipLaunchKernelGGL(k_zero_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, p, n);
    SBR_LAUNCHED();
    return SBR_OK;
}

constexpr int kSynthL = 64;   // samples per lane (128 measured slower: occupancy 1)

// Blocks of 256 threads of k_synth<L> the device holds at once (256 CUs x 3
// where the runtime cannot answer).
static int resident_synth_blocks(int L) {
    const void *k = L == kMfmaRun ? (const void *)k_synth_mfma
                    : L == 64     ? (const void *)k_synth<64>
                    : L == 32     ? (const void *)k_synth<32>
                                  : (const void *)k_synth<16>;
    return resident_blocks(k, 256, 0, 256 * 3);
}

// Paths are split into n_chunks chunks.  Every wave of the grid does the same
// work, so the chunk count is chosen to make the grid a whole number of
// device-fulls of resident blocks (about 16k waves in all, 64k for the
// matrix-core form, whose accumulators then sum about 4x fewer paths each in
// FP32): a partly filled last round leaves most of the chip idle for one
// wave's run time.  The plan
// depends only on the request's own sizes (and the device), so a request
// runs the same waves alone and in a batch.
// LDS bytes a spreading block of the non-uniform FFT form may hold: the
// device's per-block limit (160 KiB on gfx950), at most 160 KiB.
static int nu_lds_budget() {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&v, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess || v <= 0)
        v = 65536;
    return std::min(v, 160 * 1024);
}

// Non-uniform FFT form: as many chirps per spreading block as the LDS and
// the threads' accumulators hold (at most 32; each block reads its chunk's
// path records once for all of them), and path chunks enough for about
// three blocks per CU over the device, each of at least 8192 path slots (a
// chunk's partial grid rows cost as much to write and sum as a few thousand
// paths take to spread, so small requests take few chunks).  Depends only on the request's
// sizes and the device, so a request runs the same blocks alone and in a batch.
static SynthPlan nu_plan(int32_t R, int32_t K, int32_t V, int32_t C, int32_t S) {
    SynthPlan p{};
    p.nu = 1;
    p.L = 0;
    const long long row_cells = nu_row_len(S) + 1;
    p.cg = (int32_t)std::max(1LL, std::min<long long>({32LL, (long long)C, nu_lds_budget() / (row_cells * 8),
                                                       (long long)kNuCells * kNuSpreadThreads / row_cells}));
    const long long ncg = (C + p.cg - 1) / p.cg;
    const long long cap = (long long)R * K;
    const long long want = (768 + (long long)V * ncg - 1) / ((long long)V * ncg);
    p.n_chunks = (int32_t)std::max(1LL, std::min({want, (cap + 8191) / 8192, (long long)kNuMaxChunks}));
    return p;
}

SynthPlan synth_plan(int32_t R, int32_t K, int32_t V, int32_t C, int32_t S, bool nu) {
    if (nu) return nu_plan(R, K, V, C, S);
    SynthPlan p{};
    if (S % kMfmaRun == 0) {   // matrix-core form: SB runs per chirp row, waves per antenna
        p.L = kMfmaRun;
        p.SB = S / kMfmaRun;
        p.tiles_per_v = (C + kMfmaChirps - 1) / kMfmaChirps * p.SB;
    } else {
        p.L = S >= kSynthL ? kSynthL : (S >= 32 ? 32 : 16);
        p.SB = (S + p.L - 1) / p.L;
        p.tiles_per_v = (C * p.SB + 63) / 64;
    }
    long long waves = (long long)V * p.tiles_per_v;
    long long grid_x = (waves + 3) / 4;
    long long cap = (long long)R * K;
    const long long target = p.L == kMfmaRun ? 65536 : 16384;
    long long want = (target + waves - 1) / waves;
    // at least 64 path slots per chunk (1024 for the matrix-core form, whose
    // waves each write 8 chirps x 256 samples of partials)
    long long maxc = (cap + 63) / 64;
    if (p.L == kMfmaRun) maxc = (cap + 1023) / 1024;
    const long long res = resident_synth_blocks(p.L);
    long long rounds = std::max(1LL, (long long)std::llround((double)want * grid_x / res));
    long long nch = (rounds * res + grid_x - 1) / grid_x;
    p.n_chunks = (int32_t)std::max(1LL, std::min(std::min(nch, maxc), 1024LL));
    return p;
}

size_t synth_partial_elems(const SynthPlan &p, int32_t V, int32_t C, int32_t S) {
    return p.nu ? 0 : (size_t)p.n_chunks * V * C * S;
}

size_t synth_grid_words(const SynthPlan &p, int32_t V, int32_t C, int32_t S) {
    return p.nu ? (size_t)p.n_chunks * V * C * nu_row_len(S) * 2 : 0;
}

SynthArgs synth_args(const PathStage &st, const SynthPlan &p, int32_t V, int32_t C, int32_t S, float2 *partial,
                     long long *grid, float *corr, uint32_t *amax) {
    SynthArgs a{};
    a.count = st.count;
    a.rec = st.rec;
    a.V = V;
    a.C = C;
    a.S = S;
    a.SB = p.SB;
    a.tiles_per_v = p.tiles_per_v;
    a.n_chunks = p.n_chunks;
    a.gx = (int32_t)(((long long)V * p.tiles_per_v + 3) / 4);
    a.partial = partial;
    a.nu = p.nu;
    a.cg = p.cg;
    a.ncg = p.nu ? (C + p.cg - 1) / p.cg : 0;
    a.grid = grid;
    a.corr = corr;
    a.amax = amax;
    return a;
}

// Device table of a batched synthesis: the requests' arguments, then per
// kernel form (VALU runs of L = 16, 32, 64 samples per lane; the matrix-core
// form, L = 256) the requests using it and their first blocks.
struct SynthTable {
    SynthArgs *args;
    int32_t *idx[4];
    int32_t *first[4];
    int32_t *nidx;     // requests of the non-uniform FFT form
    int32_t *nfirst;   // their first spreading blocks
    int32_t *rfirst;   // their first cube rows
};

static SynthTable synth_table(void *buf, int n, size_t *bytes) {
    Carver cv(buf);
    SynthTable t;
    t.args = cv.take<SynthArgs>(n);
    for (int g = 0; g < 4; g++) {
        t.idx[g] = cv.take<int32_t>(n);
        t.first[g] = cv.take<int32_t>((size_t)n + 1);
    }
    t.nidx = cv.take<int32_t>(n);
    t.nfirst = cv.take<int32_t>((size_t)n + 1);
    t.rfirst = cv.take<int32_t>((size_t)n + 1);
    if (bytes) *bytes = align_up(cv.off, 256);
    return t;
}

size_t synth_table_bytes(int n) {
    size_t b = 0;
    synth_table(nullptr, n, &b);
    return b;
}

int launch_synth_batch(const SynthArgs *args, const int *L, int n, void *table, float2 *const *out,
                       hipStream_t s) {
    if (n <= 0) return SBR_OK;
    SynthTable t = synth_table(table, n, nullptr);
    std::vector<SynthArgs> aa(args, args + n);
    for (int i = 0; i < n; i++) aa[i].out = out[i];
    int rc = put_table(t.args, aa.data(), sizeof(SynthArgs) * n, s);
    if (rc) return rc;
    static const int kLs[4] = {16, 32, 64, kMfmaRun};
    for (int g = 0; g < 4; g++) {
        std::vector<int32_t> idx, first(1, 0);
        for (int i = 0; i < n; i++) {
            if (L[i] != kLs[g]) continue;
            const long long blocks = (long long)args[i].gx * args[i].n_chunks;
            if (first.back() + blocks > 0x7fffffffLL) {
                set_error("batched synthesis: more than 2^31 blocks in one launch");
                return SBR_E_ARG;
            }
            idx.push_back(i);
            first.push_back(first.back() + (int32_t)blocks);
        }
        if (idx.empty() || first.back() == 0) continue;
        if ((rc = put_table(t.idx[g], idx.data(), sizeof(int32_t) * idx.size(), s))) return rc;
        if ((rc = put_table(t.first[g], first.data(), sizeof(int32_t) * first.size(), s))) return rc;
        const int m = (int)idx.size();
        const dim3 grid((unsigned)first.back());
        ProfScope ps(kProfSynth, s);
        if (kLs[g] == kMfmaRun)
            hipLaunchKernelGGL(k_synth_mfma, grid, dim3(256), 0, s, t.args, t.first[g], t.idx[g], m);
        else if (kLs[g] == 64)
            hipLaunchKernelGGL(k_synth<64>, grid, dim3(256), 0, s, t.args, t.first[g], t.idx[g], m);
        else if (kLs[g] == 32)
            hipLaunchKernelGGL(k_synth<32>, grid, dim3(256), 0, s, t.args, t.first[g], t.idx[g], m);
        else
            hipLaunchKernelGGL(k_synth<16>, grid, dim3(256), 0, s, t.args, t.first[g], t.idx[g], m);
    }
    SBR_LAUNCHED();
    for (int i = 0; i < n; i++) {
        if (args[i].nu) continue;
        const size_t e = (size_t)args[i].V * args[i].C * args[i].S;
        hipLaunchKernelGGL(k_reduce_chunks, dim3((unsigned)((e + 255) / 256)), dim3(256), 0, s, args[i].partial,
                           args[i].n_chunks, e, out[i]);
    }
    SBR_LAUNCHED();
    // the non-uniform FFT form, all its requests in five launches: amplitude
    // words cleared, amplitude bounds, 1/Psi tables, spreading, row transforms
    std::vector<int32_t> nidx, nfirst(1, 0), rfirst(1, 0);
    size_t lds_spread = 0, lds_rows = 0;
    int max_s = 0, max_chunks = 1;
    for (int i = 0; i < n; i++) {
        const SynthArgs &a = args[i];
        if (!a.nu) continue;
        const long long blocks = (long long)a.n_chunks * a.V * a.ncg, rows = (long long)a.V * a.C;
        if (nfirst.back() + blocks > 0x7fffffffLL || rfirst.back() + rows > 0x7fffffffLL) {
            set_error("batched synthesis: more than 2^31 blocks in one launch");
            return SBR_E_ARG;
        }
        if ((long long)a.cg * (nu_row_len(a.S) + 1) > (long long)kNuCells * kNuSpreadThreads) {
            set_error("batched synthesis: spreading rows exceed the accumulators");
            return SBR_E_ARG;
        }
        nidx.push_back(i);
        nfirst.push_back(nfirst.back() + (int32_t)blocks);
        rfirst.push_back(rfirst.back() + (int32_t)rows);
        lds_spread = std::max(lds_spread, (size_t)a.cg * (nu_row_len(a.S) + 1) * 8);
        lds_rows = std::max(lds_rows, (size_t)2 * 2 * a.S * sizeof(double2));
        max_s = std::max(max_s, (int)a.S);
        max_chunks = std::max(max_chunks, (int)a.n_chunks);
    }
    if (!nidx.empty()) {
        const int m = (int)nidx.size();
        if ((rc = put_table(t.nidx, nidx.data(), sizeof(int32_t) * m, s))) return rc;
        if ((rc = put_table(t.nfirst, nfirst.data(), sizeof(int32_t) * (m + 1), s))) return rc;
        if ((rc = put_table(t.rfirst, rfirst.data(), sizeof(int32_t) * (m + 1), s))) return rc;
        ProfScope ps(kProfSynth, s);
        hipLaunchKernelGGL(k_nu_zero, dim3((unsigned)m), dim3(256), 0, s, t.args, t.nidx);
        hipLaunchKernelGGL(k_nu_amax, dim3((unsigned)(kNuAmaxSub * max_chunks), (unsigned)m), dim3(256), 0, s,
                           t.args, t.nidx);
        hipLaunchKernelGGL(k_nu_corr_batch, dim3((unsigned)((max_s + 255) / 256), (unsigned)m), dim3(256), 0, s,
                           t.args, t.nidx);
        SBR_LAUNCHED();
        if (lds_spread > 65536)
            SBR_HIP(hipFuncSetAttribute((const void *)k_nu_spread, hipFuncAttributeMaxDynamicSharedMemorySize,
                                        (int)lds_spread));
        {
            ProfScope pk(kProfNuSpread, s);
            hipLaunchKernelGGL(k_nu_spread, dim3((unsigned)nfirst.back()), dim3(kNuSpreadThreads), lds_spread, s,
                               t.args, t.nidx, t.nfirst, m);
        }
        SBR_LAUNCHED();
        hipLaunchKernelGGL(k_nu_synth_rows, dim3((unsigned)rfirst.back()), dim3(256), lds_rows, s, t.args, t.nidx,
                           t.rfirst, m);
        SBR_LAUNCHED();
    }
    return SBR_OK;
}

}  // namespace sbr
