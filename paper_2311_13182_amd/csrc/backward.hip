// Backpropagation: adjoint of the IF synthesis (Eqs. 11-12) per path, then
// the reverse sweep through the ray geometry of every ray (Eq. 13 chain rule)
// with per-bounce recomputation, scattering dL/dverts.
#include "sbr_internal.h"
#include "sbr_device.h"

namespace sbr {

namespace {

struct AdjArgs {
    const int32_t *count;
    PathSoA rec;
    const float2 *G;       // [V][C][S]
    int32_t V, C, S;
    int32_t rows;          // G rows per LDS stage
    int32_t Sp;            // S rounded up to a multiple of 8
    int32_t v_per;         // antennas per y-block
    int32_t nvs;           // y-blocks
    float fcf, sl_fs, tc;  // fc, slope / fs, chirp period
    float *tau_bar;        // [V][cap]
    float2 *abar_part;     // [nvs][cap]
};

constexpr int kAdjRowsMax = 8;   // G rows staged in LDS at a time (at most 64 KiB)
constexpr int kAdjPPL = 2;       // paths per lane

// Path-stationary adjoint of Eq. (8).  For each (path, v, c) the sums
//   P(x) = sum_s conj(G_s) x^s,  P'(x)   with x = e^{2 pi j delta}
// run by Horner's rule; with z0 = e^{2 pi j phi0}:
//   sum_s w_s = z0 P(x),  sum_s s w_s = z0 x P'(x),  w_s = conj(G_s) e^{j phi_s}
//   dL/dA    += conj(z0 P(x))                                  (Eq. 12)
//   dL/dtau  += -2 pi Im(A (fc z0 P + (slope/fs) z0 x P'))       (Eq. 11)
// Each lane carries PPL paths (256 apart) so every G sample read from LDS
// feeds 8 * PPL fused multiply-adds.
template <int PPL>
__global__ __launch_bounds__(256) void k_synth_adj(AdjArgs a) {
    extern __shared__ float2 gsh[];   // [rows][Sp]
    const int P = a.count[0];
    const int blk_p0 = blockIdx.x * 256 * PPL;
    if (blk_p0 >= P) return;   // uniform over the block
    int pp[PPL];
    bool act[PPL];
    float2 A[PPL];
    float beta[PPL], epsd[PPL], abr[PPL], abi[PPL];
#pragma unroll
    for (int i = 0; i < PPL; i++) {
        pp[i] = blk_p0 + i * 256 + threadIdx.x;
        act[i] = pp[i] < P;
        const int pc = act[i] ? pp[i] : blk_p0;
        A[i] = a.rec.amp[pc];
        beta[i] = a.rec.beta[pc];
        epsd[i] = a.rec.epsd[pc];
        abr[i] = 0.0f;
        abi[i] = 0.0f;
        pp[i] = pc;
    }
    const int v0 = blockIdx.y * a.v_per, v1 = min(a.V, v0 + a.v_per);
    const int S = a.S;
    for (int v = v0; v < v1; v++) {
        float alpha[PPL], gamma[PPL], tb[PPL];
#pragma unroll
        for (int i = 0; i < PPL; i++) {
            alpha[i] = a.rec.alpha[(size_t)v * a.rec.cap + pp[i]];
            gamma[i] = a.rec.gamma[(size_t)v * a.rec.cap + pp[i]];
            tb[i] = 0.0f;
        }
        for (int c0 = 0; c0 < a.C; c0 += a.rows) {
            const int nr = min(a.rows, a.C - c0);
            __syncthreads();
            // rows padded with zeros to Sp = S rounded up to 8: leading zero
            // coefficients leave Horner's recurrences unchanged
            const float2 *src = a.G + ((size_t)v * a.C + c0) * S;
            for (int i = threadIdx.x; i < nr * a.Sp; i += 256) {
                const int rr = i / a.Sp, ss = i - rr * a.Sp;
                gsh[i] = ss < S ? src[(size_t)rr * S + ss] : make_float2(0.0f, 0.0f);
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
                    tb[i] += -2.0f * (float)kPi * (A[i].x * mi + A[i].y * mr);
                }
            }
        }
#pragma unroll
        for (int i = 0; i < PPL; i++)
            if (act[i]) a.tau_bar[(size_t)v * a.rec.cap + pp[i]] = tb[i];
    }
#pragma unroll
    for (int i = 0; i < PPL; i++)
        if (act[i]) a.abar_part[(size_t)blockIdx.y * a.rec.cap + pp[i]] = make_float2(abr[i], abi[i]);
}

__global__ void k_reduce_abar(const int32_t *count, const float2 *part, int nvs, int cap, float2 *abar) {
    int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= count[0]) return;
    float r = 0.0f, i = 0.0f;
    for (int s = 0; s < nvs; s++) {
        float2 x = part[(size_t)s * cap + p];
        r += x.x;
        i += x.y;
    }
    abar[p] = make_float2(r, i);
}

struct GeomArgs {
    const float *verts;
    const int32_t *faces;
    const uint16_t *mat_id;
    const int32_t *tri;
    int32_t R;
    MatTable mt;
    int32_t any_fresnel;
    RadarDev rd;
    GridDev g;
    ChirpDev ch;
    const int32_t *ray_first;
    const float2 *abar;
    const float *tau_bar;   // [V][cap]
    int32_t cap;
    float *grad;            // [nv][3]
};

struct d3 {
    double x, y, z;
};
__device__ __forceinline__ d3 mk(double x, double y, double z) { return {x, y, z}; }
__device__ __forceinline__ d3 operator+(d3 a, d3 b) { return {a.x + b.x, a.y + b.y, a.z + b.z}; }
__device__ __forceinline__ d3 operator-(d3 a, d3 b) { return {a.x - b.x, a.y - b.y, a.z - b.z}; }
__device__ __forceinline__ d3 operator*(double s, d3 a) { return {s * a.x, s * a.y, s * a.z}; }
__device__ __forceinline__ double dot(d3 a, d3 b) { return a.x * b.x + a.y * b.y + a.z * b.z; }
__device__ __forceinline__ d3 cross(d3 a, d3 b) {
    return {a.y * b.z - a.z * b.y, a.z * b.x - a.x * b.z, a.x * b.y - a.y * b.x};
}
__device__ __forceinline__ double nrm(d3 a) { return sqrt(dot(a, a)); }
__device__ __forceinline__ d3 vload(const float *v, int i) { return {v[3 * i], v[3 * i + 1], v[3 * i + 2]}; }

__device__ __forceinline__ void scatter(float *g, int vi, d3 x) {
    atomicAdd(&g[3 * vi], (float)x.x);
    atomicAdd(&g[3 * vi + 1], (float)x.y);
    atomicAdd(&g[3 * vi + 2], (float)x.z);
}

template <int K>
__global__ __launch_bounds__(128) void k_geom_adj(GeomArgs a) {
    const int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= a.R) return;
    const int first = a.ray_first[r];
    const int n = a.ray_first[r + 1] - first;
    if (n <= 0) return;
    const int ix = r % a.g.nx, iy = r / a.g.nx;
    double d0[3], dw;
    grid_ray(a.g, a.rd, ix, iy, d0, &dw);
    const d3 O = mk(a.rd.o[0], a.rd.o[1], a.rd.o[2]);
    // ---- forward recompute (double), kept per bounce
    d3 X[K], D[K];
    double T[K], Lc[K];
    int F[K];
    d3 dir = mk(d0[0], d0[1], d0[2]);
    d3 o = O;
    double L = 0.0;
#pragma unroll
    for (int k = 0; k < K; k++) {
        if (k < n) {
            const int f = a.tri[(size_t)k * a.R + r];
            d3 va = vload(a.verts, a.faces[3 * f]), vb = vload(a.verts, a.faces[3 * f + 1]),
               vc = vload(a.verts, a.faces[3 * f + 2]);
            d3 N = cross(vb - va, vc - va);
            double t = dot(N, va - o) / dot(N, dir);
            d3 x = o + t * dir;
            L += nrm(x - o);
            X[k] = x;
            D[k] = dir;
            T[k] = t;
            Lc[k] = L;
            F[k] = f;
            double nl = nrm(N);
            d3 nh = (1.0 / nl) * N;
            dir = dir - (2.0 * dot(dir, nh)) * nh;
            o = x;
        }
    }
    // ---- path adjoints -> dL/dx_j, dL/dcos_j
    d3 xb[K];
    double cib[K];
#pragma unroll
    for (int k = 0; k < K; k++) {
        xb[k] = mk(0, 0, 0);
        cib[k] = 0.0;
    }
    const int ntx = a.rd.n_tx, nrx = a.rd.n_rx;
    const double ic0 = 1.0 / kC0;
#pragma unroll
    for (int k = 0; k < K; k++) {
        if (k < n) {
            const int p = first + k;
            const float2 ab = a.abar[p];
            // amplitude pieces of bounce k
            double ci[K];
            cd rj[K], drj[K];
            cd prod = {1.0, 0.0};
#pragma unroll
            for (int j = 0; j <= k; j++) {
                d3 va = vload(a.verts, a.faces[3 * F[j]]), vb = vload(a.verts, a.faces[3 * F[j] + 1]),
                   vc = vload(a.verts, a.faces[3 * F[j] + 2]);
                d3 N = cross(vb - va, vc - va);
                ci[j] = fabs(dot(D[j], N)) / nrm(N);
                reflect_coef(a.mt, a.mat_id ? (int)a.mat_id[F[j]] : 0, a.ch.fc, ci[j], rj[j], drj[j]);
                prod = {prod.re * rj[j].re - prod.im * rj[j].im, prod.re * rj[j].im + prod.im * rj[j].re};
            }
            const double Lk = Lc[k];
            const double Rk = nrm(X[k] - O);
            // A = dw * prod * ci_k / (L R);  u = Re(conj(Abar) * dw * prod / (L R))
            const double s = dw / (Lk * Rk);
            const double u = s * (ab.x * prod.re + ab.y * prod.im);
            const double g = u * ci[k];      // Re(conj(Abar) A)
            cib[k] += u;
            const double Lb = -g / Lk, Rb = -g / Rk;
            if (a.any_fresnel) {
#pragma unroll
                for (int j = 0; j <= k; j++) {
                    cd ex = {s * ci[k], 0.0};
#pragma unroll
                    for (int i = 0; i <= k; i++)
                        if (i != j) ex = {ex.re * rj[i].re - ex.im * rj[i].im, ex.re * rj[i].im + ex.im * rj[i].re};
                    cd dA = {ex.re * drj[j].re - ex.im * drj[j].im, ex.re * drj[j].im + ex.im * drj[j].re};
                    cib[j] += ab.x * dA.re + ab.y * dA.im;
                }
            }
            // L_k = sum_{j<=k} |x_j - x_{j-1}| (x_{-1} = O);  R_k = |x_k - O|
            d3 prv = O;
#pragma unroll
            for (int j = 0; j <= k; j++) {
                d3 sg = X[j] - prv;
                d3 uj = (1.0 / nrm(sg)) * sg;
                xb[j] = xb[j] + Lb * uj;
                if (j > 0) xb[j - 1] = xb[j - 1] - Lb * uj;
                prv = X[j];
            }
            xb[k] = xb[k] + (Rb / Rk) * (X[k] - O);
            // time of flight: tx_t -> x_0 -> ... -> x_k -> rx_m
            double TS[SBR_MAX_TX], RS[SBR_MAX_RX], Tt = 0.0;
            for (int t = 0; t < ntx; t++) TS[t] = 0.0;
            for (int m = 0; m < nrx; m++) RS[m] = 0.0;
            for (int t = 0; t < ntx; t++)
                for (int m = 0; m < nrx; m++) {
                    double tb = a.tau_bar[(size_t)(t * nrx + m) * a.cap + p];
                    TS[t] += tb;
                    RS[m] += tb;
                    Tt += tb;
                }
            for (int t = 0; t < ntx; t++) {
                d3 q = X[0] - mk(a.rd.tx[t][0], a.rd.tx[t][1], a.rd.tx[t][2]);
                xb[0] = xb[0] + (TS[t] * ic0 / nrm(q)) * q;
            }
            for (int m = 0; m < nrx; m++) {
                d3 q = X[k] - mk(a.rd.rx[m][0], a.rd.rx[m][1], a.rd.rx[m][2]);
                xb[k] = xb[k] + (RS[m] * ic0 / nrm(q)) * q;
            }
#pragma unroll
            for (int j = 1; j <= k; j++) {
                d3 sg = X[j] - X[j - 1];
                d3 uj = (Tt * ic0 / nrm(sg)) * sg;
                xb[j] = xb[j] + uj;
                xb[j - 1] = xb[j - 1] - uj;
            }
        }
    }
    // ---- reverse sweep over bounces
    d3 dnext = mk(0, 0, 0);   // dL/d d_{j+1}
#pragma unroll
    for (int j = K - 1; j >= 0; j--) {
        if (j < n) {
            const int f = F[j];
            const int ia = a.faces[3 * f], ibv = a.faces[3 * f + 1], icv = a.faces[3 * f + 2];
            d3 va = vload(a.verts, ia), vb = vload(a.verts, ibv), vc = vload(a.verts, icv);
            d3 e1 = vb - va, e2 = vc - va;
            d3 N = cross(e1, e2);
            double nl = nrm(N);
            d3 nh = (1.0 / nl) * N;
            d3 d = D[j];
            double dn = dot(d, nh);
            double sgn = dn >= 0.0 ? 1.0 : -1.0;
            double t = T[j];
            d3 ob = xb[j];                    // x = o + t d
            double tbar = dot(xb[j], d);
            d3 db = t * xb[j];
            d3 nhb = mk(0, 0, 0);
            db = db + (cib[j] * sgn) * nh;    // cos = |d . n|
            nhb = nhb + (cib[j] * sgn) * d;
            // d_{j+1} = d - 2 (d.n) n
            double ndn = dot(nh, dnext);
            db = db + dnext - (2.0 * ndn) * nh;
            nhb = nhb - 2.0 * (dn * dnext + ndn * d);
            // t = N.(a - o) / (N.d)
            double den = dot(N, d);
            d3 Nb = (tbar / den) * (va - X[j]);
            d3 ab = (tbar / den) * N;
            ob = ob - (tbar / den) * N;
            db = db - (tbar * t / den) * N;
            // n = N / |N|
            Nb = Nb + (1.0 / nl) * (nhb - dot(nhb, nh) * nh);
            // N = e1 x e2
            d3 e1b = cross(e2, Nb), e2b = cross(Nb, e1);
            d3 bb = e1b, cb = e2b;
            ab = ab - e1b - e2b;
            scatter(a.grad, ia, ab);
            scatter(a.grad, ibv, bb);
            scatter(a.grad, icv, cb);
            if (j > 0) xb[j - 1] = xb[j - 1] + ob;
            dnext = db;
        }
    }
}

}  // namespace

struct BackPlan {
    int nvs, v_per;
};

static BackPlan back_plan(long long cap, int V) {
    long long blocks = (cap + 256 * kAdjPPL - 1) / (256 * kAdjPPL);
    long long want = (4096 + blocks - 1) / std::max(1LL, blocks);
    int nvs = (int)std::max(1LL, std::min((long long)V, want));
    int v_per = (V + nvs - 1) / nvs;
    nvs = (V + v_per - 1) / v_per;
    return {nvs, v_per};
}

size_t backward_extra_bytes(int32_t R, int32_t K, int32_t V) {
    long long cap = (long long)R * K;
    BackPlan bp = back_plan(cap, V);
    Carver cv(nullptr);
    cv.take<float>((size_t)V * cap);
    cv.take<float2>((size_t)bp.nvs * cap);
    cv.take<float2>(cap);
    return align_up(cv.off, 256);
}

int launch_backward(const sbr_mesh *m, const MatTable &mt, const RadarDev &rd, const GridDev &gd,
                    const ChirpDev &cd, const sbr_hits *h, const PathStage &st, Carver &cv,
                    const float2 *G, float *grad, hipStream_t s) {
    const int V = rd.n_tx * rd.n_rx;
    const long long cap = st.rec.cap;
    BackPlan bp = back_plan(cap, V);
    float *tau_bar = cv.take<float>((size_t)V * cap);
    float2 *part = cv.take<float2>((size_t)bp.nvs * cap);
    float2 *abar = cv.take<float2>(cap);
    AdjArgs a;
    a.count = st.count;
    a.rec = st.rec;
    a.G = G;
    a.V = V;
    a.C = cd.C;
    a.S = cd.S;
    a.v_per = bp.v_per;
    a.nvs = bp.nvs;
    a.fcf = (float)cd.fc;
    a.sl_fs = (float)(cd.slope / cd.fs);
    a.tc = (float)cd.tc;
    a.tau_bar = tau_bar;
    a.abar_part = part;
    dim3 grid((unsigned)((cap + 256 * kAdjPPL - 1) / (256 * kAdjPPL)), (unsigned)bp.nvs);
    a.Sp = (cd.S + 7) / 8 * 8;
    a.rows = std::max(1, std::min(kAdjRowsMax, 8192 / a.Sp));
    size_t lds = sizeof(float2) * a.rows * a.Sp;
    {
        ProfScope ps(kProfSynthAdj, s);
        hipLaunchKernelGGL(k_synth_adj<kAdjPPL>, grid, dim3(256), lds, s, a);
    }
    hipLaunchKernelGGL(k_reduce_abar, dim3((unsigned)((cap + 255) / 256)), dim3(256), 0, s, st.count, part,
                       bp.nvs, (int)cap, abar);
    SBR_LAUNCHED();
    GeomArgs g;
    g.verts = m->verts;
    g.faces = m->faces;
    g.mat_id = m->mat_id;
    g.tri = h->tri;
    g.R = gd.nx * gd.ny;
    g.mt = mt;
    g.any_fresnel = 0;
    for (int i = 0; i < mt.n; i++)
        if (mt.mode[i] != 0) g.any_fresnel = 1;
    g.rd = rd;
    g.g = gd;
    g.ch = cd;
    g.ray_first = st.ray_first;
    g.abar = abar;
    g.tau_bar = tau_bar;
    g.cap = (int32_t)cap;
    g.grad = grad;
    dim3 gg((unsigned)((g.R + 127) / 128));
    switch (gd.K) {
    case 1: hipLaunchKernelGGL(k_geom_adj<1>, gg, dim3(128), 0, s, g); break;
    case 2: hipLaunchKernelGGL(k_geom_adj<2>, gg, dim3(128), 0, s, g); break;
    case 3: hipLaunchKernelGGL(k_geom_adj<3>, gg, dim3(128), 0, s, g); break;
    case 4: hipLaunchKernelGGL(k_geom_adj<4>, gg, dim3(128), 0, s, g); break;
    case 5: hipLaunchKernelGGL(k_geom_adj<5>, gg, dim3(128), 0, s, g); break;
    case 6: hipLaunchKernelGGL(k_geom_adj<6>, gg, dim3(128), 0, s, g); break;
    case 7: hipLaunchKernelGGL(k_geom_adj<7>, gg, dim3(128), 0, s, g); break;
    default: hipLaunchKernelGGL(k_geom_adj<8>, gg, dim3(128), 0, s, g); break;
    }
    SBR_LAUNCHED();
    return SBR_OK;
}

}  // namespace sbr
