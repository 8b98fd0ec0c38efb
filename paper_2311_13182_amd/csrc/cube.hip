// The signal-to-image map T of the spatial loss (Eq. 16): range, Doppler and
// angle DFTs and their conjugate transpose; and the CA-CFAR point extraction.
// Power-of-two range and Doppler lengths run as Stockham FFTs in LDS; the
// angle stage of a linear array is a direct DFT by Horner's rule, fused with
// the range FFT in the forward map when one Doppler bin fits in LDS; other
// lengths and the planar angle stage are dense FP32 contractions with the DFT
// matrix on the matrix cores (MFMA), twiddles by exact index (k n mod N).
#include <mutex>

#include "sbr_internal.h"

namespace sbr {

namespace {

// twiddle table e^{sign 2 pi j k / N}, k < N, built in double
__device__ void make_twiddles(float2 *tw, int N, int sign) {
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        double s, c;
        sincospi(2.0 * k / N, &s, &c);
        tw[k] = make_float2((float)c, (float)(sign * s));
    }
}

__device__ __forceinline__ float window_at(int window, int i, int N) {
    if (window == 1 && N > 1) return (float)(0.5 - 0.5 * cospi(2.0 * i / (N - 1)));
    return 1.0f;
}

typedef float f32x4 __attribute__((ext_vector_type(4)));

// D += A B for complex A, B on four real 16x16x4 FP32 MFMAs.  Lane l supplies
// A[l % 16][l / 16] and B[l / 16][l % 16]; D[4 (l / 16) + j][l % 16] is
// element j of the lane's accumulators.
__device__ __forceinline__ void cmfma(float ar, float ai, float br, float bi, f32x4 &dr, f32x4 &di) {
    dr = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, br, dr, 0, 0, 0);
    di = __builtin_amdgcn_mfma_f32_16x16x4f32(ar, bi, di, 0, 0, 0);
    dr = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai, bi, dr, 0, 0, 0);
    di = __builtin_amdgcn_mfma_f32_16x16x4f32(ai, br, di, 0, 0, 0);
}

// Workgroups are dealt to the 8 XCDs round robin.  Renumber them so that each
// XCD runs a contiguous range of logical blocks: neighbouring tiles, which
// read the same input rows, then share one L2.  The ragged tail (gridDim.x
// mod 8 blocks) keeps its index.
__device__ __forceinline__ long long xcd_logical_block() {
    const unsigned b = blockIdx.x, per = gridDim.x / 8;
    if (b >= per * 8) return b;
    return (long long)(b % 8) * per + b / 8;
}

// LDS tables shared by both transforms: Nt twiddles, then the window over the
// pre-windowed input axis (length N) or the post-windowed output axis (M).
__device__ void dft_tables(float2 *tw, float *wt, int Nt, int sign, int window, int Lw) {
    make_twiddles(tw, Nt, sign);
    for (int k = threadIdx.x; k < Lw; k += blockDim.x) wt[k] = window_at(window, k, Lw);
    __syncthreads();
}

// DFT along the innermost axis as a dense FP32 contraction on the matrix
// cores: [rows][N] -> [rows][M],
//   out[row][m] = w_post(m) sum_n w_pre(n) in[row][n] e^{sign 2 pi j (n m mod Nt) / Nt}.
// A wavefront owns 16 rows x 16 outputs.  Per step of 4 input columns: A = the
// 16 x 4 input block (global loads, lane l reads row r0 + l%16, column
// n0 + l/16), B = the 4 x 16 twiddle block from LDS (exact index n m mod Nt,
// advanced incrementally).  Waves of one block share the rows (m tiles
// fastest), so the input is read from HBM once and reused from cache.
__global__ __launch_bounds__(256) void k_dft_inner(const float2 *in, float2 *out, int rows, int N, int M, int Nt,
                                                    int sign, int window, int post) {
    extern __shared__ float2 sm[];
    float2 *tw = sm;
    float *wt = reinterpret_cast<float *>(sm + Nt);
    dft_tables(tw, wt, Nt, sign, window, post ? M : N);
    const int mt = (M + 15) / 16;
    const long long tile = xcd_logical_block() * 4 + (threadIdx.x >> 6);
    if (tile >= (long long)mt * ((rows + 15) / 16)) return;   // wave-uniform; no barrier follows
    const int m_t = (int)(tile % mt), r_t = (int)(tile / mt);
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int row = r_t * 16 + r;   // A row of this lane
    const int m = m_t * 16 + r;     // B column of this lane
    const float2 *src = in + (size_t)(row < rows ? row : 0) * N;
    const int step = (int)((4LL * m) % Nt);
    int idx = (int)(((long long)q * m) % Nt);
    // 16 input columns per stage, two register buffers in turn: the loads of
    // one stage are in flight while the MFMAs of the previous one run (no
    // copy between buffers, so no wait on loads still in flight).  Loads are
    // unconditional (clamped addresses; weight zero outside the matrix).
    // Alternate steps go to two accumulator pairs.
    const int N1 = N - 1;
    f32x4 dr0 = {0.f, 0.f, 0.f, 0.f}, di0 = dr0, dr1 = dr0, di1 = dr0;
    auto load = [&](float2 *buf, int n0) {
#pragma unroll
        for (int u = 0; u < 4; u++) buf[u] = src[min(n0 + 4 * u + q, N1)];
    };
    auto stage = [&](const float2 *buf, int n0) {
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int n = n0 + 4 * u + q;
            const float w = (row < rows && n < N) ? (post ? 1.0f : wt[min(n, N1)]) : 0.0f;
            const float2 t = tw[idx];
            idx += step;
            if (idx >= Nt) idx -= Nt;
            if (u & 1) cmfma(buf[u].x * w, buf[u].y * w, t.x, t.y, dr1, di1);
            else cmfma(buf[u].x * w, buf[u].y * w, t.x, t.y, dr0, di0);
        }
    };
    float2 ba[4], bb[4];
    load(ba, 0);
    for (int n0 = 0; n0 < N; n0 += 32) {
        load(bb, n0 + 16);
        stage(ba, n0);
        load(ba, n0 + 32);
        if (n0 + 16 < N) stage(bb, n0 + 16);
    }
    const f32x4 dr = dr0 + dr1, di = di0 + di1;
    const int mo = m_t * 16 + r;
    if (mo >= M) return;
    const float w = post ? wt[mo] : 1.0f;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int ro = r_t * 16 + 4 * q + j;
        if (ro < rows) out[(size_t)ro * M + mo] = make_float2(dr[j] * w, di[j] * w);
    }
}

// DFT along a middle axis as a dense FP32 contraction on the matrix cores:
// [outer][N][inner] -> [outer][M][inner],
//   out[o][m][i] = w_post(m) sum_n e^{sign 2 pi j (m n mod Nt) / Nt} w_pre(n) in[o][n][i].
// A wavefront owns 16 (m) x 16 (i) outputs.  Per step of 4 input rows: A = the
// 16 x 4 twiddle block from LDS (window folded in), B = the 4 x 16 input block
// (four 128-byte row segments).
__global__ __launch_bounds__(256) void k_dft_mid(const float2 *in, float2 *out, int outer, int N, int M, int Nt,
                                                  int inner, int sign, int window, int post) {
    extern __shared__ float2 sm[];
    float2 *tw = sm;
    float *wt = reinterpret_cast<float *>(sm + Nt);
    dft_tables(tw, wt, Nt, sign, window, post ? M : N);
    const int mt = (M + 15) / 16, it = (inner + 15) / 16;
    // m tiles fastest: the waves of a block, and neighbouring blocks, share
    // their input columns
    const long long tile = xcd_logical_block() * 4 + (threadIdx.x >> 6);
    if (tile >= (long long)outer * mt * it) return;   // wave-uniform; no barrier follows
    const int m_t = (int)(tile % mt);
    const long long rest = tile / mt;
    const int i_t = (int)(rest % it), o = (int)(rest / it);
    const int lane = threadIdx.x & 63, r = lane & 15, q = lane >> 4;
    const int m = m_t * 16 + r;   // A row of this lane
    const int i = i_t * 16 + r;   // B column of this lane
    const float2 *src = in + (size_t)o * N * inner + (i < inner ? i : 0);
    const int step = (int)((4LL * m) % Nt);
    int idx = (int)(((long long)q * m) % Nt);
    // 16 input rows per stage, two register buffers in turn (as in
    // k_dft_inner).  A (row m, column n) and B (row n, column i) are
    // different elements: the window and the bounds of each are taken on its
    // own indices.
    const int N1 = N - 1;
    const float bi_ok = i < inner ? 1.0f : 0.0f;
    f32x4 dr0 = {0.f, 0.f, 0.f, 0.f}, di0 = dr0, dr1 = dr0, di1 = dr0;
    auto load = [&](float2 *buf, int n0) {
#pragma unroll
        for (int u = 0; u < 4; u++) buf[u] = src[(size_t)min(n0 + 4 * u + q, N1) * inner];
    };
    auto stage = [&](const float2 *buf, int n0) {
#pragma unroll
        for (int u = 0; u < 4; u++) {
            const int n = n0 + 4 * u + q;
            const float w = n < N ? (post ? 1.0f : wt[min(n, N1)]) : 0.0f;
            const float bw = n < N ? bi_ok : 0.0f;
            const float2 t = tw[idx];
            idx += step;
            if (idx >= Nt) idx -= Nt;
            if (u & 1) cmfma(t.x * w, t.y * w, buf[u].x * bw, buf[u].y * bw, dr1, di1);
            else cmfma(t.x * w, t.y * w, buf[u].x * bw, buf[u].y * bw, dr0, di0);
        }
    };
    float2 ba[4], bb[4];
    load(ba, 0);
    for (int n0 = 0; n0 < N; n0 += 32) {
        load(bb, n0 + 16);
        stage(ba, n0);
        load(ba, n0 + 32);
        if (n0 + 16 < N) stage(bb, n0 + 16);
    }
    const f32x4 dr = dr0 + dr1, di = di0 + di1;
    if (i >= inner) return;
#pragma unroll
    for (int j = 0; j < 4; j++) {
        const int mo = m_t * 16 + 4 * q + j;
        if (mo < M) {
            const float w = post ? wt[mo] : 1.0f;
            out[((size_t)o * M + mo) * inner + i] = make_float2(dr[j] * w, di[j] * w);
        }
    }
}

// ---- FFT stages (power-of-two axes) and the direct angle stage ------------
// For power-of-two lengths the range and Doppler DFTs run as Stockham FFTs
// (decimation in frequency, self-sorting: no bit reversal) on the VALU with
// the sequences held in LDS: O(N log N) work instead of the dense form's
// O(N^2), which leaves these stages bound by their memory traffic.  A radix-r
// stage with sub-length n (stride s = N / n, m = n / r) computes
//   y[q + s (r p + k)] = e^{sign 2 pi j k p / n} sum_{i < r} x[q + s (p + i m)] e^{sign 2 pi j i k / r}
// for p < m, q < s, k < r; radix-4 stages while 4 divides n, then one
// radix-2 stage if n = 2 is left.  The twiddle e^{sign 2 pi j k p / n} is the
// N-entry table's entry k p s (exact index).
constexpr int kFftLogTile = 10;
constexpr int kFftTile = 1 << kFftLogTile;   // complex elements per block (per LDS buffer)

__device__ __forceinline__ float2 cmul2(float2 a, float2 b) {
    return make_float2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
__device__ __forceinline__ float2 cadd2(float2 a, float2 b) { return make_float2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ float2 csub2(float2 a, float2 b) { return make_float2(a.x - b.x, a.y - b.y); }

// W independent sequences of length N = 2^logN in LDS, element n of
// sequence j at n * sn + j * sj; x and y are two buffers of the same layout.
// Returns the buffer holding the result.  Consecutive threads take
// consecutive butterflies of one sequence (sn = 1) or the same butterfly of
// consecutive sequences (sj = 1, JFAST): either way neighbouring lanes touch
// neighbouring LDS words.
// W is any count for the sequence-major form (JFAST false) and 2^logW for
// JFAST.
template <bool JFAST>
__device__ float2 *lds_fft(float2 *x, float2 *y, int logN, int W, int logW, int sn, int sj, const float2 *tw,
                           int sign) {
    int ls = 0;   // log2 of the stride s
    while (logN - ls >= 2) {   // radix 4: n = N / s divisible by 4
        const int s = 1 << ls, lm = logN - ls - 2, m = 1 << lm;
        const int total = W << (logN - 2);
        for (int b = threadIdx.x; b < total; b += blockDim.x) {
            const int j = JFAST ? (b & (W - 1)) : (b >> (logN - 2));
            const int r = JFAST ? (b >> logW) : (b & ((1 << (logN - 2)) - 1));
            const int p = r >> ls, q = r & (s - 1);
            const int base = (q + s * p) * sn + j * sj, step = (s * m) * sn;
            const float2 a = x[base], bb = x[base + step], c = x[base + 2 * step], d = x[base + 3 * step];
            const float2 apc = cadd2(a, c), amc = csub2(a, c), bpd = cadd2(bb, d), t = csub2(bb, d);
            // sign * j * (b - d)
            const float2 jt = sign < 0 ? make_float2(t.y, -t.x) : make_float2(-t.y, t.x);
            const int o = (q + s * 4 * p) * sn + j * sj, os = s * sn;
            y[o] = cadd2(apc, bpd);
            y[o + os] = cmul2(cadd2(amc, jt), tw[(p << ls)]);
            y[o + 2 * os] = cmul2(csub2(apc, bpd), tw[(2 * p) << ls]);
            y[o + 3 * os] = cmul2(csub2(amc, jt), tw[(3 * p) << ls]);
        }
        __syncthreads();
        float2 *tmp = x;
        x = y;
        y = tmp;
        ls += 2;
    }
    if (logN - ls == 1) {   // radix 2, n = 2: m = 1, p = 0, no twiddle
        const int s = 1 << ls;
        const int total = W << (logN - 1);
        for (int b = threadIdx.x; b < total; b += blockDim.x) {
            const int j = JFAST ? (b & (W - 1)) : (b >> (logN - 1));
            const int q = JFAST ? (b >> logW) : (b & (s - 1));
            const float2 a = x[q * sn + j * sj], c = x[(q + s) * sn + j * sj];
            y[q * sn + j * sj] = cadd2(a, c);
            y[(q + s) * sn + j * sj] = csub2(a, c);
        }
        __syncthreads();
        x = y;
    }
    return x;
}

// LDS tables of an FFT block: N twiddles e^{sign 2 pi j k / N}, then the
// window over the N samples (single precision: sincospi of an exact
// argument 2k / N).
__device__ void fft_tables(float2 *tw, float *wt, int N, int sign, int window) {
    for (int k = threadIdx.x; k < N; k += blockDim.x) {
        float sn, cs;
        sincospif(2.0f * (float)k / (float)N, &sn, &cs);
        tw[k] = make_float2(cs, sign * sn);
        wt[k] = (window == 1 && N > 1) ? 0.5f - 0.5f * cospif(2.0f * (float)k / (float)(N - 1)) : 1.0f;
    }
    __syncthreads();
}

// FFT along the innermost axis: [rows][N] -> [rows][N], R = kFftTile / N rows
// per block; the window multiplies the input (post = 0) or the output.
// The global loads of a block are issued before its tables are built, so
// the table work hides under their latency.
constexpr int kFftThreads = 256;
constexpr int kFftPer = kFftTile / kFftThreads;

__global__ __launch_bounds__(kFftThreads) void k_fft_inner(const float2 *in, float2 *out, int rows, int logN,
                                                           int sign, int window, int post) {
    extern __shared__ float2 sm[];
    const int N = 1 << logN, R = kFftTile >> logN;
    float2 *tw = sm;
    float *wt = reinterpret_cast<float *>(sm + N);
    float2 *b0 = sm + N + (N + 1) / 2, *b1 = b0 + kFftTile;
    const long long row0 = (long long)blockIdx.x * R;
    float2 v[kFftPer];
#pragma unroll
    for (int u = 0; u < kFftPer; u++) {
        const int i = threadIdx.x + u * kFftThreads, r = i >> logN, n = i & (N - 1);
        v[u] = row0 + r < rows ? in[(row0 + r) * N + n] : make_float2(0.0f, 0.0f);
    }
    fft_tables(tw, wt, N, sign, window);
#pragma unroll
    for (int u = 0; u < kFftPer; u++) {
        const int i = threadIdx.x + u * kFftThreads, n = i & (N - 1);
        b0[i] = post ? v[u] : make_float2(v[u].x * wt[n], v[u].y * wt[n]);
    }
    __syncthreads();
    const float2 *res = lds_fft<false>(b0, b1, logN, R, 0, 1, N, tw, sign);
    for (int i = threadIdx.x; i < kFftTile; i += blockDim.x) {
        const int r = i >> logN, k = i & (N - 1);
        if (row0 + r < rows) {
            float2 v = res[i];
            if (post) v = make_float2(v.x * wt[k], v.y * wt[k]);
            out[(row0 + r) * N + k] = v;
        }
    }
}

// FFT along a middle axis: [outer][N][inner] -> [outer][N][inner].  A block
// takes one outer index and W = kFftTile / N consecutive inner columns (the
// loads and stores run along the inner axis).
__global__ __launch_bounds__(kFftThreads) void k_fft_mid(const float2 *in, float2 *out, int outer, int logN,
                                                         int inner, int sign, int window, int post) {
    extern __shared__ float2 sm[];
    const int N = 1 << logN, logW = kFftLogTile - logN, W = 1 << logW;
    float2 *tw = sm;
    float *wt = reinterpret_cast<float *>(sm + N);
    float2 *b0 = sm + N + (N + 1) / 2, *b1 = b0 + kFftTile;
    const int ct = (inner + W - 1) / W;
    const int o = blockIdx.x / ct, i0 = (blockIdx.x % ct) * W;
    const float2 *src = in + (size_t)o * N * inner;
    float2 *dst = out + (size_t)o * N * inner;
    float2 v[kFftPer];
#pragma unroll
    for (int u = 0; u < kFftPer; u++) {
        const int i = threadIdx.x + u * kFftThreads, n = i >> logW, j = i & (W - 1);
        v[u] = i0 + j < inner ? src[(size_t)n * inner + i0 + j] : make_float2(0.0f, 0.0f);
    }
    fft_tables(tw, wt, N, sign, window);
#pragma unroll
    for (int u = 0; u < kFftPer; u++) {
        const int i = threadIdx.x + u * kFftThreads, n = i >> logW;
        b0[i] = post ? v[u] : make_float2(v[u].x * wt[n], v[u].y * wt[n]);
    }
    __syncthreads();
    const float2 *res = lds_fft<true>(b0, b1, logN, W, logW, W, 1, tw, sign);
    for (int i = threadIdx.x; i < kFftTile; i += blockDim.x) {
        const int k = i >> logW, j = i & (W - 1);
        if (i0 + j < inner) {
            float2 v = res[i];
            if (post) v = make_float2(v.x * wt[k], v.y * wt[k]);
            dst[(size_t)k * inner + i0 + j] = v;
        }
    }
}

constexpr int kAngleVMax = 32;   // antennas of the direct angle stage (registers)
constexpr int kAngleGroup = 8;   // angle bins per thread of the forward stage

// acc_k = acc_k w_k + y for the thread's kAngleGroup angle bins: independent
// complex multiply-adds, so the chains interleave.
__device__ __forceinline__ void horner_step(float2 (&acc)[kAngleGroup], const float2 (&w)[kAngleGroup], float2 y) {
#pragma unroll
    for (int k = 0; k < kAngleGroup; k++) {
        const float nr = fmaf(acc[k].x, w[k].x, fmaf(-acc[k].y, w[k].y, y.x));
        acc[k].y = fmaf(acc[k].x, w[k].y, fmaf(acc[k].y, w[k].x, y.y));
        acc[k].x = nr;
    }
}

// Forward angle stage of a linear array as a direct DFT:
//   out[a][e] = sum_{v < V} w_a^v y[v][e],  w_a = e^{-2 pi j a / Na},
// by Horner's rule in w_a (V - 1 complex multiply-adds per output).  A thread
// owns one (chirp, sample) cell e (coalesced along e) and the block row's
// kAngleGroup consecutive angle bins.  The antenna values sit in registers.
// EXACT instances have V = VB and straight-line steps; otherwise each
// unrolled step is guarded by the wave-uniform test v < V (a branch, so no
// step runs for antennas beyond V; VB is only the register bound).
template <int VB, bool EXACT>
__global__ __launch_bounds__(256) void k_angle(const float2 *y, float2 *out, int V, int Na, long long CS) {
    __shared__ float2 w_s[kAngleGroup];
    const int a0 = blockIdx.y * kAngleGroup;
    if (threadIdx.x < kAngleGroup) {
        float sn, cs;
        sincospif(2.0f * (float)(a0 + (int)threadIdx.x) / (float)Na, &sn, &cs);
        w_s[threadIdx.x] = make_float2(cs, -sn);
    }
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    const bool live = e < CS;
    float2 yv[VB];
#pragma unroll
    for (int v = 0; v < VB; v++)
        if (EXACT || v < V) yv[v] = live ? y[(size_t)v * CS + e] : make_float2(0.0f, 0.0f);
    __syncthreads();
    if (!live) return;
    float2 w[kAngleGroup], acc[kAngleGroup];
#pragma unroll
    for (int k = 0; k < kAngleGroup; k++) {
        w[k] = w_s[k];
        acc[k] = make_float2(0.0f, 0.0f);
    }
#pragma unroll
    for (int v = VB - 1; v >= 0; v--)
        if (EXACT || v < V) horner_step(acc, w, yv[v]);
#pragma unroll
    for (int k = 0; k < kAngleGroup; k++)
        if (a0 + k < Na) out[(size_t)(a0 + k) * CS + e] = acc[k];
}

// Conjugate transpose of the angle stage: out[v][e] = sum_a
// e^{+2 pi j (a v mod Na) / Na} y[a][e] for every v < V, twiddles by exact
// index from an LDS table; one thread per cell.
template <int VB>
__global__ __launch_bounds__(256) void k_angle_adj(const float2 *y, float2 *out, int V, int Na, long long CS) {
    extern __shared__ float2 tw[];
    for (int k = threadIdx.x; k < Na; k += blockDim.x) {
        float sn, cs;
        sincospif(2.0f * (float)k / (float)Na, &sn, &cs);
        tw[k] = make_float2(cs, sn);
    }
    __syncthreads();
    const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
    if (e >= CS) return;
    float2 acc[VB];
#pragma unroll
    for (int v = 0; v < VB; v++) acc[v] = make_float2(0.0f, 0.0f);
    for (int a = 0; a < Na; a++) {
        const float2 x = y[(size_t)a * CS + e];
        int idx = 0;
#pragma unroll
        for (int v = 0; v < VB; v++) {
            if (v >= V) continue;
            const float2 w = tw[idx];
            acc[v].x = fmaf(w.x, x.x, fmaf(-w.y, x.y, acc[v].x));
            acc[v].y = fmaf(w.x, x.y, fmaf(w.y, x.x, acc[v].y));
            idx += a;
            if (idx >= Na) idx -= Na;
        }
    }
#pragma unroll
    for (int v = 0; v < VB; v++)
        if (v < V) out[(size_t)v * CS + e] = acc[v];
}

// ---- Forward range FFT + angle DFT, fused (256 samples) -------------------
// cos and sin of 2 pi m / 16, m < 16
constexpr float kCos16[16] = {1.0f, 0.92387953f, 0.70710678f, 0.38268343f, 0.0f, -0.38268343f,
                              -0.70710678f, -0.92387953f, -1.0f, -0.92387953f, -0.70710678f, -0.38268343f,
                              0.0f, 0.38268343f, 0.70710678f, 0.92387953f};
constexpr float kSin16[16] = {0.0f, 0.38268343f, 0.70710678f, 0.92387953f, 1.0f, 0.92387953f,
                              0.70710678f, 0.38268343f, 0.0f, -0.38268343f, -0.70710678f, -0.92387953f,
                              -1.0f, -0.92387953f, -0.70710678f, -0.38268343f};

// Forward 4-point DFT (e^{-2 pi j n k / 4}) of a0..a3, in place.
__device__ __forceinline__ void dft4(float2 &a0, float2 &a1, float2 &a2, float2 &a3) {
    const float2 t0 = cadd2(a0, a2), t1 = csub2(a0, a2), t2 = cadd2(a1, a3), t3 = csub2(a1, a3);
    a0 = cadd2(t0, t2);
    a2 = csub2(t0, t2);
    a1 = make_float2(t1.x + t3.y, t1.y - t3.x);   // t1 - j t3
    a3 = make_float2(t1.x - t3.y, t1.y + t3.x);   // t1 + j t3
}

// Forward 16-point DFT of x in registers, result in natural order:
// n = 4 n1 + n2, k = k1 + 4 k2; a 4-point DFT over n1 for each n2, the
// twiddle e^{-2 pi j n2 k1 / 16}, then a 4-point DFT over n2 for each k1.
__device__ __forceinline__ void dft16(float2 (&x)[16]) {
#pragma unroll
    for (int n2 = 0; n2 < 4; n2++) dft4(x[n2], x[4 + n2], x[8 + n2], x[12 + n2]);   // x[4 k1 + n2]
#pragma unroll
    for (int n2 = 1; n2 < 4; n2++)
#pragma unroll
        for (int k1 = 1; k1 < 4; k1++) {
            const int m = n2 * k1;
            x[4 * k1 + n2] = cmul2(x[4 * k1 + n2], make_float2(kCos16[m], -kSin16[m]));
        }
    float2 y[16];
#pragma unroll
    for (int k1 = 0; k1 < 4; k1++) {
        float2 a0 = x[4 * k1], a1 = x[4 * k1 + 1], a2 = x[4 * k1 + 2], a3 = x[4 * k1 + 3];
        dft4(a0, a1, a2, a3);   // over n2 -> k2
        y[k1] = a0;
        y[k1 + 4] = a1;
        y[k1 + 8] = a2;
        y[k1 + 12] = a3;
    }
#pragma unroll
    for (int i = 0; i < 16; i++) x[i] = y[i];
}

// Forward 2- and 8-point DFTs in registers (natural order); the 8-point one
// as n = 2 n1 + n2, k = k1 + 4 k2.
__device__ __forceinline__ void dft2(float2 &a0, float2 &a1) {
    const float2 t = a0;
    a0 = cadd2(t, a1);
    a1 = csub2(t, a1);
}

template <int P>
__device__ __forceinline__ void dft_small(float2 (&v)[P]);
template <>
__device__ __forceinline__ void dft_small<2>(float2 (&v)[2]) { dft2(v[0], v[1]); }
template <>
__device__ __forceinline__ void dft_small<4>(float2 (&v)[4]) { dft4(v[0], v[1], v[2], v[3]); }
template <>
__device__ __forceinline__ void dft_small<8>(float2 (&v)[8]) {
    dft4(v[0], v[2], v[4], v[6]);   // n2 = 0: v[2 k1]
    dft4(v[1], v[3], v[5], v[7]);   // n2 = 1: v[2 k1 + 1]
#pragma unroll
    for (int k1 = 1; k1 < 4; k1++) v[2 * k1 + 1] = cmul2(v[2 * k1 + 1], make_float2(kCos16[2 * k1], -kSin16[2 * k1]));
    float2 y[8];
#pragma unroll
    for (int k1 = 0; k1 < 4; k1++) {
        y[k1] = cadd2(v[2 * k1], v[2 * k1 + 1]);
        y[k1 + 4] = csub2(v[2 * k1], v[2 * k1 + 1]);
    }
#pragma unroll
    for (int i = 0; i < 8; i++) v[i] = y[i];
}
template <>
__device__ __forceinline__ void dft_small<16>(float2 (&v)[16]) { dft16(v); }

// Forward Doppler FFT (windowed, [V][C][S] -> [V][C][S]) for C = 16 P chirps:
// chirp n = t + P m.  Thread (column s, t) holds its 16 values in registers,
// takes the 16-point DFT over m and multiplies by e^{-2 pi j t k1 / C}; after
// one exchange through LDS (column index fastest, so both sides are
// conflict-free) the same thread takes the P-point DFTs over t of its 16 / P
// values of k1, giving Doppler bin k1 + 16 k2.  Lanes run along the samples,
// so loads and stores are coalesced rows.
constexpr int kDopThreads = 128;

template <int P>
__global__ __launch_bounds__(kDopThreads) void k_doppler(const float2 *in, float2 *out, int S, int window) {
    constexpr int C = 16 * P, NCOL = kDopThreads / P, PER = 16 / P;
    __shared__ float2 tw[C];
    __shared__ float wt[C];
    __shared__ float2 ex[16 * P * NCOL];
    const int tid = threadIdx.x, j = tid % NCOL, t = tid / NCOL;
    const int sblocks = (S + NCOL - 1) / NCOL;
    const int v = blockIdx.x / sblocks, s = (blockIdx.x % sblocks) * NCOL + j;
    const bool live = s < S;
    const float2 *src = in + (size_t)v * C * S;
    float2 x[16];
#pragma unroll
    for (int m = 0; m < 16; m++) x[m] = live ? src[(size_t)(t + P * m) * S + s] : make_float2(0.0f, 0.0f);
    for (int i = tid; i < C; i += kDopThreads) {
        float sn, cs;
        sincospif(2.0f * (float)i / (float)C, &sn, &cs);
        tw[i] = make_float2(cs, -sn);
        wt[i] = window == 1 ? 0.5f - 0.5f * cospif(2.0f * (float)i / (float)(C - 1)) : 1.0f;
    }
    __syncthreads();
#pragma unroll
    for (int m = 0; m < 16; m++) {
        const float w = wt[t + P * m];
        x[m] = make_float2(x[m].x * w, x[m].y * w);
    }
    dft16(x);
#pragma unroll
    for (int k1 = 0; k1 < 16; k1++) ex[(k1 * P + t) * NCOL + j] = k1 == 0 ? x[0] : cmul2(x[k1], tw[t * k1]);
    __syncthreads();
    float2 *dst = out + (size_t)v * C * S;
#pragma unroll
    for (int q = 0; q < PER; q++) {
        const int k1 = t * PER + q;
        float2 u[P];
#pragma unroll
        for (int tt = 0; tt < P; tt++) u[tt] = ex[(k1 * P + tt) * NCOL + j];
        dft_small<P>(u);
        if (live) {
#pragma unroll
            for (int k2 = 0; k2 < P; k2++) dst[(size_t)(k1 + 16 * k2) * S + s] = u[k2];
        }
    }
}

// A block takes Doppler bin k (the Doppler stage has already run; the DFT
// axes commute): the V <= 16 rows in[v][k][*] of 256 samples, windowed.  The
// range FFT splits each row as n = t + 16 m: thread (row r, t) holds its 16
// values in registers, takes the 16-point DFT over m, multiplies by
// e^{-2 pi j t k1 / 256} and leaves them in LDS; thread (r, k1) then takes
// the 16-point DFT over t, giving range bin k1 + 16 k2.  LDS rows are padded
// (kRaRow) and the exchange uses a stride of 17, so neither access pattern
// has lanes on one bank.  Then one thread per range bin s writes out[a][k][s]
// for the block's kRangeAngleBins angle bins (coalesced rows of 256 values).
// When Na = 16 q, bins a = a1 + q a2 (a2 < 16) are the 16-point DFT over v
// (zero-padded) of y_v e^{-2 pi j a1 v / Na}; block row y takes a1 in
// [y kRaSplit, (y + 1) kRaSplit).  Other angle counts take kRangeAngleBins
// consecutive bins per block row by Horner's rule over the antennas, in
// passes of kAngleGroup bins.
constexpr int kRaS = 256;              // samples per row
constexpr int kRaRow = 16 * 17;        // padded LDS row (complex values)
constexpr int kRaVMax = 16;            // rows (antennas) of one block
constexpr int kRangeAngleBins = 16;    // angle bins per block
constexpr int kRaSplit = kRangeAngleBins / 16;   // 16-point angle DFTs per block (split form)

template <int VB, bool EXACT>
__global__ __launch_bounds__(256) void k_range_angle(const float2 *in, float2 *out, int V, int C, int Na,
                                                     int window) {
    extern __shared__ float2 sm[];
    float2 *tw = sm;                              // e^{-2 pi j i / 256}
    float2 *wa = tw + kRaS;                       // angle steps, or the antenna twiddles of a1
    float *wt = reinterpret_cast<float *>(wa + kRangeAngleBins);
    float2 *buf = wa + kRangeAngleBins + kRaS / 2;   // V rows of kRaRow
    const int k = blockIdx.x, a_lo = blockIdx.y * kRangeAngleBins, tid = threadIdx.x;
    const int r = tid >> 4, t = tid & 15;
    const bool fft = r < V;
    float2 x[16];
    if (fft) {
        const float2 *row = in + ((size_t)r * C + k) * kRaS;
#pragma unroll
        for (int m = 0; m < 16; m++) x[m] = row[t + 16 * m];
    }
    {
        float sn, cs;
        sincospif(2.0f * (float)tid / (float)kRaS, &sn, &cs);
        tw[tid] = make_float2(cs, -sn);
        wt[tid] = window == 1 ? 0.5f - 0.5f * cospif(2.0f * (float)tid / (float)(kRaS - 1)) : 1.0f;
        if (tid < kRangeAngleBins) {
            // split form: e^{-2 pi j a1 v / Na} for antenna v = tid % 16 of the
            // block's a1 = blockIdx.y kRaSplit + tid / 16
            const int e = Na % 16 == 0 ? ((int)blockIdx.y * kRaSplit + tid / 16) * (tid % 16) % Na : a_lo + tid;
            sincospif(2.0f * (float)e / (float)Na, &sn, &cs);
            wa[tid] = make_float2(cs, -sn);
        }
    }
    __syncthreads();
    if (fft) {
#pragma unroll
        for (int m = 0; m < 16; m++) {
            const float w = wt[t + 16 * m];
            x[m] = make_float2(x[m].x * w, x[m].y * w);
        }
        dft16(x);
#pragma unroll
        for (int k1 = 0; k1 < 16; k1++)
            buf[r * kRaRow + k1 * 17 + t] = k1 == 0 ? x[0] : cmul2(x[k1], tw[t * k1]);
    }
    __syncthreads();
    if (fft) {
#pragma unroll
        for (int u = 0; u < 16; u++) x[u] = buf[r * kRaRow + t * 17 + u];   // k1 = t, over u = t'
    }
    __syncthreads();
    if (fft) {
        dft16(x);
#pragma unroll
        for (int k2 = 0; k2 < 16; k2++) buf[r * kRaRow + t + 16 * k2] = x[k2];   // range bin t + 16 k2
    }
    __syncthreads();
    const int sb = tid;   // range bin
    float2 yv[VB];
#pragma unroll
    for (int a = 0; a < VB; a++)
        if (EXACT || a < V) yv[a] = buf[a * kRaRow + sb];
    const size_t plane = (size_t)C * kRaS;
    if (Na % 16 == 0) {
        static_assert(kRangeAngleBins % 16 == 0 && VB <= 16, "split form: 16-point DFTs over the antennas");
        const int q = Na / 16;
        for (int j = 0; j < kRaSplit; j++) {
            const int a1 = (int)blockIdx.y * kRaSplit + j;
            if (a1 >= q) break;
            float2 z[16];
#pragma unroll
            for (int v = 0; v < 16; v++)
                z[v] = v >= VB || !(EXACT || v < V) ? make_float2(0.0f, 0.0f)
                                                     : v == 0 ? yv[0] : cmul2(yv[v], wa[16 * j + v]);
            dft16(z);
#pragma unroll
            for (int a2 = 0; a2 < 16; a2++) out[(size_t)(a1 + q * a2) * plane + (size_t)k * kRaS + sb] = z[a2];
        }
        return;
    }
    for (int g = 0; g < kRangeAngleBins; g += kAngleGroup) {
        const int a0 = a_lo + g;
        if (a0 >= Na) break;
        float2 w[kAngleGroup], acc[kAngleGroup];
#pragma unroll
        for (int q = 0; q < kAngleGroup; q++) {
            w[q] = wa[g + q];
            acc[q] = make_float2(0.0f, 0.0f);
        }
#pragma unroll
        for (int a = VB - 1; a >= 0; a--)
            if (EXACT || a < V) horner_step(acc, w, yv[a]);
#pragma unroll
        for (int q = 0; q < kAngleGroup; q++)
            if (a0 + q < Na) out[(size_t)(a0 + q) * plane + (size_t)k * kRaS + sb] = acc[q];
    }
}

static size_t range_angle_lds(int V) {
    return sizeof(float2) * ((size_t)kRaS + kRangeAngleBins + kRaS / 2 + (size_t)V * kRaRow);
}

// ---- CFAR ------------------------------------------------------------------
// Power map P[e] = sum_a |X[a][e]|^2 and its argmax over a (lowest index on
// ties).  The angle range is split over kPowSplit block rows and 4 lanes per
// cell, so a cube with thousands of angle bins (planar arrays) still fills
// the chip; partials are combined in a fixed order.
constexpr int kPowSplit = 16;

__global__ __launch_bounds__(256) void k_power_part(const float2 *X, int Na, int plane, float *psum, float *pmax,
                                                    int *parg) {
    __shared__ float ss[4][64], sm[4][64];
    __shared__ int sa[4][64];
    const int cl = threadIdx.x & 63, g = threadIdx.x >> 6;
    const int e = blockIdx.x * 64 + cl;
    const int per = (Na + kPowSplit - 1) / kPowSplit;
    const int a0 = blockIdx.y * per, a1 = min(Na, a0 + per);
    float acc = 0.0f, best = -1.0f;
    int ba = a0;
    if (e < plane) {
        for (int a = a0 + g; a < a1; a += 4) {
            const float2 x = X[(size_t)a * plane + e];
            const float q = x.x * x.x + x.y * x.y;
            acc += q;
            if (q > best) {
                best = q;
                ba = a;
            }
        }
    }
    ss[g][cl] = acc;
    sm[g][cl] = best;
    sa[g][cl] = ba;
    __syncthreads();
    if (g == 0 && e < plane) {
        float sum = ss[0][cl], m = sm[0][cl];
        int am = sa[0][cl];
        for (int k = 1; k < 4; k++) {
            sum += ss[k][cl];
            if (sm[k][cl] > m || (sm[k][cl] == m && sa[k][cl] < am)) {
                m = sm[k][cl];
                am = sa[k][cl];
            }
        }
        psum[(size_t)blockIdx.y * plane + e] = sum;
        pmax[(size_t)blockIdx.y * plane + e] = m;
        parg[(size_t)blockIdx.y * plane + e] = am;
    }
}

__global__ void k_power_final(int plane, const float *psum, const float *pmax, const int *parg, float *P,
                              int *am) {
    const int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= plane) return;
    float sum = 0.0f, m = -1.0f;
    int a = 0;
    for (int k = 0; k < kPowSplit; k++) {
        sum += psum[(size_t)k * plane + e];
        const float mk = pmax[(size_t)k * plane + e];
        const int ak = parg[(size_t)k * plane + e];
        if (mk > m || (mk == m && ak < a)) {
            m = mk;
            a = ak;
        }
    }
    P[e] = sum;
    am[e] = a;
}

__global__ void k_cfar_cells(const float *P, int C, int S, int guard, int train, double pfa, float *ratio) {
    int e = blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= C * S) return;
    const int d = e / S, r = e % S, w = guard + train;
    float sum = 0.0f;
    int nt = 0;
    for (int dd = -w; dd <= w; dd++) {
        int d2 = ((d + dd) % C + C) % C;
        for (int rr = -w; rr <= w; rr++) {
            if (abs(dd) <= guard && abs(rr) <= guard) continue;
            int r2 = r + rr;
            if (r2 < 0 || r2 >= S) continue;
            sum += P[(size_t)d2 * S + r2];
            nt++;
        }
    }
    float rt = 0.0f;
    if (nt > 0) {
        double alpha = nt * (pow(pfa, -1.0 / nt) - 1.0);
        double thr = alpha * (double)sum / nt;
        rt = thr > 0.0 ? (float)((double)P[e] / thr) : (P[e] > 0.0f ? INFINITY : 0.0f);
    }
    ratio[e] = rt;
}

// ordered compaction of detections (ratio > 1), one block
__global__ __launch_bounds__(1024) void k_cfar_compact(const float *ratio, const int *am, int n, int S,
                                                       int32_t *points, float *pratio, int maxp,
                                                       int32_t *npts) {
    __shared__ int wsum[16];
    __shared__ int base;
    const int t = threadIdx.x, lane = t & 63, w = t >> 6;
    if (t == 0) base = 0;
    __syncthreads();
    for (int e0 = 0; e0 < n; e0 += 1024) {
        int e = e0 + t;
        int hit = (e < n && ratio[e] > 1.0f) ? 1 : 0;
        uint64_t m = __ballot(hit);
        int before = __popcll(m & ((lane == 0) ? 0ull : (~0ull >> (64 - lane))));
        if (lane == 0) wsum[w] = __popcll(m);
        __syncthreads();
        int off = base;
        for (int i = 0; i < w; i++) off += wsum[i];
        int pos = off + before;
        if (hit && pos < maxp) {
            points[4 * pos] = e % S;
            points[4 * pos + 1] = e / S;
            points[4 * pos + 2] = am[e];
            points[4 * pos + 3] = 0;
            if (pratio) pratio[pos] = ratio[e];
        }
        __syncthreads();
        if (t == 0) {
            int tot = 0;
            for (int i = 0; i < 16; i++) tot += wsum[i];
            base += tot;
        }
        __syncthreads();
    }
    if (t == 0) *npts = base;
}

// Detections -> world points.  Range bin r: beat frequency r f_s / S = mu tau,
// R = c tau / 2; Doppler bin d: d / C cycles per chirp = f_c T_c taudot,
// v = c taudot / 2; angle bins over a lambda/2 array with DFT sign -1: the
// element phase step is -pi u, so u = -2 a_s / N with a_s the signed bin.
struct CloudArgs {
    const int32_t *points;
    const int32_t *n_points;
    int32_t max_points;
    int32_t n_ax, n_ay;
    double o[3], rot[9];
    double fc, slope, fs, tc;
    int32_t S, C;
    float4 *out;
};

__device__ __forceinline__ double signed_bin(int a, int N) { return a >= (N + 1) / 2 ? (double)(a - N) : (double)a; }

__global__ void k_cloud(CloudArgs a) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= a.max_points) return;
    if (i >= min(a.n_points[0], a.max_points)) {
        a.out[i] = make_float4(NAN, NAN, NAN, NAN);
        return;
    }
    const int rb = a.points[4 * i], db = a.points[4 * i + 1], ang = a.points[4 * i + 2];
    const double R = kC0 * (rb * a.fs / ((double)a.S * a.slope)) / 2.0;
    const int ax = ang % a.n_ax, ay = ang / a.n_ax;
    const double ux = -2.0 * signed_bin(ax, a.n_ax) / a.n_ax;
    const double uy = a.n_ay > 1 ? -2.0 * signed_bin(ay, a.n_ay) / a.n_ay : 0.0;
    const double uz2 = 1.0 - ux * ux - uy * uy;
    const double p[3] = {R * ux, R * uy, uz2 > 0.0 ? R * sqrt(uz2) : 0.0};
    double w[3];
    for (int k = 0; k < 3; k++) w[k] = a.o[k] + a.rot[3 * k] * p[0] + a.rot[3 * k + 1] * p[1] + a.rot[3 * k + 2] * p[2];
    const double tdot = signed_bin(db, a.C) / ((double)a.C * a.fc * a.tc);
    a.out[i] = make_float4((float)w[0], (float)w[1], (float)w[2], (float)(kC0 * tdot / 2.0));
}

// ---- angle peaks of detected cells ------------------------------------------
// q[a] = |X[a][d][r]|^2 of a detection's cell; a is a peak when q[a] >= rel *
// max_a q, q[a] > q[b] for ring / torus neighbours b < a and q[a] >= q[b] for
// b > a.  Points are written detection-major, angle ascending (ordered scan).
struct PeakArgs {
    const float2 *X;
    int32_t n_ax, n_ay, plane, S;
    const int32_t *det;
    const int32_t *n_det;
    int32_t max_det;
    float rel;
    float *qmax;         // [max_det]
    int32_t *blk;        // [nblk] counts, then exclusive offsets
    int32_t nblk;
    int32_t *points;
    int32_t max_points;
    int32_t *n_points;
};

__device__ __forceinline__ float cell_q(const PeakArgs &a, size_t e, int ang) {
    const float2 x = a.X[(size_t)ang * a.plane + e];
    return x.x * x.x + x.y * x.y;
}

__global__ __launch_bounds__(256) void k_peak_max(PeakArgs a) {
    const int i = blockIdx.x;
    const int nd = min(a.n_det[0], a.max_det);
    if (i >= nd) return;
    __shared__ float sh[256];
    const int r = a.det[4 * i], d = a.det[4 * i + 1];
    if (r < 0 || r >= a.S || d < 0 || d >= a.plane / a.S) {   // not a cell of this cube
        if (threadIdx.x == 0) a.qmax[i] = INFINITY;
        return;
    }
    const size_t e = (size_t)d * a.S + r;
    const int Na = a.n_ax * a.n_ay;
    float m = 0.0f;
    for (int ang = threadIdx.x; ang < Na; ang += 256) m = fmaxf(m, cell_q(a, e, ang));
    sh[threadIdx.x] = m;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] = fmaxf(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) a.qmax[i] = sh[0];
}

__device__ bool is_peak(const PeakArgs &a, long long g) {
    const int Na = a.n_ax * a.n_ay;
    const int i = (int)(g / Na), ang = (int)(g % Na);
    if (i >= min(a.n_det[0], a.max_det)) return false;
    const int r = a.det[4 * i], d = a.det[4 * i + 1];
    if (r < 0 || r >= a.S || d < 0 || d >= a.plane / a.S) return false;
    const size_t e = (size_t)d * a.S + r;
    const float q = cell_q(a, e, ang);
    if (!(q >= a.rel * a.qmax[i]) || q <= 0.0f) return false;
    const int ax = ang % a.n_ax, ay = ang / a.n_ax;
    const int ylo = a.n_ay > 1 ? -1 : 0, yhi = a.n_ay > 1 ? 1 : 0;
    for (int dy = ylo; dy <= yhi; dy++)
        for (int dx = -1; dx <= 1; dx++) {
            if (dx == 0 && dy == 0) continue;
            const int b = ((ay + dy + a.n_ay) % a.n_ay) * a.n_ax + (ax + dx + a.n_ax) % a.n_ax;
            if (b == ang) continue;
            const float qb = cell_q(a, e, b);
            if (b < ang ? !(q > qb) : !(q >= qb)) return false;
        }
    return true;
}

__global__ __launch_bounds__(256) void k_peak_count(PeakArgs a) {
    __shared__ int sh[4];
    const long long g = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long total = (long long)a.max_det * a.n_ax * a.n_ay;
    int f = (g < total && is_peak(a, g)) ? 1 : 0;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    f = __popcll(__ballot(f));
    if (lane == 0) sh[w] = f;
    __syncthreads();
    if (threadIdx.x == 0) a.blk[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

__global__ __launch_bounds__(1024) void k_peak_scan(PeakArgs a) {
    __shared__ int part[1024];
    const int t = threadIdx.x, nb = a.nblk;
    const int chunk = (nb + 1023) / 1024;
    const int b = t * chunk, e = min(nb, b + chunk);
    int s = 0;
    for (int i = b; i < e; i++) s += a.blk[i];
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
        int x = a.blk[i];
        a.blk[i] = run;
        run += x;
    }
    if (t == 1023) *a.n_points = part[1023];
}

__global__ __launch_bounds__(256) void k_peak_write(PeakArgs a) {
    __shared__ int sh[4];
    const long long g = (long long)blockIdx.x * 256 + threadIdx.x;
    const long long total = (long long)a.max_det * a.n_ax * a.n_ay;
    const bool f = g < total && is_peak(a, g);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const uint64_t m = __ballot(f);
    if (lane == 0) sh[w] = __popcll(m);
    __syncthreads();
    int off = a.blk[blockIdx.x];
    for (int k = 0; k < w; k++) off += sh[k];
    const int pos = off + __popcll(m & ((1ull << lane) - 1ull));
    if (f && pos < a.max_points) {
        const int Na = a.n_ax * a.n_ay;
        const int i = (int)(g / Na), ang = (int)(g % Na);
        a.points[4 * pos] = a.det[4 * i];
        a.points[4 * pos + 1] = a.det[4 * i + 1];
        a.points[4 * pos + 2] = ang;
        a.points[4 * pos + 3] = 0;
    }
}

}  // namespace

size_t peaks_scratch_bytes(int max_det, int Na) {
    Carver cv(nullptr);
    cv.take<float>((size_t)std::max(1, max_det));
    const long long total = (long long)max_det * Na;
    cv.take<int32_t>((size_t)std::max(1LL, (total + 255) / 256));
    return align_up(cv.off, 256);
}

int peaks_launch(const float2 *X, int n_ax, int n_ay, int C, int S, const int32_t *det, const int32_t *n_det,
                 int max_det, float rel, int32_t *points, int max_points, int32_t *n_points, void *scratch,
                 hipStream_t s) {
    PeakArgs a;
    Carver cv(scratch);
    a.X = X;
    a.n_ax = n_ax;
    a.n_ay = n_ay;
    a.plane = C * S;
    a.S = S;
    a.det = det;
    a.n_det = n_det;
    a.max_det = max_det;
    a.rel = rel;
    a.qmax = cv.take<float>((size_t)std::max(1, max_det));
    const long long total = (long long)max_det * n_ax * n_ay;
    a.nblk = (int)std::max(1LL, (total + 255) / 256);
    a.blk = cv.take<int32_t>((size_t)a.nblk);
    a.points = points;
    a.max_points = max_points;
    a.n_points = n_points;
    if (max_det > 0) hipLaunchKernelGGL(k_peak_max, dim3(max_det), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_peak_count, dim3(a.nblk), dim3(256), 0, s, a);
    hipLaunchKernelGGL(k_peak_scan, dim3(1), dim3(1024), 0, s, a);
    hipLaunchKernelGGL(k_peak_write, dim3(a.nblk), dim3(256), 0, s, a);
    SBR_LAUNCHED();
    return SBR_OK;
}

int cloud_launch(const int32_t *points, const int32_t *n_points, int32_t max_points, const RadarDev &rd,
                 const ChirpDev &cd, int32_t n_ax, int32_t n_ay, float *out, hipStream_t s) {
    if (max_points == 0) return SBR_OK;
    CloudArgs a;
    a.points = points;
    a.n_points = n_points;
    a.max_points = max_points;
    a.n_ax = n_ax;
    a.n_ay = n_ay;
    for (int k = 0; k < 3; k++) a.o[k] = rd.o[k];
    for (int k = 0; k < 9; k++) a.rot[k] = rd.rot[k];
    a.fc = cd.fc;
    a.slope = cd.slope;
    a.fs = cd.fs;
    a.tc = cd.tc;
    a.S = cd.S;
    a.C = cd.C;
    a.out = reinterpret_cast<float4 *>(out);
    hipLaunchKernelGGL(k_cloud, dim3((max_points + 255) / 256), dim3(256), 0, s, a);
    SBR_LAUNCHED();
    return SBR_OK;
}

// two staging buffers, each large enough for any intermediate of the chain
static size_t cube_stage_elems(int Vx, int Vy, int C, int S, int Nax) {
    return (size_t)std::max(Vx * Vy, Vy * Nax) * C * S;
}

size_t cube2_scratch_bytes(int Vx, int Vy, int C, int S, int Nax, int Nay) {
    (void)Nay;
    Carver cv(nullptr);
    size_t big = cube_stage_elems(Vx, Vy, C, S, Nax);
    cv.take<float2>(big);
    cv.take<float2>(big);
    return align_up(cv.off, 256);
}

size_t cube_scratch_bytes(int V, int C, int S, int Na) { return cube2_scratch_bytes(V, 1, C, S, Na, 1); }

size_t cfar_scratch_bytes(int C, int S) {
    Carver cv(nullptr);
    cv.take<float>((size_t)C * S);
    cv.take<int>((size_t)C * S);
    cv.take<float>((size_t)C * S);
    cv.take<float>((size_t)kPowSplit * C * S);
    cv.take<float>((size_t)kPowSplit * C * S);
    cv.take<int>((size_t)kPowSplit * C * S);
    return align_up(cv.off, 256);
}

static size_t dft_lds_bytes(int N, int M, int Nt) {
    return sizeof(float2) * (size_t)Nt + sizeof(float) * (size_t)std::max(N, M);
}

static int launch_inner(const float2 *in, float2 *out, int rows, int N, int sign, int window, int post,
                        hipStream_t s) {
    const long long tiles = (long long)((N + 15) / 16) * ((rows + 15) / 16);
    hipLaunchKernelGGL(k_dft_inner, dim3((unsigned)((tiles + 3) / 4)), dim3(256), dft_lds_bytes(N, N, N), s, in,
                       out, rows, N, N, N, sign, window, post);
    SBR_LAUNCHED();
    return SBR_OK;
}

static int launch_mid(const float2 *in, float2 *out, int outer, int N, int M, int Nt, int inner, int sign,
                      int window, int post, hipStream_t s) {
    const long long tiles = (long long)outer * ((M + 15) / 16) * ((inner + 15) / 16);
    hipLaunchKernelGGL(k_dft_mid, dim3((unsigned)((tiles + 3) / 4)), dim3(256), dft_lds_bytes(N, M, Nt), s, in,
                       out, outer, N, M, Nt, inner, sign, window, post);
    SBR_LAUNCHED();
    return SBR_OK;
}

static int log2_exact(int n) {
    if (n < 2 || (n & (n - 1)) != 0 || n > kFftTile) return -1;
    int l = 0;
    while ((1 << l) < n) l++;
    return l;
}

static size_t fft_lds_bytes(int N) { return sizeof(float2) * ((size_t)N + (N + 1) / 2 + 2 * (size_t)kFftTile); }

// Range stage: FFT for power-of-two S (<= 1024), else the dense contraction.
static int launch_range(const float2 *in, float2 *out, int rows, int S, int sign, int window, int post,
                        hipStream_t s) {
    const int lg = log2_exact(S);
    if (lg < 0) return launch_inner(in, out, rows, S, sign, window, post, s);
    const int R = kFftTile >> lg;
    hipLaunchKernelGGL(k_fft_inner, dim3((unsigned)((rows + R - 1) / R)), dim3(256), fft_lds_bytes(S), s, in, out,
                       rows, lg, sign, window, post);
    SBR_LAUNCHED();
    return SBR_OK;
}

// Doppler stage: FFT for power-of-two C (<= 1024), else the dense contraction.
static int launch_doppler(const float2 *in, float2 *out, int V, int C, int S, int sign, int window, int post,
                          hipStream_t s) {
    const int lg = log2_exact(C);
    if (lg < 0) return launch_mid(in, out, V, C, C, C, S, sign, window, post, s);
    const int W = kFftTile >> lg;
    const long long blocks = (long long)V * ((S + W - 1) / W);
    hipLaunchKernelGGL(k_fft_mid, dim3((unsigned)blocks), dim3(256), fft_lds_bytes(C), s, in, out, V, lg, S, sign,
                       window, post);
    SBR_LAUNCHED();
    return SBR_OK;
}

// Launch an angle-stage kernel template K<VB, EXACT> for V antennas: the
// exact instance for V <= kAngleExact, else the guarded one with room for
// kAngleVMax.
constexpr int kAngleExact = 16;

// run() returns whether a kernel was launched.
template <template <int, bool> class K, int VV = 1>
struct AngleDispatch {
    template <typename... A>
    static bool run(int V, dim3 grid, size_t lds, hipStream_t s, A... args) {
        if (V == VV) return K<VV, true>::launch(grid, lds, s, args...);
        return AngleDispatch<K, VV + 1>::run(V, grid, lds, s, args...);
    }
};
template <template <int, bool> class K>
struct AngleDispatch<K, kAngleExact + 1> {
    template <typename... A>
    static bool run(int, dim3 grid, size_t lds, hipStream_t s, A... args) {
        return K<kAngleVMax, false>::launch(grid, lds, s, args...);
    }
};

template <int VB, bool EXACT>
struct AngleFwd {
    static bool launch(dim3 grid, size_t lds, hipStream_t s, const float2 *in, float2 *out, int V, int Na,
                       long long CS) {
        hipLaunchKernelGGL((k_angle<VB, EXACT>), grid, dim3(256), lds, s, in, out, V, Na, CS);
        return true;
    }
};

template <int VB, bool EXACT>
struct RangeAngle {
    static bool launch(dim3 grid, size_t lds, hipStream_t s, const float2 *in, float2 *out, int V, int C, int Na,
                       int window) {
        // the fused kernel holds at most kRaVMax = kAngleExact rows: there is
        // no guarded instance, and the caller reports the miss
        if constexpr (EXACT) {
            hipLaunchKernelGGL((k_range_angle<VB, true>), grid, dim3(256), lds, s, in, out, V, C, Na, window);
            return true;
        }
        return false;
    }
};

// Angle stage of a linear array: direct DFT for V <= 32, else the dense
// contraction.  dir 0: [V][CS] -> [Na][CS]; dir 1: [Na][CS] -> [V][CS].
static int launch_angle(const float2 *in, float2 *out, int V, int Na, long long CS, int dir, hipStream_t s) {
    if (V > kAngleVMax) {
        if (dir == 0) return launch_mid(in, out, 1, V, Na, Na, (int)CS, -1, 0, 0, s);
        return launch_mid(in, out, 1, Na, V, Na, (int)CS, +1, 0, 0, s);
    }
    const unsigned bx = (unsigned)((CS + 255) / 256);
    if (dir == 0) {
        const dim3 grid(bx, (unsigned)((Na + kAngleGroup - 1) / kAngleGroup));
        (void)AngleDispatch<AngleFwd>::run(V, grid, 0, s, in, out, V, Na, CS);   // every count has an instance
    } else {
        if (V <= 16)
            hipLaunchKernelGGL(k_angle_adj<16>, dim3(bx), dim3(256), sizeof(float2) * Na, s, in, out, V, Na, CS);
        else
            hipLaunchKernelGGL(k_angle_adj<kAngleVMax>, dim3(bx), dim3(256), sizeof(float2) * Na, s, in, out, V,
                               Na, CS);
    }
    SBR_LAUNCHED();
    return SBR_OK;
}

// Planar array: virtual antenna v = vy * Vx + vx; angle index a = ay * Nax + ax.
// Range and Doppler as for the linear array, then the angle DFT along vx
// (zero-padded to Nax) and along vy (to Nay): separable, each a middle-axis
// transform.  Vy = Nay = 1 is the linear array (one angle stage).
int radar_cube2_launch(const float2 *in, int Vx, int Vy, int C, int S, int Nax, int Nay, int window, int dir,
                       float2 *out, void *scratch, hipStream_t s) {
    Carver cv(scratch);
    const size_t big = cube_stage_elems(Vx, Vy, C, S, Nax);
    float2 *y1 = cv.take<float2>(big);
    float2 *y2 = cv.take<float2>(big);
    const int V = Vx * Vy, CS = C * S;
    const bool planar = Vy > 1 || Nay > 1;
    int rc;
    static_assert(kRaVMax == kAngleExact, "fused rows are dispatched by exact antenna count");
    if (dir == 0 && !planar && Vx <= kRaVMax && S == kRaS && log2_exact(C) >= 0) {
        // Doppler first, then range and angle in one pass per Doppler bin
        const int P = C / 16;
        const bool reg = C % 16 == 0 && (P == 2 || P == 4 || P == 8 || P == 16);
        if (reg) {
            const unsigned blocks = (unsigned)V * (unsigned)((S + kDopThreads / P - 1) / (kDopThreads / P));
            if (P == 2) hipLaunchKernelGGL(k_doppler<2>, dim3(blocks), dim3(kDopThreads), 0, s, in, y1, S, window);
            if (P == 4) hipLaunchKernelGGL(k_doppler<4>, dim3(blocks), dim3(kDopThreads), 0, s, in, y1, S, window);
            if (P == 8) hipLaunchKernelGGL(k_doppler<8>, dim3(blocks), dim3(kDopThreads), 0, s, in, y1, S, window);
            if (P == 16) hipLaunchKernelGGL(k_doppler<16>, dim3(blocks), dim3(kDopThreads), 0, s, in, y1, S, window);
        } else if ((rc = launch_doppler(in, y1, V, C, S, -1, window, 0, s))) {
            return rc;
        }
        const dim3 grid((unsigned)C, (unsigned)((Nax + kRangeAngleBins - 1) / kRangeAngleBins));
        if (!AngleDispatch<RangeAngle>::run(Vx, grid, range_angle_lds(Vx), s, (const float2 *)y1, out, Vx, C, Nax,
                                            window)) {
            set_error("fused range + angle stage has no instance for %d antennas", Vx);
            return SBR_E_UNSUPPORTED;
        }
        SBR_LAUNCHED();
        return SBR_OK;
    }
    if (dir == 0) {
        if ((rc = launch_range(in, y1, V * C, S, -1, window, 0, s))) return rc;
        if ((rc = launch_doppler(y1, y2, V, C, S, -1, window, 0, s))) return rc;
        if (!planar) return launch_angle(y2, out, Vx, Nax, CS, 0, s);
        if ((rc = launch_mid(y2, y1, Vy, Vx, Nax, Nax, CS, -1, 0, 0, s))) return rc;   // [Vy][Nax][CS]
        return launch_mid(y1, out, 1, Vy, Nay, Nay, Nax * CS, -1, 0, 0, s);          // [Nay][Nax][CS]
    }
    if (!planar) {
        if ((rc = launch_angle(in, y2, Vx, Nax, CS, 1, s))) return rc;
    } else {
        if ((rc = launch_mid(in, y1, 1, Nay, Vy, Nay, Nax * CS, +1, 0, 0, s))) return rc;   // [Vy][Nax][CS]
        if ((rc = launch_mid(y1, y2, Vy, Nax, Vx, Nax, CS, +1, 0, 0, s))) return rc;        // [Vy][Vx][CS]
    }
    if ((rc = launch_doppler(y2, y1, V, C, S, +1, window, 1, s))) return rc;
    return launch_range(y1, out, V * C, S, +1, window, 1, s);
}

int radar_cube_launch(const float2 *in, int V, int C, int S, int Na, int window, int dir, float2 *out,
                      void *scratch, hipStream_t s) {
    return radar_cube2_launch(in, V, 1, C, S, Na, 1, window, dir, out, scratch, s);
}

// Staging buffers of sbr_radar_cube_noalloc: a file-scope device array that
// every GPU the library runs on holds until the process ends.  In host code
// `scratch` names a host-side stand-in, never a device address: kernels get
// the per-device address hipGetSymbolAddress returns.
static __device__ __align__(256) char scratch[SBR_NOALLOC_SCRATCH_BYTES];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_noalloc_mu;
void *g_noalloc_ptr[kMaxDevices] = {};
}  // namespace

int noalloc_scratch(void **ptr) {
    int dev = 0;
    SBR_HIP(hipGetDevice(&dev));
    if (dev < 0 || dev >= kMaxDevices) {
        set_error("device %d beyond the %d the scratch-free entry point tracks", dev, kMaxDevices);
        return SBR_E_UNSUPPORTED;
    }
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {   // once per device, with that device current
        void *p = nullptr;
        SBR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
        g_noalloc_ptr[dev] = p;
    }
    *ptr = g_noalloc_ptr[dev];
    return SBR_OK;
}

int cfar_launch(const float2 *cube, int Na, int C, int S, int guard, int train, double pfa, int32_t *points,
                float *ratio_out, int maxp, int32_t *npts, void *scratch, hipStream_t s) {
    Carver cv(scratch);
    const int plane = C * S;
    float *P = cv.take<float>(plane);
    int *am = cv.take<int>(plane);
    float *ratio = cv.take<float>(plane);
    float *psum = cv.take<float>((size_t)kPowSplit * plane);
    float *pmax = cv.take<float>((size_t)kPowSplit * plane);
    int *parg = cv.take<int>((size_t)kPowSplit * plane);
    hipLaunchKernelGGL(k_power_part, dim3((plane + 63) / 64, kPowSplit), dim3(256), 0, s, cube, Na, plane, psum,
                       pmax, parg);
    hipLaunchKernelGGL(k_power_final, dim3((plane + 255) / 256), dim3(256), 0, s, plane, psum, pmax, parg, P, am);
    hipLaunchKernelGGL(k_cfar_cells, dim3((plane + 255) / 256), dim3(256), 0, s, P, C, S, guard, train, pfa,
                       ratio);
    hipLaunchKernelGGL(k_cfar_compact, dim3(1), dim3(1024), 0, s, ratio, am, plane, S, points, ratio_out, maxp,
                       npts);
    SBR_LAUNCHED();
    return SBR_OK;
}

}  // namespace sbr
