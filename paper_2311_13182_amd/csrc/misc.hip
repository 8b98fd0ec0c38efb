// Loss entry of the backward pass and benchmark timing hooks.
#include <mutex>
#include <vector>

#include <algorithm>

#include <cstring>

#include "sbr_internal.h"

namespace sbr {

namespace {

constexpr int kLossBlocks = 1024;   // stage-1 blocks at most (partials in scratch)

// Stage 1: elementwise gradient and per-block partial sums of the loss, each
// block reducing its strided share in a fixed order, in double.
__global__ __launch_bounds__(256) void k_loss_part(int mode, const float2 *a, const float *b, long long n,
                                                   float2 *grad, double *part) {
    __shared__ double sh[256];
    const long long stride = (long long)gridDim.x * 256;
    double s = 0.0;
    for (long long i = (long long)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) {
        const float2 x = a[i];
        double e;
        if (mode == 0) {
            const float2 y = reinterpret_cast<const float2 *>(b)[i];
            if (grad) grad[i] = make_float2(2.0f * (x.x - y.x), 2.0f * (x.y - y.y));
            const double dr = (double)x.x - y.x, di = (double)x.y - y.y;
            e = dr * dr + di * di;
        } else {
            const float q = x.x * x.x + x.y * x.y - b[i];
            if (grad) {
                const float g = 4.0f * q / (float)n;
                grad[i] = make_float2(g * x.x, g * x.y);
            }
            const double qd = (double)x.x * x.x + (double)x.y * x.y - b[i];
            e = qd * qd;
        }
        s += e;
    }
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0 && part) part[blockIdx.x] = sh[0];
}

// Stage 2: the partials in a fixed order (one block).
__global__ __launch_bounds__(1024) void k_loss_final(const double *part, int nb, int mode, long long n,
                                                     float *loss) {
    __shared__ double sh[1024];
    sh[threadIdx.x] = (int)threadIdx.x < nb ? part[threadIdx.x] : 0.0;
    __syncthreads();
    for (int off = 512; off >= 1; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] += sh[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) *loss = (float)(mode == 0 ? sh[0] : sh[0] / (double)n);
}

struct ProfRec {
    hipEvent_t a, b;
};
std::mutex g_mu;
bool g_on = false;
std::vector<ProfRec> g_rec[kProfIds];

}  // namespace

ProfScope::ProfScope(int id, hipStream_t s) : id_(id), s_(s), active_(false) {
    std::lock_guard<std::mutex> lk(g_mu);
    if (!g_on || id < 0 || id >= kProfIds) return;
    if (hipEventCreate(&a_) != hipSuccess) return;
    if (hipEventCreate(&b_) != hipSuccess) {
        (void)hipEventDestroy(a_);
        return;
    }
    if (hipEventRecord(a_, s_) != hipSuccess) {
        (void)hipEventDestroy(a_);
        (void)hipEventDestroy(b_);
        return;
    }
    active_ = true;
}

ProfScope::~ProfScope() {
    if (!active_) return;
    std::lock_guard<std::mutex> lk(g_mu);
    if (hipEventRecord(b_, s_) == hipSuccess) {
        g_rec[id_].push_back({a_, b_});
    } else {
        (void)hipEventSynchronize(a_);
        (void)hipEventDestroy(a_);
        (void)hipEventDestroy(b_);
    }
}

int fill_zero_f32(float *p, size_t n, hipStream_t s);

namespace {
constexpr int kPutWords = 448;   // 1792 bytes of data per launch, within the kernel-argument limit
struct PutChunk {
    uint32_t w[kPutWords];
};
__global__ void k_put_words(PutChunk c, uint32_t *dst, int n) {
    for (int i = threadIdx.x; i < n; i += blockDim.x) dst[i] = c.w[i];
}
}  // namespace

int put_table(void *dst, const void *src, size_t bytes, hipStream_t s) {
    if (bytes % 4 != 0) {
        set_error("put_table: %zu bytes is not a multiple of 4", bytes);
        return SBR_E_ARG;
    }
    const uint32_t *w = static_cast<const uint32_t *>(src);
    uint32_t *d = static_cast<uint32_t *>(dst);
    const size_t nw = bytes / 4;
    for (size_t off = 0; off < nw; off += kPutWords) {
        PutChunk c;
        const int n = (int)std::min<size_t>(kPutWords, nw - off);
        memcpy(c.w, w + off, sizeof(uint32_t) * n);
        hipLaunchKernelGGL(k_put_words, dim3(1), dim3(256), 0, s, c, d + off, n);
    }
    SBR_LAUNCHED();
    return SBR_OK;
}

}  // namespace sbr

using namespace sbr;

extern "C" {

int sbr_loss_grad(int32_t mode, const float *a, const float *b, int64_t n, float *grad, float *loss,
                  void *scratch, size_t scratch_bytes, void *stream) {
    clear_error();
    SBR_CHECK_ARG(mode == 0 || mode == 1, "mode must be 0 (IF) or 1 (heatmap)");
    SBR_CHECK_ARG(n >= 0, "n must be >= 0");
    SBR_CHECK_ARG(n == 0 || (a && b), "a/b is NULL");
    if (loss && (!scratch || scratch_bytes < SBR_LOSS_SCRATCH_BYTES)) {
        set_error("loss scratch too small: %zu bytes given, %d needed", scratch_bytes, SBR_LOSS_SCRATCH_BYTES);
        return SBR_E_SCRATCH;
    }
    hipStream_t s = (hipStream_t)stream;
    if (n == 0) {
        if (loss) return fill_zero_f32(loss, 1, s);
        return SBR_OK;
    }
    if (!grad && !loss) return SBR_OK;
    const float2 *a2 = reinterpret_cast<const float2 *>(a);
    const int nb = (int)std::min<long long>(kLossBlocks, (n + 1023) / 1024);
    double *part = loss ? reinterpret_cast<double *>(scratch) : nullptr;
    hipLaunchKernelGGL(k_loss_part, dim3((unsigned)nb), dim3(256), 0, s, (int)mode, a2, b, (long long)n,
                       reinterpret_cast<float2 *>(grad), part);
    if (loss) hipLaunchKernelGGL(k_loss_final, dim3(1), dim3(1024), 0, s, part, nb, (int)mode, (long long)n, loss);
    SBR_LAUNCHED();
    return SBR_OK;
}

int sbr_profile(int32_t op) {
    clear_error();
    std::lock_guard<std::mutex> lk(g_mu);
    if (op == 0 || op == 1) {
        g_on = op == 1;
        return SBR_OK;
    }
    if (op == 2) {
        for (auto &v : g_rec) {
            for (auto &r : v) {
                (void)hipEventSynchronize(r.b);
                (void)hipEventDestroy(r.a);
                (void)hipEventDestroy(r.b);
            }
            v.clear();
        }
        return SBR_OK;
    }
    set_error("sbr_profile: op must be 0, 1 or 2");
    return SBR_E_ARG;
}

int sbr_profile_read(int32_t kernel, double *total_ms, int64_t *launches) {
    clear_error();
    SBR_CHECK_ARG(kernel >= 0 && kernel < kProfIds, "kernel id must be in [0, %d)", kProfIds);
    SBR_CHECK_ARG(total_ms && launches, "outputs are NULL");
    std::vector<ProfRec> recs;
    {
        std::lock_guard<std::mutex> lk(g_mu);
        recs.swap(g_rec[kernel]);
    }
    double tot = 0.0;
    int rc = SBR_OK;
    for (auto &r : recs) {
        float ms = 0.0f;
        hipError_t e = hipEventSynchronize(r.b);
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, r.a, r.b);
        if (e != hipSuccess && rc == SBR_OK) {
            set_error("event timing failed: %s", hipGetErrorString(e));
            rc = SBR_E_HIP;
        }
        tot += ms;
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    *total_ms = tot;
    *launches = (int64_t)recs.size();
    return rc;
}

}  // extern "C"
