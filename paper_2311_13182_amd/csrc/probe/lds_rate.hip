// Standalone measurement of the LDS access rates that bound the spreading
// kernel of the FFT synthesis (64-bit integer atomic adds into LDS grid rows).
// Not part of libsbr.so; built next to it as the executable lds_rate_probe.
//
// Every block has 1024 threads (16 waves, as the spreading kernel) and four
// LDS rows of kCells 64-bit cells; wave w works on row w mod 4.  Each lane
// makes 7 accesses per iteration, like the 7 taps of a path:
//   random: cells j .. j + 6 of its row, j drawn per lane by a xorshift
//           generator, so the lanes of an instruction meet the banks at random;
//   linear: cell lane + 64 k with k = (7 it + t) mod 16, so the 64 lanes of an
//           instruction cover 512 contiguous bytes (no bank conflicts).
// The rate is reported in lanes per clock per CU at the kernel's own clock:
// s_memtime (shader clock) against the constant 100 MHz wall clock, both read
// by one lane around the timed loop.
#include <hip/hip_runtime.h>

#include <cstdio>

namespace {

constexpr int kCells = 1040;   // > 1023, the largest linear index
constexpr int kRows = 4;
constexpr int kTaps = 7;

enum Mode {
    kAddU64Random, kAddU32Random, kStoreB64Random, kAddU64Linear, kAddU32Linear, kStoreB64Linear,
    kAddF32Random, kAddF32Linear
};

template <int MODE>
__global__ __launch_bounds__(1024) void k_lds_rate(unsigned long long *out, unsigned long long *clk, int iters) {
    __shared__ unsigned long long cell[kCells * kRows];
    for (int i = threadIdx.x; i < kCells * kRows; i += 1024) cell[i] = 0;
    __syncthreads();
    const unsigned long long c0 = clock64(), w0 = wall_clock64();
    unsigned int x = 2463534242u ^ (threadIdx.x * 2654435761u) ^ (blockIdx.x * 97u);
    const int row = (threadIdx.x >> 6) % kRows, lane = threadIdx.x & 63;
    constexpr bool linear = MODE == kAddU64Linear || MODE == kAddU32Linear || MODE == kStoreB64Linear ||
                            MODE == kAddF32Linear;
    for (int it = 0; it < iters; it++) {
        x ^= x << 13;
        x ^= x >> 17;
        x ^= x << 5;
        const int j = (int)(x % (unsigned)(kCells - 8));   // j + 6 < kCells
#pragma unroll
        for (int t = 0; t < kTaps; t++) {
            const int col = linear ? lane + 64 * ((it * kTaps + t) & 15) : j + t;
            unsigned long long *c = cell + row * kCells + col;
            if (MODE == kAddU64Random || MODE == kAddU64Linear)
                atomicAdd(c, (unsigned long long)(x + t));
            else if (MODE == kAddU32Random || MODE == kAddU32Linear)
                atomicAdd(reinterpret_cast<unsigned int *>(c), x + t);
            else if (MODE == kAddF32Random || MODE == kAddF32Linear)
                atomicAdd(reinterpret_cast<float *>(c), (float)(x & 1023));
            else
                *c = (unsigned long long)(x + t);
        }
    }
    __syncthreads();
    const unsigned long long c1 = clock64(), w1 = wall_clock64();
    if (blockIdx.x == 0 && threadIdx.x == 0) {
        clk[0] = c1 - c0;
        clk[1] = w1 - w0;
    }
    unsigned long long s = 0;   // keeps the accesses live
    for (int i = threadIdx.x; i < kCells * kRows; i += 1024) s += cell[i];
    out[blockIdx.x * 1024 + threadIdx.x] = s;
}

template <int MODE>
int measure(const char *name, unsigned long long *out, unsigned long long *clk, int blocks, int iters) {
    hipEvent_t e0, e1;
    if (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess) return 1;
    hipLaunchKernelGGL(k_lds_rate<MODE>, dim3(blocks), dim3(1024), 0, 0, out, clk, iters);   // warm-up
    if (hipDeviceSynchronize() != hipSuccess) return 1;
    float best = 1e30f;
    unsigned long long cycles[2] = {0, 0};
    for (int r = 0; r < 3; r++) {
        (void)hipEventRecord(e0, 0);
        hipLaunchKernelGGL(k_lds_rate<MODE>, dim3(blocks), dim3(1024), 0, 0, out, clk, iters);
        (void)hipEventRecord(e1, 0);
        if (hipEventSynchronize(e1) != hipSuccess) return 1;
        float ms = 0.0f;
        (void)hipEventElapsedTime(&ms, e0, e1);
        if (ms < best) {
            best = ms;
            if (hipMemcpy(cycles, clk, sizeof(cycles), hipMemcpyDeviceToHost) != hipSuccess) return 1;
        }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    int n_cu = 0;
    if (hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, 0) != hipSuccess || n_cu <= 0) return 1;
    const double ghz = cycles[1] ? 0.1 * (double)cycles[0] / (double)cycles[1] : 0.0;
    const double per_ns = (double)blocks * 1024 * iters * kTaps / (best * 1e6) / n_cu;
    printf("%-20s %8.3f ms  %6.2f lanes/ns/CU  clock %.2f GHz  %5.2f lanes/clk/CU  (%5.1f B/clk/CU)\n", name, best,
           per_ns, ghz, ghz > 0 ? per_ns / ghz : 0.0,
           (ghz > 0 ? per_ns / ghz : 0.0) *
               ((MODE == kAddU32Random || MODE == kAddU32Linear || MODE == kAddF32Random || MODE == kAddF32Linear)
                    ? 4 : 8));
    fflush(stdout);
    return 0;
}

}  // namespace

int main() {
    const int blocks = 512, iters = 2000;
    unsigned long long *out = nullptr, *clk = nullptr;
    if (hipMalloc(&out, (size_t)blocks * 1024 * sizeof(unsigned long long)) != hipSuccess) return 1;
    if (hipMalloc(&clk, 2 * sizeof(unsigned long long)) != hipSuccess) return 1;
    int rc = 0;
    rc |= measure<kAddU64Random>("ds_add_u64 random", out, clk, blocks, iters);
    rc |= measure<kAddU32Random>("ds_add_u32 random", out, clk, blocks, iters);
    rc |= measure<kStoreB64Random>("64-bit store random", out, clk, blocks, iters);
    rc |= measure<kAddU64Linear>("ds_add_u64 linear", out, clk, blocks, iters);
    rc |= measure<kAddU32Linear>("ds_add_u32 linear", out, clk, blocks, iters);
    rc |= measure<kStoreB64Linear>("64-bit store linear", out, clk, blocks, iters);
    rc |= measure<kAddF32Random>("ds_add_f32 random", out, clk, blocks, iters);
    rc |= measure<kAddF32Linear>("ds_add_f32 linear", out, clk, blocks, iters);
    (void)hipFree(out);
    (void)hipFree(clk);
    printf(rc ? "error\n" : "done\n");
    return rc;
}
