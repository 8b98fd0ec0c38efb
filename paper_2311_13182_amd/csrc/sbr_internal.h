// Internal definitions shared by the libsbr HIP sources (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>

#include <algorithm>
#include <string>

#include "sbr.h"

namespace sbr {

// ----------------------------------------------------------------- errors
void set_error(const char *fmt, ...);
void clear_error();

#define SBR_CHECK_ARG(cond, ...)              \
    do {                                      \
        if (!(cond)) {                        \
            ::sbr::set_error(__VA_ARGS__);    \
            return SBR_E_ARG;                 \
        }                                     \
    } while (0)

#define SBR_HIP(call)                                                              \
    do {                                                                           \
        hipError_t e_ = (call);                                                    \
        if (e_ != hipSuccess) {                                                    \
            ::sbr::set_error("%s failed: %s (%s:%d)", #call, hipGetErrorString(e_), \
                             __FILE__, __LINE__);                                  \
            return SBR_E_HIP;                                                      \
        }                                                                          \
    } while (0)

#define SBR_LAUNCHED()                                                                \
    do {                                                                              \
        hipError_t e_ = hipGetLastError();                                            \
        if (e_ != hipSuccess) {                                                       \
            ::sbr::set_error("kernel launch failed: %s (%s:%d)", hipGetErrorString(e_), \
                             __FILE__, __LINE__);                                     \
            return SBR_E_HIP;                                                         \
        }                                                                             \
    } while (0)

static inline size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

// Carve sub-buffers out of a caller-provided byte buffer.
struct Carver {
    char *base;
    size_t off = 0;
    explicit Carver(void *b) : base(static_cast<char *>(b)) {}
    template <class T>
    T *take(size_t count) {
        off = align_up(off, 256);
        T *p = base ? reinterpret_cast<T *>(base + off) : nullptr;
        off += count * sizeof(T);
        return p;
    }
};

// ----------------------------------------------------------------- BVH
// Node of the depth-first layout: box, escape index (next node after this
// subtree; == node count ends traversal), leaf slot (-1 for internal nodes;
// the left child of an internal node is the next node).
struct __align__(32) BvhNode {
    float lo[3];
    float hi[3];
    int32_t escape;
    int32_t leaf;
};

// Triangle of a leaf: three vertices, .w of the first = original face id bits.
struct __align__(16) LeafTri {
    float4 a, b, c;
};

struct BvhView {
    int32_t n;          // triangles
    int32_t n_nodes;    // 2n - 1
    BvhNode *nodes;     // [n_nodes], depth-first order
    LeafTri *tris;      // [n], Morton order (leaf slot order)
    int32_t *order;     // [n] leaf slot -> original face
    int32_t *parent;    // [n_nodes] radix-tree parent (tree indices; -1 root)
    int2 *child;        // [n-1] radix-tree children
    int32_t *dfs_of;    // [n_nodes] radix-tree index -> depth-first index
    uint32_t *visits;   // [n-1] bottom-up arrival counters
    int32_t *header;    // [16] [0] n, [1] kBvhMagic once a BUILD of n faces has
                        // finished, [2] set to 1 by a REFIT that found no such BUILD
};

// Seal of a built BVH buffer (header[1]); refit and traversal check it
// together with header[0] == face count before they follow any stored index.
constexpr int32_t kBvhMagic = 0x48564253;

BvhView bvh_view(void *buf, int32_t nf, size_t *bytes_out);

// ----------------------------------------------------------------- constants
constexpr double kC0 = 299792458.0;
constexpr double kEps0 = 8.8541878128e-12;
constexpr double kPi = 3.14159265358979323846;

// Arguments of the path stage, passed by value to kernels.
struct MatTable {
    int32_t n;
    int32_t mode[SBR_MAX_MATERIALS];
    double eps_r[SBR_MAX_MATERIALS];
    double sigma[SBR_MAX_MATERIALS];
};

struct RadarDev {
    double o[3];
    double rot[9];
    int32_t n_tx, n_rx;
    double tx[SBR_MAX_TX][3];   // world frame
    double rx[SBR_MAX_RX][3];   // world frame
    double vel[3];
    double atten;               // amplitude attenuation of the medium, 1/m
    double n_tg, n_rg;          // TX / RX gain exponents (cos^n about boresight)
};

struct GridDev {
    int32_t nx, ny, K, options;
    double thx, thy, t_min;
    uint32_t seed_lo, seed_hi;
};

struct ChirpDev {
    double fc, slope, fs, tc;
    int32_t S, C;
};

// Device-side path records (structure of arrays, capacity = K * R).
struct PathSoA {
    int32_t cap;
    int32_t V;
    float *alpha;     // [V][cap] frac(fc * tau_v), cycles
    float *gamma;     // [V][cap] slope * tau_v / fs, cycles per sample
    float2 *amp;      // [cap] I^s
    float *beta;      // [cap] frac(fc * tc * taudot), cycles per chirp
    float *epsd;      // [cap] slope * tc * taudot / fs, cycles per sample per chirp
};

// Scratch layout of the path stage (compaction + records).
struct PathStage {
    int32_t *count;       // [4]: [0] = number of paths P
    int32_t *ray_first;   // [R + 1] first path index of each ray
    int32_t *blk;         // [nblk] per-block path counts then offsets
    int32_t nblk;
    PathSoA rec;
};

constexpr int kPathBlock = 256;   // rays per block of the compaction kernels

// Launch shape of the IF synthesis: L samples per lane, SB sample blocks per
// chirp row, tiles_per_v wavefronts per antenna, n_chunks path chunks.
struct SynthPlan {
    int32_t L, SB, tiles_per_v, n_chunks;
    int32_t nu, cg;      // non-uniform FFT form (L = 0): chirps per spreading block
};

// A pointer read from a device table is generic; marking it global lets the
// compiler use scalar or global (not flat) loads through it.  The qualifier
// exists in the device pass only (the host pass merely parses these bodies).
#if defined(__HIP_DEVICE_COMPILE__)
#define SBR_GLOBAL_AS __attribute__((address_space(1)))
#else
#define SBR_GLOBAL_AS
#endif
template <class T>
__device__ __forceinline__ SBR_GLOBAL_AS T *gmem(T *p) {
    return (SBR_GLOBAL_AS T *)p;
}
// plain pair of floats with float2's layout, for address-space-qualified access
struct F2 {
    float x, y;
};
__device__ __forceinline__ SBR_GLOBAL_AS const F2 *gmem(const float2 *p) { return (SBR_GLOBAL_AS const F2 *)p; }
__device__ __forceinline__ SBR_GLOBAL_AS F2 *gmem(float2 *p) { return (SBR_GLOBAL_AS F2 *)p; }

// Arguments of one request's IF synthesis (device-table entry of a batch).
struct SynthArgs {
    const int32_t *count;
    PathSoA rec;
    int32_t V, C, S;
    int32_t SB;          // sample blocks per chirp row
    int32_t tiles_per_v; // wavefront tiles per antenna
    int32_t n_chunks;
    int32_t gx;          // blocks per chunk (4 wavefronts each)
    float2 *partial;     // [n_chunks][V][C][S] (direct forms)
    // non-uniform FFT form (nu = 1): chirps per spreading block, chirp groups;
    // the max-amplitude word, the 1/Psi table and the fixed-point grids
    int32_t nu, cg, ncg;
    uint32_t *amax;      // [kNuMaxChunks] per path chunk: max over its paths of max(|Re A|, |Im A|), float bits
    float *corr;         // [S]
    long long *grid;     // [n_chunks][V][C][re, im][nu_row_len(S)]
    float2 *out;         // [V][C][S] the IF cube (set by launch_synth_batch)
};

PathStage carve_path_stage(Carver &cv, int32_t R, int32_t K, int32_t V);
SynthPlan synth_plan(int32_t R, int32_t K, int32_t V, int32_t C, int32_t S, bool nu);
size_t synth_partial_elems(const SynthPlan &p, int32_t V, int32_t C, int32_t S);
// Fixed-point grid words (long long) of the non-uniform FFT form.
size_t synth_grid_words(const SynthPlan &p, int32_t V, int32_t C, int32_t S);
SynthArgs synth_args(const PathStage &st, const SynthPlan &p, int32_t V, int32_t C, int32_t S, float2 *partial,
                     long long *grid, float *corr, uint32_t *amax);
// Device-table bytes of a batch of n syntheses.
size_t synth_table_bytes(int n);
// IF synthesis of n requests whose path stages are enqueued: one launch per
// sample-run length over all their blocks (args[i] and L[i] = synth_plan's L),
// then each request's fixed-order chunk reduction into out[i]; requests of the
// non-uniform FFT form (L[i] = 0) run their own spreading and row launches.
int launch_synth_batch(const SynthArgs *args, const int *L, int n, void *table, float2 *const *out,
                       hipStream_t s);

// One request of a (batched) backward pass: validated arguments, path stage
// enqueued into st, `extra` = its scratch after the path stage.
struct BackwardReq {
    const sbr_mesh *mesh;
    MatTable mt;
    RadarDev rd;
    GridDev gd;
    ChirpDev cd;
    const sbr_hits *hits;
    PathStage st;
    void *extra;
    const float2 *G;
    float *grad;
    const sbr_radar *radar;
    const sbr_param_grads *params;
    int32_t flags;
};
size_t backward_extra_bytes(int32_t R, int32_t K, int32_t V, int32_t C, int32_t S);
// Device-table bytes of a batch of n adjoints.
size_t adj_table_bytes(int n);
// Synthesis adjoint of n requests as one work-queue launch over all their
// (antenna group, path tile) items, then each request's reduction and
// geometry adjoint.
int launch_backward_batch(const BackwardReq *reqs, int n, void *table, hipStream_t s);

// ---- non-uniform FFT forms of Eq. (8) (type 1) and Eqs. (11)-(12) (type 2)
// A sum over the S samples of a chirp, sum_s h_s e^{2 pi j s g}, is a finite
// Fourier series at the beat frequency g of a path.  With the modes centred
// (s' = s - S/2), a grid of M = 2S points and a kernel psi of width kNuW grid
// points whose Fourier transform is Psi:
//   e^{2 pi j s' g} Psi(s'/M) = sum_l e^{2 pi j s' l / M} psi(gM - l)
// up to the kernel's aliasing error, which is below 1e-6 of the sum of the
// magnitudes of the terms for the exponential-of-semicircle kernel
// psi(z) = exp(beta (sqrt(1 - (2z/W)^2) - 1)), W = 7, beta = 2.3 W.  Rows of
// grid values hold l = -M/2 - 3 .. M/2 + 3 at index l + M/2 + 3, plus one
// padding entry.
constexpr int kNuW = 7;
constexpr int kNuHalf = (kNuW - 1) / 2;
constexpr double kNuBeta = 2.30 * kNuW;
constexpr int kNuMinS = 16;     // shorter chirps use the direct forms (cheap there)
constexpr int kNuMaxS = 1024;   // longer chirps use the direct forms
constexpr int kNuMaxChunks = 256;   // path chunks of a spreading launch, each with its own scale
__host__ __device__ constexpr int nu_row_len(int S) { return 2 * S + 8; }
static inline bool nu_size(int S) { return S >= kNuMinS && S <= kNuMaxS; }

// Copy `bytes` (a multiple of 4) of host data into device memory on stream s
// with fill kernels that carry the data as kernel arguments: no memcpy node,
// and the host data need not outlive the call.
int put_table(void *dst, const void *src, size_t bytes, hipStream_t s);

// host-side conversions / validation shared by the entry points
int check_mesh(const sbr_mesh *m);
int check_common(const sbr_mesh *m, const sbr_material *mats, int32_t n_mats,
                 const sbr_radar *r, const sbr_rays *g, const sbr_hits *h,
                 const sbr_chirp *ch);
MatTable make_mats(const sbr_material *mats, int32_t n_mats);
RadarDev make_radar(const sbr_radar *r);
GridDev make_grid(const sbr_rays *g);
ChirpDev make_chirp(const sbr_chirp *c);

// Brackets one kernel launch with HIP events while sbr_profile(1) is on.
class ProfScope {
   public:
    ProfScope(int id, hipStream_t s);
    ~ProfScope();

   private:
    int id_;
    hipStream_t s_;
    bool active_;
    hipEvent_t a_{}, b_{};
};
enum { kProfSynth = 0, kProfSynthAdj = 1, kProfTrace = 2, kProfNuSpread = 3, kProfNuTaps = 4, kProfIds = 5 };

// Blocks of `kernel` (launched with `threads` threads and `lds` bytes of
// dynamic LDS) the current device holds at once: CUs times the occupancy the
// runtime reports for the compiled kernel, cached per (device, kernel,
// threads, lds); `fallback` where the runtime cannot answer.
int resident_blocks(const void *kernel, int threads, size_t lds, int fallback);

// zero n floats with a fill kernel on stream s (no memset node, so the call
// can sit in a captured graph)
int fill_zero_f32(float *p, size_t n, hipStream_t s);

// enqueue path compaction + FP64 refinement; records go to st.rec
int launch_paths(const sbr_mesh *m, const MatTable &mt, const RadarDev &rd, const GridDev &gd,
                 const ChirpDev &cd, const sbr_hits *h, int32_t flags, const PathStage &st,
                 hipStream_t s);

}  // namespace sbr
