// C ABI of libsbr: argument checks, scratch carving, launches.
#include <stdarg.h>

#include <algorithm>
#include <map>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "sbr_internal.h"

namespace sbr {

static thread_local std::string g_err;

void set_error(const char *fmt, ...) {
    char buf[1024];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof(buf), fmt, ap);
    va_end(ap);
    g_err = buf;
}
void clear_error() { g_err.clear(); }

// implemented in the kernel sources
int bvh_build(const sbr_mesh *m, void *bvh, size_t bvh_bytes, int32_t mode, void *scratch,
              size_t scratch_bytes, hipStream_t st);
size_t build_scratch_bytes(int32_t nf);
int trace_launch(const sbr_mesh *m, const void *bvh, const RadarDev &rd, const GridDev &gd,
                 const sbr_hits *h, uint64_t *counters, hipStream_t st);
size_t cube_scratch_bytes(int V, int C, int S, int Na);
size_t cube2_scratch_bytes(int Vx, int Vy, int C, int S, int Nax, int Nay);
int cloud_launch(const int32_t *points, const int32_t *n_points, int32_t max_points, const RadarDev &rd,
                 const ChirpDev &cd, int32_t n_ax, int32_t n_ay, float *out, hipStream_t s);
size_t peaks_scratch_bytes(int max_det, int Na);
int peaks_launch(const float2 *X, int n_ax, int n_ay, int C, int S, const int32_t *det, const int32_t *n_det,
                 int max_det, float rel, int32_t *points, int max_points, int32_t *n_points, void *scratch,
                 hipStream_t s);
int radar_cube2_launch(const float2 *in, int Vx, int Vy, int C, int S, int Nax, int Nay, int window, int dir,
                       float2 *out, void *scratch, hipStream_t s);
size_t cfar_scratch_bytes(int C, int S);
int radar_cube_launch(const float2 *in, int V, int C, int S, int Na, int window, int dir, float2 *out,
                      void *scratch, hipStream_t s);
int cfar_launch(const float2 *cube, int Na, int C, int S, int guard, int train, double pfa, int32_t *points,
                float *ratio_out, int maxp, int32_t *npts, void *scratch, hipStream_t s);
int fill_zero_f32(float *p, size_t n, hipStream_t s);
int noalloc_scratch(void **ptr);

int resident_blocks(const void *kernel, int threads, size_t lds, int fallback) {
    static std::mutex mu;
    static std::map<std::tuple<int, const void *, int, size_t>, int> cache;
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess) {
        (void)hipGetLastError();
        return fallback;
    }
    std::lock_guard<std::mutex> lk(mu);
    const auto key = std::make_tuple(dev, kernel, threads, lds);
    auto it = cache.find(key);
    if (it != cache.end()) return it->second;
    int cus = 0, nb = 0;
    hipError_t e1 = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
    hipError_t e2 = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, kernel, threads, lds);
    int res = fallback;
    if (e1 == hipSuccess && e2 == hipSuccess && cus > 0 && nb > 0) res = cus * nb;
    else (void)hipGetLastError();
    cache[key] = res;
    return res;
}

int check_mesh(const sbr_mesh *m) {
    SBR_CHECK_ARG(m, "mesh is NULL");
    SBR_CHECK_ARG(m->nf >= 0 && m->nv >= 0, "negative mesh size (nv=%d nf=%d)", m->nv, m->nf);
    SBR_CHECK_ARG(m->nf == 0 || (m->verts && m->faces && m->nv > 0), "mesh verts/faces are NULL");
    SBR_CHECK_ARG(m->nf <= (1 << 27), "too many faces (%d)", m->nf);
    return SBR_OK;
}

static int check_radar(const sbr_radar *r) {
    SBR_CHECK_ARG(r, "radar is NULL");
    SBR_CHECK_ARG(r->n_tx >= 1 && r->n_tx <= SBR_MAX_TX, "n_tx=%d out of [1,%d]", r->n_tx, SBR_MAX_TX);
    SBR_CHECK_ARG(r->n_rx >= 1 && r->n_rx <= SBR_MAX_RX, "n_rx=%d out of [1,%d]", r->n_rx, SBR_MAX_RX);
    SBR_CHECK_ARG(r->n_tx * r->n_rx <= SBR_MAX_VIRTUAL, "n_tx*n_rx=%d > %d", r->n_tx * r->n_rx,
                  SBR_MAX_VIRTUAL);
    SBR_CHECK_ARG(r->attenuation >= 0.0 && r->attenuation < 1e6, "attenuation must be in [0, 1e6) per metre");
    SBR_CHECK_ARG(r->tx_gain_exp >= 0.0 && r->tx_gain_exp <= 1000.0 && r->rx_gain_exp >= 0.0 &&
                      r->rx_gain_exp <= 1000.0,
                  "gain exponents must be in [0, 1000]");
    return SBR_OK;
}

static int check_rays(const sbr_rays *g) {
    SBR_CHECK_ARG(g, "rays is NULL");
    SBR_CHECK_ARG(g->nx >= 0 && g->ny >= 0, "negative grid (%d x %d)", g->nx, g->ny);
    SBR_CHECK_ARG((long long)g->nx * g->ny <= (1LL << 26), "grid too large (%d x %d)", g->nx, g->ny);
    SBR_CHECK_ARG(g->max_bounces >= 1 && g->max_bounces <= SBR_MAX_BOUNCES, "max_bounces=%d out of [1,%d]",
                  g->max_bounces, SBR_MAX_BOUNCES);
    SBR_CHECK_ARG((g->options & ~(SBR_RAYS_SHADOW | SBR_RAYS_JITTER)) == 0, "unknown sbr_rays.options bits 0x%x",
                  g->options);
    SBR_CHECK_ARG(g->tan_half_x > 0 && g->tan_half_y > 0, "grid half-widths must be positive");
    SBR_CHECK_ARG(g->t_min >= 0, "t_min must be >= 0");
    return SBR_OK;
}

static int check_chirp(const sbr_chirp *c) {
    SBR_CHECK_ARG(c, "chirp is NULL");
    SBR_CHECK_ARG(c->n_samples >= 1 && c->n_chirps >= 1, "chirp sizes must be >= 1 (S=%d C=%d)",
                  c->n_samples, c->n_chirps);
    SBR_CHECK_ARG(c->n_samples <= 4096 && c->n_chirps <= 4096, "chirp sizes must be <= 4096");
    SBR_CHECK_ARG(c->fs > 0 && c->fc > 0, "fs and fc must be positive");
    return SBR_OK;
}

static int check_hits(const sbr_hits *h, const sbr_rays *g) {
    SBR_CHECK_ARG(h, "hits is NULL");
    if ((long long)g->nx * g->ny == 0) return SBR_OK;   // nothing is read or written
    SBR_CHECK_ARG(h->tri && h->t && h->u && h->v && h->flags, "a hits array is NULL");
    return SBR_OK;
}

int check_common(const sbr_mesh *m, const sbr_material *mats, int32_t n_mats, const sbr_radar *r,
                 const sbr_rays *g, const sbr_hits *h, const sbr_chirp *ch) {
    int rc;
    if ((rc = check_mesh(m))) return rc;
    if ((rc = check_radar(r))) return rc;
    if ((rc = check_rays(g))) return rc;
    if ((rc = check_hits(h, g))) return rc;
    if ((rc = check_chirp(ch))) return rc;
    SBR_CHECK_ARG(n_mats >= 0 && n_mats <= SBR_MAX_MATERIALS, "n_mats=%d out of [0,%d]", n_mats,
                  SBR_MAX_MATERIALS);
    SBR_CHECK_ARG(n_mats == 0 || mats, "mats is NULL with n_mats=%d", n_mats);
    for (int i = 0; i < n_mats; i++)
        SBR_CHECK_ARG(mats[i].mode >= 0 && mats[i].mode <= 2, "material %d: mode %d not in {0,1,2}", i,
                      mats[i].mode);
    return SBR_OK;
}

MatTable make_mats(const sbr_material *mats, int32_t n_mats) {
    MatTable t;
    t.n = mats ? n_mats : 0;
    for (int i = 0; i < SBR_MAX_MATERIALS; i++) {
        t.mode[i] = i < t.n ? mats[i].mode : 0;
        t.eps_r[i] = i < t.n ? mats[i].eps_r : 1.0;
        t.sigma[i] = i < t.n ? mats[i].sigma : 0.0;
    }
    return t;
}

RadarDev make_radar(const sbr_radar *r) {
    RadarDev d;
    for (int i = 0; i < 3; i++) {
        d.o[i] = r->origin[i];
        d.vel[i] = r->velocity[i];
    }
    for (int i = 0; i < 9; i++) d.rot[i] = r->rot[i];
    d.atten = r->attenuation;
    d.n_tg = r->tx_gain_exp;
    d.n_rg = r->rx_gain_exp;
    d.n_tx = r->n_tx;
    d.n_rx = r->n_rx;
    auto world = [&](const double *p, double *o) {
        for (int i = 0; i < 3; i++)
            o[i] = r->origin[i] + r->rot[3 * i] * p[0] + r->rot[3 * i + 1] * p[1] + r->rot[3 * i + 2] * p[2];
    };
    for (int t = 0; t < SBR_MAX_TX; t++) {
        if (t < r->n_tx) world(r->tx[t], d.tx[t]);
        else d.tx[t][0] = d.tx[t][1] = d.tx[t][2] = 0.0;
    }
    for (int m = 0; m < SBR_MAX_RX; m++) {
        if (m < r->n_rx) world(r->rx[m], d.rx[m]);
        else d.rx[m][0] = d.rx[m][1] = d.rx[m][2] = 0.0;
    }
    return d;
}

GridDev make_grid(const sbr_rays *g) {
    GridDev d;
    d.nx = g->nx;
    d.ny = g->ny;
    d.K = g->max_bounces;
    d.options = g->options;
    d.seed_lo = g->seed_lo;
    d.seed_hi = g->seed_hi;
    d.thx = g->tan_half_x;
    d.thy = g->tan_half_y;
    d.t_min = g->t_min;
    return d;
}

ChirpDev make_chirp(const sbr_chirp *c) {
    ChirpDev d;
    d.fc = c->fc;
    d.slope = c->slope;
    d.fs = c->fs;
    d.tc = c->t_chirp;
    d.S = c->n_samples;
    d.C = c->n_chirps;
    return d;
}

// Scratch of one synthesis: path stage, chunk partials (direct forms) or
// fixed-point grids, 1/Psi table and amplitude word (non-uniform FFT form), a
// one-request table.
struct SynthCarve {
    PathStage st;
    SynthPlan p;
    float2 *partial;
    long long *grid;
    float *corr;
    uint32_t *amax;
    void *table;
    size_t bytes;
};

static SynthCarve synth_carve(void *scratch, int R, int K, int V, int C, int S, bool nu) {
    SynthCarve c;
    Carver cv(scratch);
    c.st = carve_path_stage(cv, R, K, V);
    c.p = synth_plan(R, K, V, C, S, nu);
    c.partial = nu ? nullptr : cv.take<float2>(synth_partial_elems(c.p, V, C, S));
    c.grid = nu ? cv.take<long long>(synth_grid_words(c.p, V, C, S)) : nullptr;
    c.corr = nu ? cv.take<float>((size_t)S) : nullptr;
    c.amax = nu ? cv.take<uint32_t>(kNuMaxChunks) : nullptr;
    c.table = cv.take<char>(synth_table_bytes(1));
    c.bytes = align_up(cv.off, 256);
    return c;
}

// Whether a synthesis request runs as the non-uniform FFT form.
static bool synth_nu(int S, int32_t flags) { return nu_size(S) && !(flags & SBR_DIRECT_SUMS); }

// Scratch bytes of a synthesis, whichever form its flags select.
static size_t synth_bytes(int R, int K, int V, int C, int S) {
    size_t b = synth_carve(nullptr, R, K, V, C, S, false).bytes;
    if (nu_size(S)) b = std::max(b, synth_carve(nullptr, R, K, V, C, S, true).bytes);
    return b;
}

// Scratch of one backward pass: path stage, adjoint buffers, a one-request table.
struct BackCarve {
    PathStage st;
    void *extra;
    void *table;
    size_t bytes;
};

static BackCarve back_carve(void *scratch, int R, int K, int V, int C, int S) {
    BackCarve c;
    Carver cv(scratch);
    c.st = carve_path_stage(cv, R, K, V);
    c.extra = cv.take<char>(backward_extra_bytes(R, K, V, C, S));
    c.table = cv.take<char>(adj_table_bytes(1));
    c.bytes = align_up(cv.off, 256);
    return c;
}

static size_t backward_bytes(int R, int K, int V, int C, int S) { return back_carve(nullptr, R, K, V, C, S).bytes; }

// Checks of one sbr_synth_if request; 0 if it may be enqueued.
static int check_synth(const sbr_mesh *mesh, const sbr_material *mats, int32_t n_mats, const sbr_radar *radar,
                       const sbr_rays *rays, const sbr_hits *hits, const sbr_chirp *chirp, int32_t flags,
                       const float *if_cube, const void *scratch, size_t scratch_bytes) {
    int rc;
    if ((rc = check_common(mesh, mats, n_mats, radar, rays, hits, chirp))) return rc;
    SBR_CHECK_ARG(if_cube, "if_cube is NULL");
    SBR_CHECK_ARG((flags & ~(SBR_DROP_FLAGGED | SBR_EXIT_ONLY | SBR_DIRECT_SUMS)) == 0, "unknown flags 0x%x", flags);
    const size_t need = synth_bytes(rays->nx * rays->ny, rays->max_bounces, radar->n_tx * radar->n_rx,
                                    chirp->n_chirps, chirp->n_samples);
    if (!scratch || scratch_bytes < need) {
        set_error("synth scratch too small: %zu bytes given, %zu needed", scratch_bytes, need);
        return SBR_E_SCRATCH;
    }
    return SBR_OK;
}

// Checks of one sbr_backward request; 0 if it may be enqueued.
static int check_backward(const sbr_mesh *mesh, const sbr_material *mats, int32_t n_mats, const sbr_radar *radar,
                          const sbr_rays *rays, const sbr_hits *hits, const sbr_chirp *chirp, int32_t flags,
                          const float *grad_if, const float *grad_verts, const sbr_param_grads *params,
                          const void *scratch, size_t scratch_bytes) {
    int rc;
    if ((rc = check_common(mesh, mats, n_mats, radar, rays, hits, chirp))) return rc;
    SBR_CHECK_ARG(grad_if && grad_verts, "grad_if/grad_verts is NULL");
    SBR_CHECK_ARG((flags & ~(SBR_DROP_FLAGGED | SBR_ATTACHED | SBR_EXIT_ONLY | SBR_DIRECT_SUMS |
                             SBR_PATHS_IN_SCRATCH)) == 0,
                  "unknown flags 0x%x", flags);
    SBR_CHECK_ARG(!params || !params->materials || (mats && n_mats > 0),
                  "material gradients requested without a material table");
    const size_t need = backward_bytes(rays->nx * rays->ny, rays->max_bounces, radar->n_tx * radar->n_rx,
                                       chirp->n_chirps, chirp->n_samples);
    if (!scratch || scratch_bytes < need) {
        set_error("backward scratch too small: %zu bytes given, %zu needed", scratch_bytes, need);
        return SBR_E_SCRATCH;
    }
    return SBR_OK;
}

// Enqueue the path stage of a synthesis request and fill its batch entry;
// *skip = 1 when its cube is all zero (empty grid: zero-filled here).
static int enqueue_synth(const sbr_mesh *mesh, const sbr_material *mats, int32_t n_mats, const sbr_radar *radar,
                         const sbr_rays *rays, const sbr_hits *hits, const sbr_chirp *chirp, int32_t flags,
                         float *if_cube, void *scratch, hipStream_t s, SynthArgs *args, int *L, void **table,
                         int *skip) {
    const int R = rays->nx * rays->ny, K = rays->max_bounces;
    const int V = radar->n_tx * radar->n_rx, C = chirp->n_chirps, S = chirp->n_samples;
    *skip = 0;
    if (R == 0) {
        *skip = 1;
        return fill_zero_f32(if_cube, (size_t)2 * V * C * S, s);
    }
    SynthCarve c = synth_carve(scratch, R, K, V, C, S, synth_nu(S, flags));
    int rc;
    if ((rc = launch_paths(mesh, make_mats(mats, n_mats), make_radar(radar), make_grid(rays), make_chirp(chirp),
                           hits, flags, c.st, s)))
        return rc;
    *args = synth_args(c.st, c.p, V, C, S, c.partial, c.grid, c.corr, c.amax);
    *L = c.p.L;
    if (table) *table = c.table;
    return SBR_OK;
}

// Enqueue the path stage of a backward request and fill its batch entry;
// *skip = 1 when it adds nothing (empty grid or mesh).
static int enqueue_backward(const sbr_mesh *mesh, const sbr_material *mats, int32_t n_mats, const sbr_radar *radar,
                            const sbr_rays *rays, const sbr_hits *hits, const sbr_chirp *chirp, int32_t flags,
                            const float *grad_if, float *grad_verts, const sbr_param_grads *params, void *scratch,
                            hipStream_t s, BackwardReq *q, void **table, int *skip) {
    const int R = rays->nx * rays->ny, K = rays->max_bounces;
    const int V = radar->n_tx * radar->n_rx;
    *skip = 0;
    if (R == 0 || mesh->nf == 0) {
        *skip = 1;
        return SBR_OK;
    }
    BackCarve c = back_carve(scratch, R, K, V, chirp->n_chirps, chirp->n_samples);
    q->mesh = mesh;
    q->mt = make_mats(mats, n_mats);
    q->rd = make_radar(radar);
    q->gd = make_grid(rays);
    q->cd = make_chirp(chirp);
    q->hits = hits;
    q->st = c.st;
    q->extra = c.extra;
    q->G = reinterpret_cast<const float2 *>(grad_if);
    q->grad = grad_verts;
    q->radar = radar;
    q->params = params;
    q->flags = flags;
    if (table) *table = c.table;
    if (flags & SBR_PATHS_IN_SCRATCH) return SBR_OK;   // records of the preceding synthesis
    return launch_paths(mesh, q->mt, q->rd, q->gd, q->cd, hits, flags, q->st, s);
}

}  // namespace sbr

using namespace sbr;

extern "C" {

const char *sbr_last_error(void) { return g_err.c_str(); }

size_t sbr_bvh_bytes(int32_t nf) {
    if (nf < 1) return 0;
    size_t b = 0;
    bvh_view(nullptr, nf, &b);
    return b;
}

size_t sbr_scratch_bytes(int32_t op, const sbr_mesh *mesh, const sbr_rays *rays, const sbr_radar *radar,
                         const sbr_chirp *chirp) {
    switch (op) {
    case SBR_OP_BUILD_BVH:
        if (!mesh || mesh->nf < 1) return 0;
        return build_scratch_bytes(mesh->nf);
    case SBR_OP_SYNTH:
    case SBR_OP_BACKWARD: {
        if (!rays || !radar || !chirp) return 0;
        long long R = (long long)rays->nx * rays->ny;
        if (R < 0 || rays->max_bounces < 1 || radar->n_tx < 1 || radar->n_rx < 1) return 0;
        int V = radar->n_tx * radar->n_rx;
        if (op == SBR_OP_SYNTH)
            return synth_bytes((int)R, rays->max_bounces, V, chirp->n_chirps, chirp->n_samples);
        return backward_bytes((int)R, rays->max_bounces, V, chirp->n_chirps, chirp->n_samples);
    }
    case SBR_OP_RADAR_CUBE: {
        if (!radar || !chirp) return 0;
        int V = radar->n_tx * radar->n_rx;
        return cube_scratch_bytes(V, chirp->n_chirps, chirp->n_samples, std::max(64, V));
    }
    case SBR_OP_CFAR:
        if (!chirp) return 0;
        return cfar_scratch_bytes(chirp->n_chirps, chirp->n_samples);
    default:
        return 0;
    }
}

int sbr_build_bvh(const sbr_mesh *mesh, void *bvh, size_t bvh_bytes, int32_t mode, void *scratch,
                  size_t scratch_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = check_mesh(mesh))) return rc;
    SBR_CHECK_ARG(mesh->nf >= 1, "BVH needs at least one face");
    SBR_CHECK_ARG(bvh, "bvh is NULL");
    SBR_CHECK_ARG(mode == 0 || mode == 1, "mode must be 0 (build) or 1 (refit)");
    return bvh_build(mesh, bvh, bvh_bytes, mode, scratch, scratch_bytes, (hipStream_t)stream);
}

int sbr_trace(const sbr_mesh *mesh, const void *bvh, const sbr_radar *radar, const sbr_rays *rays,
              const sbr_hits *out, uint64_t *counters, void *stream) {
    clear_error();
    int rc;
    if ((rc = check_mesh(mesh))) return rc;
    if ((rc = check_radar(radar))) return rc;
    if ((rc = check_rays(rays))) return rc;
    if ((rc = check_hits(out, rays))) return rc;
    SBR_CHECK_ARG(mesh->nf == 0 || bvh, "bvh is NULL");
    if ((long long)rays->nx * rays->ny == 0) return SBR_OK;
    RadarDev rd = make_radar(radar);
    GridDev gd = make_grid(rays);
    return trace_launch(mesh, bvh, rd, gd, out, counters, (hipStream_t)stream);
}

int sbr_synth_if(const sbr_mesh *mesh, const sbr_material *mats, int32_t n_mats, const sbr_radar *radar,
                 const sbr_rays *rays, const sbr_hits *hits, const sbr_chirp *chirp, int32_t flags,
                 float *if_cube, void *scratch, size_t scratch_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = check_synth(mesh, mats, n_mats, radar, rays, hits, chirp, flags, if_cube, scratch, scratch_bytes)))
        return rc;
    hipStream_t s = (hipStream_t)stream;
    SynthArgs a;
    int L = 0, skip = 0;
    void *table = nullptr;
    if ((rc = enqueue_synth(mesh, mats, n_mats, radar, rays, hits, chirp, flags, if_cube, scratch, s, &a, &L, &table,
                            &skip)))
        return rc;
    if (skip) return SBR_OK;
    float2 *out = reinterpret_cast<float2 *>(if_cube);
    return launch_synth_batch(&a, &L, 1, table, &out, s);
}

size_t sbr_batch_table_bytes(int32_t n_requests) {
    if (n_requests < 1 || n_requests > SBR_MAX_BATCH) return 0;
    return std::max(synth_table_bytes(n_requests), adj_table_bytes(n_requests));
}

// Batched calls: no two requests may write the same device bytes (scratch,
// IF cube, gradient).  The written ranges are sorted by start address and
// neighbours compared; a shared range is an argument error naming both.
namespace {
struct Span {
    uintptr_t lo, hi;
    int req;
    const char *what;
};

int check_disjoint(std::vector<Span> &sp) {
    std::sort(sp.begin(), sp.end(), [](const Span &a, const Span &b) { return a.lo < b.lo; });
    uintptr_t end = 0;
    int owner = -1;
    const char *what = "";
    for (const Span &x : sp) {
        if (x.hi <= x.lo) continue;
        if (owner >= 0 && x.lo < end && x.req != owner) {
            set_error("requests %d and %d share device memory (%s of %d overlaps %s of %d)", owner, x.req, what,
                      owner, x.what, x.req);
            return SBR_E_ARG;
        }
        if (x.hi > end || owner < 0) {
            end = x.hi;
            owner = x.req;
            what = x.what;
        }
    }
    return SBR_OK;
}

size_t cube_bytes_of(const sbr_request &q) {
    return (size_t)q.radar->n_tx * q.radar->n_rx * q.chirp->n_chirps * q.chirp->n_samples * 2 * sizeof(float);
}
}  // namespace

int sbr_synth_if_batched(const sbr_request *reqs, int32_t n, void *table, size_t table_bytes, void *stream) {
    clear_error();
    SBR_CHECK_ARG(n >= 0 && n <= SBR_MAX_BATCH, "n=%d out of [0, %d]", n, SBR_MAX_BATCH);
    SBR_CHECK_ARG(n == 0 || reqs, "reqs is NULL");
    if (n == 0) return SBR_OK;
    const size_t need = sbr_batch_table_bytes(n);
    if (!table || table_bytes < need) {
        set_error("batch table too small: %zu bytes given, %zu needed", table_bytes, need);
        return SBR_E_SCRATCH;
    }
    int rc;
    for (int i = 0; i < n; i++) {
        const sbr_request &q = reqs[i];
        if ((rc = check_synth(q.mesh, q.mats, q.n_mats, q.radar, q.rays, q.hits, q.chirp, q.flags, q.if_cube,
                              q.scratch, q.scratch_bytes))) {
            const std::string msg = sbr_last_error();
            set_error("request %d: %s", i, msg.c_str());
            return rc;
        }
    }
    {
        std::vector<Span> sp;
        for (int i = 0; i < n; i++) {
            const sbr_request &q = reqs[i];
            sp.push_back({(uintptr_t)q.scratch, (uintptr_t)q.scratch + q.scratch_bytes, i, "scratch"});
            sp.push_back({(uintptr_t)q.if_cube, (uintptr_t)q.if_cube + cube_bytes_of(q), i, "if_cube"});
        }
        if ((rc = check_disjoint(sp))) return rc;
    }
    hipStream_t s = (hipStream_t)stream;
    std::vector<SynthArgs> args;
    std::vector<int> Ls;
    std::vector<float2 *> outs;
    for (int i = 0; i < n; i++) {
        const sbr_request &q = reqs[i];
        SynthArgs a;
        int L = 0, skip = 0;
        if ((rc = enqueue_synth(q.mesh, q.mats, q.n_mats, q.radar, q.rays, q.hits, q.chirp, q.flags, q.if_cube,
                                q.scratch, s, &a, &L, nullptr, &skip)))
            return rc;
        if (skip) continue;
        args.push_back(a);
        Ls.push_back(L);
        outs.push_back(reinterpret_cast<float2 *>(q.if_cube));
    }
    return launch_synth_batch(args.data(), Ls.data(), (int)args.size(), table, outs.data(), s);
}

int sbr_backward_batched(const sbr_request *reqs, int32_t n, void *table, size_t table_bytes, void *stream) {
    clear_error();
    SBR_CHECK_ARG(n >= 0 && n <= SBR_MAX_BATCH, "n=%d out of [0, %d]", n, SBR_MAX_BATCH);
    SBR_CHECK_ARG(n == 0 || reqs, "reqs is NULL");
    if (n == 0) return SBR_OK;
    const size_t need = sbr_batch_table_bytes(n);
    if (!table || table_bytes < need) {
        set_error("batch table too small: %zu bytes given, %zu needed", table_bytes, need);
        return SBR_E_SCRATCH;
    }
    int rc;
    for (int i = 0; i < n; i++) {
        const sbr_request &q = reqs[i];
        if ((rc = check_backward(q.mesh, q.mats, q.n_mats, q.radar, q.rays, q.hits, q.chirp, q.flags, q.grad_if,
                                 q.grad_verts, q.params, q.scratch, q.scratch_bytes))) {
            const std::string msg = sbr_last_error();
            set_error("request %d: %s", i, msg.c_str());
            return rc;
        }
    }
    {
        std::vector<Span> sp;
        for (int i = 0; i < n; i++) {
            const sbr_request &q = reqs[i];
            sp.push_back({(uintptr_t)q.scratch, (uintptr_t)q.scratch + q.scratch_bytes, i, "scratch"});
            sp.push_back({(uintptr_t)q.grad_verts, (uintptr_t)q.grad_verts + (size_t)q.mesh->nv * 3 * sizeof(float),
                          i, "grad_verts"});
            if (q.params) {
                const sbr_param_grads &g = *q.params;
                const size_t nm = (size_t)(q.mats ? q.n_mats : 0);
                sp.push_back({(uintptr_t)g.materials, (uintptr_t)g.materials + (g.materials ? 2 * nm * sizeof(float) : 0),
                              i, "params.materials"});
                sp.push_back({(uintptr_t)g.radar, (uintptr_t)g.radar + (g.radar ? 6 * sizeof(float) : 0), i,
                              "params.radar"});
                sp.push_back({(uintptr_t)g.rot, (uintptr_t)g.rot + (g.rot ? 9 * sizeof(float) : 0), i, "params.rot"});
                sp.push_back({(uintptr_t)g.attenuation, (uintptr_t)g.attenuation + (g.attenuation ? sizeof(float) : 0),
                              i, "params.attenuation"});
            }
        }
        if ((rc = check_disjoint(sp))) return rc;
    }
    hipStream_t s = (hipStream_t)stream;
    std::vector<BackwardReq> qs;
    for (int i = 0; i < n; i++) {
        const sbr_request &q = reqs[i];
        BackwardReq b;
        int skip = 0;
        if ((rc = enqueue_backward(q.mesh, q.mats, q.n_mats, q.radar, q.rays, q.hits, q.chirp, q.flags, q.grad_if,
                                   q.grad_verts, q.params, q.scratch, s, &b, nullptr, &skip)))
            return rc;
        if (!skip) qs.push_back(b);
    }
    return launch_backward_batch(qs.data(), (int)qs.size(), table, s);
}

int sbr_radar_cube(const float *in, int32_t V, int32_t C, int32_t S, int32_t n_angle, int32_t window,
                   int32_t direction, float *out, void *scratch, size_t scratch_bytes, void *stream) {
    clear_error();
    SBR_CHECK_ARG(in && out, "in/out is NULL");
    SBR_CHECK_ARG(V >= 1 && C >= 1 && S >= 1, "sizes must be >= 1 (V=%d C=%d S=%d)", V, C, S);
    SBR_CHECK_ARG(V <= 4096 && C <= 4096 && S <= 4096 && n_angle <= 4096, "sizes must be <= 4096");
    SBR_CHECK_ARG(n_angle >= V, "n_angle=%d < V=%d", n_angle, V);
    SBR_CHECK_ARG(window == 0 || window == 1, "window must be 0 or 1");
    SBR_CHECK_ARG(direction == 0 || direction == 1, "direction must be 0 or 1");
    size_t need = cube_scratch_bytes(V, C, S, n_angle);
    if (!scratch || scratch_bytes < need) {
        set_error("radar cube scratch too small: %zu bytes given, %zu needed", scratch_bytes, need);
        return SBR_E_SCRATCH;
    }
    return radar_cube_launch(reinterpret_cast<const float2 *>(in), V, C, S, n_angle, window, direction,
                             reinterpret_cast<float2 *>(out), scratch, (hipStream_t)stream);
}

int sbr_radar_cube_noalloc(const float *in, int32_t V, int32_t C, int32_t S, int32_t n_angle, int32_t window,
                           int32_t direction, float *out, void *stream) {
    clear_error();
    SBR_CHECK_ARG(in && out, "in/out is NULL");
    SBR_CHECK_ARG(V >= 1 && C >= 1 && S >= 1, "sizes must be >= 1 (V=%d C=%d S=%d)", V, C, S);
    SBR_CHECK_ARG(V <= 4096 && C <= 4096 && S <= 4096 && n_angle <= 4096, "sizes must be <= 4096");
    SBR_CHECK_ARG(n_angle >= V, "n_angle=%d < V=%d", n_angle, V);
    SBR_CHECK_ARG(window == 0 || window == 1, "window must be 0 or 1");
    SBR_CHECK_ARG(direction == 0 || direction == 1, "direction must be 0 or 1");
    const size_t need = cube_scratch_bytes(V, C, S, n_angle);
    if (need > (size_t)SBR_NOALLOC_SCRATCH_BYTES) {
        set_error("radar cube of %d x %d x %d -> %d angles needs %zu bytes of staging, more than the %d bytes "
                  "the scratch-free entry point holds; use sbr_radar_cube with a caller scratch",
                  V, C, S, n_angle, need, SBR_NOALLOC_SCRATCH_BYTES);
        return SBR_E_SCRATCH;
    }
    void *scratch = nullptr;
    int rc;
    if ((rc = noalloc_scratch(&scratch))) return rc;
    return radar_cube_launch(reinterpret_cast<const float2 *>(in), V, C, S, n_angle, window, direction,
                             reinterpret_cast<float2 *>(out), scratch, (hipStream_t)stream);
}

static int check_cube2(int32_t Vx, int32_t Vy, int32_t C, int32_t S, int32_t n_ax, int32_t n_ay) {
    SBR_CHECK_ARG(Vx >= 1 && Vy >= 1 && C >= 1 && S >= 1, "sizes must be >= 1 (Vx=%d Vy=%d C=%d S=%d)", Vx, Vy,
                  C, S);
    SBR_CHECK_ARG(Vx <= 4096 && Vy <= 4096 && C <= 4096 && S <= 4096 && n_ax <= 4096 && n_ay <= 4096,
                  "sizes must be <= 4096");
    SBR_CHECK_ARG(n_ax >= Vx && n_ay >= Vy, "n_ax=%d < Vx=%d or n_ay=%d < Vy=%d", n_ax, Vx, n_ay, Vy);
    SBR_CHECK_ARG((long long)n_ax * n_ay * C * S < (1LL << 31) - 64 && (long long)Vx * Vy * C * S < (1LL << 31) - 64,
                  "cube too large (2^31 cells or more)");
    return SBR_OK;
}

size_t sbr_radar_cube_2d_bytes(int32_t Vx, int32_t Vy, int32_t C, int32_t S, int32_t n_ax, int32_t n_ay) {
    clear_error();
    if (check_cube2(Vx, Vy, C, S, n_ax, n_ay)) return 0;
    return cube2_scratch_bytes(Vx, Vy, C, S, n_ax, n_ay);
}

int sbr_radar_cube_2d(const float *in, int32_t Vx, int32_t Vy, int32_t C, int32_t S, int32_t n_ax, int32_t n_ay,
                      int32_t window, int32_t direction, float *out, void *scratch, size_t scratch_bytes,
                      void *stream) {
    clear_error();
    SBR_CHECK_ARG(in && out, "in/out is NULL");
    int rc;
    if ((rc = check_cube2(Vx, Vy, C, S, n_ax, n_ay))) return rc;
    SBR_CHECK_ARG(window == 0 || window == 1, "window must be 0 or 1");
    SBR_CHECK_ARG(direction == 0 || direction == 1, "direction must be 0 or 1");
    size_t need = cube2_scratch_bytes(Vx, Vy, C, S, n_ax, n_ay);
    if (!scratch || scratch_bytes < need) {
        set_error("radar cube scratch too small: %zu bytes given, %zu needed", scratch_bytes, need);
        return SBR_E_SCRATCH;
    }
    return radar_cube2_launch(reinterpret_cast<const float2 *>(in), Vx, Vy, C, S, n_ax, n_ay, window, direction,
                              reinterpret_cast<float2 *>(out), scratch, (hipStream_t)stream);
}

size_t sbr_angle_peaks_bytes(int32_t max_det, int32_t n_ax, int32_t n_ay) {
    clear_error();
    if (max_det < 0 || n_ax < 1 || n_ay < 1 || (long long)n_ax * n_ay > 65536) return 0;
    return peaks_scratch_bytes(max_det, n_ax * n_ay);
}

int sbr_angle_peaks(const float *cube, int32_t n_ax, int32_t n_ay, int32_t C, int32_t S, const int32_t *det,
                    const int32_t *n_det, int32_t max_det, float rel, int32_t *points, int32_t max_points,
                    int32_t *n_points, void *scratch, size_t scratch_bytes, void *stream) {
    clear_error();
    SBR_CHECK_ARG(cube && n_det && n_points, "cube/n_det/n_points is NULL");
    SBR_CHECK_ARG(n_ax >= 1 && n_ay >= 1 && (long long)n_ax * n_ay <= 65536, "angle grid out of range");
    SBR_CHECK_ARG(C >= 1 && S >= 1 && (long long)C * S * n_ax * n_ay < (1LL << 31), "cube size out of range");
    SBR_CHECK_ARG(max_det >= 0 && (max_det == 0 || det), "det is NULL");
    SBR_CHECK_ARG(max_points >= 0 && (max_points == 0 || points), "points is NULL");
    SBR_CHECK_ARG((long long)max_det * n_ax * n_ay < (1LL << 31), "max_det * angle bins too large");
    SBR_CHECK_ARG(rel >= 0.0f && rel <= 1.0f, "rel must be in [0, 1]");
    size_t need = peaks_scratch_bytes(max_det, n_ax * n_ay);
    if (!scratch || scratch_bytes < need) {
        set_error("angle-peak scratch too small: %zu bytes given, %zu needed", scratch_bytes, need);
        return SBR_E_SCRATCH;
    }
    return peaks_launch(reinterpret_cast<const float2 *>(cube), n_ax, n_ay, C, S, det, n_det, max_det, rel, points,
                        max_points, n_points, scratch, (hipStream_t)stream);
}

int sbr_cloud(const int32_t *points, const int32_t *n_points, int32_t max_points, const sbr_radar *radar,
              const sbr_chirp *chirp, int32_t n_ax, int32_t n_ay, float *out, void *stream) {
    clear_error();
    SBR_CHECK_ARG(radar && chirp && n_points, "radar/chirp/n_points is NULL");
    SBR_CHECK_ARG(max_points >= 0 && (max_points == 0 || (points && out)), "points/out is NULL");
    SBR_CHECK_ARG(n_ax >= 1 && n_ay >= 1 && n_ax <= 4096 && n_ay <= 4096, "n_ax/n_ay out of [1, 4096]");
    SBR_CHECK_ARG(chirp->n_samples >= 1 && chirp->n_chirps >= 1 && chirp->fs > 0.0 && chirp->slope > 0.0 &&
                      chirp->fc > 0.0 && chirp->t_chirp > 0.0,
                  "chirp parameters must be positive");
    return cloud_launch(points, n_points, max_points, make_radar(radar), make_chirp(chirp), n_ax, n_ay, out,
                        (hipStream_t)stream);
}

int sbr_cfar(const float *cube, int32_t Na, int32_t C, int32_t S, int32_t guard, int32_t train, double pfa,
             int32_t *points, float *ratio, int32_t max_points, int32_t *n_points, void *scratch,
             size_t scratch_bytes, void *stream) {
    clear_error();
    SBR_CHECK_ARG(cube && n_points, "cube/n_points is NULL");
    SBR_CHECK_ARG(max_points >= 0 && (max_points == 0 || points), "points is NULL");
    SBR_CHECK_ARG(Na >= 1 && C >= 1 && S >= 1, "sizes must be >= 1");
    SBR_CHECK_ARG(Na <= 65536 && C <= 4096 && S <= 4096, "sizes out of range (Na <= 65536, C and S <= 4096)");
    SBR_CHECK_ARG(guard >= 0 && train >= 1 && guard + train < 4096, "guard >= 0, train >= 1, guard + train < 4096");
    SBR_CHECK_ARG(pfa > 0.0 && pfa < 1.0, "pfa must be in (0, 1)");
    size_t need = cfar_scratch_bytes(C, S);
    if (!scratch || scratch_bytes < need) {
        set_error("cfar scratch too small: %zu bytes given, %zu needed", scratch_bytes, need);
        return SBR_E_SCRATCH;
    }
    return cfar_launch(reinterpret_cast<const float2 *>(cube), Na, C, S, guard, train, pfa, points, ratio,
                       max_points, n_points, scratch, (hipStream_t)stream);
}

int sbr_backward(const sbr_mesh *mesh, const sbr_material *mats, int32_t n_mats, const sbr_radar *radar,
                 const sbr_rays *rays, const sbr_hits *hits, const sbr_chirp *chirp, int32_t flags,
                 const float *grad_if, float *grad_verts, const sbr_param_grads *params, void *scratch,
                 size_t scratch_bytes, void *stream) {
    clear_error();
    int rc;
    if ((rc = check_backward(mesh, mats, n_mats, radar, rays, hits, chirp, flags, grad_if, grad_verts, params,
                             scratch, scratch_bytes)))
        return rc;
    hipStream_t s = (hipStream_t)stream;
    BackwardReq q;
    void *table = nullptr;
    int skip = 0;
    if ((rc = enqueue_backward(mesh, mats, n_mats, radar, rays, hits, chirp, flags, grad_if, grad_verts, params,
                               scratch, s, &q, &table, &skip)))
        return rc;
    if (skip) return SBR_OK;
    return launch_backward_batch(&q, 1, table, s);
}

}  // extern "C"
