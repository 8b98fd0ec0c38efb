// Linear BVH over the triangle mesh: Morton codes, LSD radix sort, binary
// radix tree (Karras, HPG 2012), bottom-up boxes, depth-first relayout with
// escape links for stackless traversal.  Refit reuses the tree.
#include "sbr_internal.h"

namespace sbr {

namespace {

constexpr int kThreads = 256;
constexpr int kRsItems = 8;
constexpr int kRsTile = kThreads * kRsItems;

__device__ __forceinline__ uint32_t f2ord(float f) {
    uint32_t b = __float_as_uint(f);
    return (b & 0x80000000u) ? ~b : (b | 0x80000000u);
}
__device__ __forceinline__ float ord2f(uint32_t u) {
    return __uint_as_float((u & 0x80000000u) ? (u & 0x7fffffffu) : ~u);
}

__device__ __forceinline__ float3 load_vert(const float *v, int i) {
    return make_float3(v[3 * i], v[3 * i + 1], v[3 * i + 2]);
}

// every node starts as an empty box that ends traversal
__global__ void k_init_nodes(BvhNode *nodes, int nn) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nn) return;
    BvhNode z;
    for (int k = 0; k < 3; k++) {
        z.lo[k] = INFINITY;
        z.hi[k] = -INFINITY;
    }
    z.escape = nn;
    z.leaf = -1;
    nodes[i] = z;
}

__global__ void k_fill_u32(uint32_t *p, uint32_t val, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = val;
}

// centroid bounds: bounds[0..2] ordered-min, bounds[3..5] ordered-max
__global__ void k_bounds(const float *verts, const int32_t *faces, int nf, uint32_t *bounds) {
    __shared__ uint32_t red[6];
    if (threadIdx.x < 6) red[threadIdx.x] = threadIdx.x < 3 ? 0xffffffffu : 0u;
    __syncthreads();
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    uint32_t v[6] = {0xffffffffu, 0xffffffffu, 0xffffffffu, 0u, 0u, 0u};
    if (f < nf) {
        float3 a = load_vert(verts, faces[3 * f]);
        float3 b = load_vert(verts, faces[3 * f + 1]);
        float3 c = load_vert(verts, faces[3 * f + 2]);
        float cx = (a.x + b.x + c.x) * (1.0f / 3.0f);
        float cy = (a.y + b.y + c.y) * (1.0f / 3.0f);
        float cz = (a.z + b.z + c.z) * (1.0f / 3.0f);
        v[0] = v[3] = f2ord(cx);
        v[1] = v[4] = f2ord(cy);
        v[2] = v[5] = f2ord(cz);
    }
    // wavefront min / max first, then one LDS atomic per wavefront and value
#pragma unroll
    for (int off = 32; off >= 1; off >>= 1) {
#pragma unroll
        for (int q = 0; q < 3; q++) {
            v[q] = min(v[q], (uint32_t)__shfl_xor((int)v[q], off));
            v[3 + q] = max(v[3 + q], (uint32_t)__shfl_xor((int)v[3 + q], off));
        }
    }
    if ((threadIdx.x & 63) == 0) {
        for (int q = 0; q < 3; q++) {
            atomicMin(&red[q], v[q]);
            atomicMax(&red[3 + q], v[3 + q]);
        }
    }
    __syncthreads();
    if (threadIdx.x < 3) atomicMin(&bounds[threadIdx.x], red[threadIdx.x]);
    else if (threadIdx.x < 6) atomicMax(&bounds[threadIdx.x], red[threadIdx.x]);
}

__device__ __forceinline__ uint32_t expand_bits10(uint32_t v) {
    v = (v * 0x00010001u) & 0xFF0000FFu;
    v = (v * 0x00000101u) & 0x0F00F00Fu;
    v = (v * 0x00000011u) & 0xC30C30C3u;
    v = (v * 0x00000005u) & 0x49249249u;
    return v;
}

__global__ void k_morton(const float *verts, const int32_t *faces, int nf, const uint32_t *bounds,
                         uint32_t *keys, int32_t *vals) {
    int f = blockIdx.x * blockDim.x + threadIdx.x;
    if (f >= nf) return;
    float lo[3], ext[3];
    for (int i = 0; i < 3; i++) {
        lo[i] = ord2f(bounds[i]);
        ext[i] = ord2f(bounds[3 + i]) - lo[i];
    }
    float3 a = load_vert(verts, faces[3 * f]);
    float3 b = load_vert(verts, faces[3 * f + 1]);
    float3 c = load_vert(verts, faces[3 * f + 2]);
    float cc[3] = {(a.x + b.x + c.x) * (1.0f / 3.0f), (a.y + b.y + c.y) * (1.0f / 3.0f),
                   (a.z + b.z + c.z) * (1.0f / 3.0f)};
    uint32_t q[3];
    for (int i = 0; i < 3; i++) {
        float t = ext[i] > 0.0f ? (cc[i] - lo[i]) / ext[i] : 0.5f;
        t = fminf(fmaxf(t * 1024.0f, 0.0f), 1023.0f);
        q[i] = (uint32_t)t;
    }
    keys[f] = (expand_bits10(q[0]) << 2) | (expand_bits10(q[1]) << 1) | expand_bits10(q[2]);
    vals[f] = f;
}

// ---- LSD radix sort, 8-bit digits, stable --------------------------------
__global__ void k_rs_hist(const uint32_t *keys, int n, int shift, uint32_t *hist, int nblk) {
    __shared__ uint32_t h[256];
    h[threadIdx.x] = 0;
    __syncthreads();
    int base = blockIdx.x * kRsTile;
    for (int it = 0; it < kRsItems; it++) {
        int i = base + it * kThreads + threadIdx.x;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[threadIdx.x * nblk + blockIdx.x] = h[threadIdx.x];
}

// exclusive scan of n values in place, one block of 1024 threads
__global__ __launch_bounds__(1024) void k_scan_u32(uint32_t *a, int n, uint32_t *total) {
    __shared__ uint32_t part[1024];
    int t = threadIdx.x;
    int chunk = (n + 1023) / 1024;
    int b = t * chunk, e = min(n, b + chunk);
    uint32_t s = 0;
    for (int i = b; i < e; i++) s += a[i];
    part[t] = s;
    __syncthreads();
    for (int off = 1; off < 1024; off <<= 1) {
        uint32_t v = t >= off ? part[t - off] : 0u;
        __syncthreads();
        part[t] += v;
        __syncthreads();
    }
    uint32_t run = part[t] - s;
    for (int i = b; i < e; i++) {
        uint32_t x = a[i];
        a[i] = run;
        run += x;
    }
    if (t == 1023 && total) *total = part[1023];
}

__global__ __launch_bounds__(kThreads) void k_rs_scatter(const uint32_t *kin, const int32_t *vin,
                                                         uint32_t *kout, int32_t *vout, int n,
                                                         int shift, const uint32_t *offs, int nblk) {
    __shared__ uint32_t base_d[256];
    __shared__ uint32_t wcnt[kThreads / 64][256];
    const int t = threadIdx.x, w = t >> 6, lane = t & 63;
    base_d[t] = offs[t * nblk + blockIdx.x];
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64 - lane));
    for (int it = 0; it < kRsItems; it++) {
        for (int j = 0; j < kThreads / 64; j++) wcnt[j][t] = 0;
        __syncthreads();
        int i = blockIdx.x * kRsTile + it * kThreads + t;
        bool valid = i < n;
        uint32_t key = valid ? kin[i] : 0u;
        int32_t val = valid ? vin[i] : 0;
        uint32_t dg = (key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
        for (int b = 0; b < 8; b++) {
            bool bit = (dg >> b) & 1u;
            uint64_t m = __ballot(valid && bit);
            peers &= bit ? m : ~m;
        }
        uint32_t rank = __popcll(peers & lt);
        if (valid && rank == 0) wcnt[w][dg] = __popcll(peers);
        __syncthreads();
        if (valid) {
            uint32_t pos = base_d[dg] + rank;
            for (int j = 0; j < w; j++) pos += wcnt[j][dg];
            kout[pos] = key;
            vout[pos] = val;
        }
        __syncthreads();
        uint32_t add = 0;
        for (int j = 0; j < kThreads / 64; j++) add += wcnt[j][t];
        base_d[t] += add;
        __syncthreads();
    }
}

// ---- binary radix tree ----------------------------------------------------
__device__ __forceinline__ int prefix_len(const uint32_t *k, int n, int i, int j) {
    if (j < 0 || j >= n) return -1;
    uint32_t a = k[i], b = k[j];
    if (a == b) return 32 + __clz((uint32_t)(i ^ j));
    return __clz(a ^ b);
}

// tree indices: internal nodes 0..n-2, leaf slot i = n-1+i
__global__ void k_karras(const uint32_t *keys, int n, int32_t *parent, int2 *child, int2 *range) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n - 1) return;
    int d = prefix_len(keys, n, i, i + 1) > prefix_len(keys, n, i, i - 1) ? 1 : -1;
    int dmin = prefix_len(keys, n, i, i - d);
    int lmax = 2;
    while (prefix_len(keys, n, i, i + lmax * d) > dmin) lmax <<= 1;
    int l = 0;
    for (int t = lmax >> 1; t >= 1; t >>= 1)
        if (prefix_len(keys, n, i, i + (l + t) * d) > dmin) l += t;
    int j = i + l * d;
    int dnode = prefix_len(keys, n, i, j);
    int s = 0;
    for (int div = 2;; div <<= 1) {
        int t = (l + div - 1) / div;
        if (prefix_len(keys, n, i, i + (s + t) * d) > dnode) s += t;
        if (t <= 1) break;
    }
    int g = i + s * d + min(d, 0);
    int lo = min(i, j), hi = max(i, j);
    int left = (lo == g) ? (n - 1 + g) : g;
    int right = (hi == g + 1) ? (n - 1 + g + 1) : g + 1;
    child[i] = make_int2(left, right);
    range[i] = make_int2(lo, hi);
    parent[left] = i;
    parent[right] = i;
    if (i == 0) parent[0] = -1;
}

// depth-first index = 2 * (first leaf) + (left turns on the root path);
// escape = index + subtree size (2 * leaves - 1)
__global__ void k_dfs(int n, const int32_t *parent, const int2 *child, const int2 *range,
                      int32_t *dfs_of, BvhNode *nodes) {
    int x = blockIdx.x * blockDim.x + threadIdx.x;
    int nn = 2 * n - 1;
    if (x >= nn) return;
    int first, nleaf;
    if (x >= n - 1) {
        first = x - (n - 1);
        nleaf = 1;
    } else {
        int2 r = range[x];
        first = r.x;
        nleaf = r.y - r.x + 1;
    }
    int lefts = 0;
    int c = x;
    if (n > 1) {
        while (true) {
            int p = parent[c];
            if (p < 0) break;
            if (child[p].x == c) lefts++;
            c = p;
        }
    }
    int di = 2 * first + lefts;
    dfs_of[x] = di;
    nodes[di].escape = di + 2 * nleaf - 1;
    nodes[di].leaf = (x >= n - 1) ? first : -1;
}

__device__ __forceinline__ float ld_coherent(const float *p) {
    return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// header of a finished BUILD: face count and seal
__global__ void k_bvh_seal(int32_t *header, int n) {
    if (threadIdx.x == 0) {
        header[0] = n;
        header[1] = kBvhMagic;
        header[2] = 0;
    }
}

// bottom-up arrival counters cleared for a refit, only in a buffer sealed
// for this face count (its layout is then the one bvh_view computes)
__global__ void k_zero_visits(const int32_t *header, int n, uint32_t *visits) {
    if (header[1] != kBvhMagic || header[0] != n) return;
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n - 1) visits[i] = 0u;
}

// leaf triangles + boxes, then bottom-up unions (second arrival continues).
// The stored order, parent, child and depth-first maps are followed only in a
// buffer sealed by a BUILD for this face count; otherwise nothing is written
// but the header's refit-rejected word.
__global__ void k_leaves(const float *verts, const int32_t *faces, BvhView bv) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    int n = bv.n;
    if (bv.header[1] != kBvhMagic || bv.header[0] != n) {
        if (i == 0) bv.header[2] = 1;
        return;
    }
    if (i >= n) return;
    int f = bv.order[i];
    float3 a = load_vert(verts, faces[3 * f]);
    float3 b = load_vert(verts, faces[3 * f + 1]);
    float3 c = load_vert(verts, faces[3 * f + 2]);
    LeafTri lt;
    lt.a = make_float4(a.x, a.y, a.z, __int_as_float(f));
    lt.b = make_float4(b.x, b.y, b.z, 0.0f);
    lt.c = make_float4(c.x, c.y, c.z, 0.0f);
    bv.tris[i] = lt;
    float lo[3] = {fminf(a.x, fminf(b.x, c.x)), fminf(a.y, fminf(b.y, c.y)), fminf(a.z, fminf(b.z, c.z))};
    float hi[3] = {fmaxf(a.x, fmaxf(b.x, c.x)), fmaxf(a.y, fmaxf(b.y, c.y)), fmaxf(a.z, fmaxf(b.z, c.z))};
    // pad by a few ulps so rounding in the slab test never culls a true hit
    for (int k = 0; k < 3; k++) {
        float m = fmaxf(fabsf(lo[k]), fabsf(hi[k]));
        float pad = m * 2.4e-7f + 1e-30f;
        lo[k] -= pad;
        hi[k] += pad;
    }
    int x = n - 1 + i;
    BvhNode *nd = &bv.nodes[bv.dfs_of[x]];
    for (int k = 0; k < 3; k++) {
        nd->lo[k] = lo[k];
        nd->hi[k] = hi[k];
    }
    int p = bv.parent[x];
    // the acquire-release counter orders this thread's box stores before the
    // sibling thread's reads of them (no separate fence)
    while (p >= 0) {
        uint32_t prev = __hip_atomic_fetch_add(&bv.visits[p], 1u, __ATOMIC_ACQ_REL,
                                               __HIP_MEMORY_SCOPE_AGENT);
        if (prev == 0) return;  // sibling subtree not finished; it will continue
        int2 ch = bv.child[p];
        const BvhNode *l = &bv.nodes[bv.dfs_of[ch.x]];
        const BvhNode *r = &bv.nodes[bv.dfs_of[ch.y]];
        BvhNode *q = &bv.nodes[bv.dfs_of[p]];
        for (int k = 0; k < 3; k++) {
            q->lo[k] = fminf(ld_coherent(&l->lo[k]), ld_coherent(&r->lo[k]));
            q->hi[k] = fmaxf(ld_coherent(&l->hi[k]), ld_coherent(&r->hi[k]));
        }
        p = bv.parent[p];
    }
}

}  // namespace

BvhView bvh_view(void *buf, int32_t nf, size_t *bytes_out) {
    Carver cv(buf);
    BvhView v;
    v.n = nf;
    v.n_nodes = 2 * nf - 1;
    v.header = cv.take<int32_t>(16);
    v.nodes = cv.take<BvhNode>(v.n_nodes);
    v.tris = cv.take<LeafTri>(nf);
    v.order = cv.take<int32_t>(nf);
    v.parent = cv.take<int32_t>(v.n_nodes);
    v.child = cv.take<int2>(nf > 1 ? nf - 1 : 1);
    v.dfs_of = cv.take<int32_t>(v.n_nodes);
    v.visits = cv.take<uint32_t>(nf > 1 ? nf - 1 : 1);
    if (bytes_out) *bytes_out = align_up(cv.off, 256);
    return v;
}

struct BuildScratch {
    uint32_t *bounds;
    uint32_t *keys[2];
    int32_t *vals[2];
    uint32_t *hist;
    int2 *range;
    int nblk;
};

static BuildScratch carve_build(void *buf, int32_t nf, size_t *bytes) {
    Carver cv(buf);
    BuildScratch s;
    s.nblk = (nf + kRsTile - 1) / kRsTile;
    s.bounds = cv.take<uint32_t>(8);
    s.keys[0] = cv.take<uint32_t>(nf);
    s.keys[1] = cv.take<uint32_t>(nf);
    s.vals[0] = cv.take<int32_t>(nf);
    s.vals[1] = cv.take<int32_t>(nf);
    s.hist = cv.take<uint32_t>((size_t)256 * s.nblk);
    s.range = cv.take<int2>(nf > 1 ? nf - 1 : 1);
    if (bytes) *bytes = align_up(cv.off, 256);
    return s;
}

size_t build_scratch_bytes(int32_t nf) {
    size_t b = 0;
    carve_build(nullptr, nf, &b);
    return b;
}

static inline int nblocks(long long n, int t) { return (int)((n + t - 1) / t); }

int bvh_build(const sbr_mesh *m, void *bvh, size_t bvh_bytes, int32_t mode, void *scratch,
              size_t scratch_bytes, hipStream_t st) {
    const int nf = m->nf;
    size_t need = 0;
    BvhView bv = bvh_view(bvh, nf, &need);
    if (bvh_bytes < need) {
        set_error("BVH buffer too small: %zu bytes given, %zu needed", bvh_bytes, need);
        return SBR_E_SCRATCH;
    }
    if (mode == 0) {
        size_t sneed = 0;
        BuildScratch s = carve_build(scratch, nf, &sneed);
        if (!scratch || scratch_bytes < sneed) {
            set_error("BVH build scratch too small: %zu bytes given, %zu needed", scratch_bytes, sneed);
            return SBR_E_SCRATCH;
        }
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, s.bounds, 0xffffffffu, 3);
        hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, s.bounds + 3, 0u, 3);
        hipLaunchKernelGGL(k_bounds, dim3(nblocks(nf, kThreads)), dim3(kThreads), 0, st, m->verts,
                           m->faces, nf, s.bounds);
        hipLaunchKernelGGL(k_morton, dim3(nblocks(nf, kThreads)), dim3(kThreads), 0, st, m->verts,
                           m->faces, nf, s.bounds, s.keys[0], s.vals[0]);
        SBR_LAUNCHED();
        int cur = 0;
        for (int pass = 0; pass < 4; pass++) {
            int shift = 8 * pass;
            hipLaunchKernelGGL(k_rs_hist, dim3(s.nblk), dim3(kThreads), 0, st, s.keys[cur], nf, shift,
                               s.hist, s.nblk);
            hipLaunchKernelGGL(k_scan_u32, dim3(1), dim3(1024), 0, st, s.hist, 256 * s.nblk,
                               (uint32_t *)nullptr);
            hipLaunchKernelGGL(k_rs_scatter, dim3(s.nblk), dim3(kThreads), 0, st, s.keys[cur],
                               s.vals[cur], s.keys[1 - cur], s.vals[1 - cur], nf, shift, s.hist, s.nblk);
            cur = 1 - cur;
        }
        SBR_LAUNCHED();
        SBR_HIP(hipMemcpyAsync(bv.order, s.vals[cur], sizeof(int32_t) * nf, hipMemcpyDeviceToDevice, st));
        if (nf > 1) {
            hipLaunchKernelGGL(k_karras, dim3(nblocks(nf - 1, kThreads)), dim3(kThreads), 0, st,
                               s.keys[cur], nf, bv.parent, bv.child, s.range);
        } else {
            hipLaunchKernelGGL(k_fill_u32, dim3(1), dim3(64), 0, st, (uint32_t *)bv.parent, 0xffffffffu, 1);
        }
        hipLaunchKernelGGL(k_init_nodes, dim3(nblocks(2 * nf - 1, kThreads)), dim3(kThreads), 0, st, bv.nodes,
                           2 * nf - 1);
        hipLaunchKernelGGL(k_dfs, dim3(nblocks(2 * nf - 1, kThreads)), dim3(kThreads), 0, st, nf,
                           bv.parent, bv.child, s.range, bv.dfs_of, bv.nodes);
        hipLaunchKernelGGL(k_bvh_seal, dim3(1), dim3(64), 0, st, bv.header, nf);
        SBR_LAUNCHED();
    }
    if (nf > 1)
        hipLaunchKernelGGL(k_zero_visits, dim3(nblocks(nf - 1, kThreads)), dim3(kThreads), 0, st, bv.header, nf,
                           bv.visits);
    hipLaunchKernelGGL(k_leaves, dim3(nblocks(nf, kThreads)), dim3(kThreads), 0, st, m->verts,
                       m->faces, bv);
    SBR_LAUNCHED();
    return SBR_OK;
}

}  // namespace sbr
