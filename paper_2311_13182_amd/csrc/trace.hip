// Ray launch + stackless BVH traversal + watertight ray-triangle test +
// specular multi-bounce, one lane per ray, 8x8 ray tiles per wavefront.
#include "sbr_internal.h"
#include "sbr_device.h"

namespace sbr {

namespace {

struct TraceArgs {
    const int32_t *header;   // BVH header: [0] faces, [1] seal
    const BvhNode *nodes;
    const LeafTri *tris;
    int32_t n_nodes;
    int32_t n_tris;
    GridDev g;
    double o[3];
    double rot[9];
    int32_t *tri;
    float *t;
    float *u;
    float *v;
    uint8_t *flags;
    unsigned long long *counters;
};

__device__ __forceinline__ float sel3(float3 p, int k) { return k == 0 ? p.x : (k == 1 ? p.y : p.z); }

struct Shear {
    int kx, ky, kz;
    float sx, sy, sz;
};

// Watertight ray/triangle intersection (Woop, Benthin, Wald, JCGT 2013),
// two-sided, inclusive edges.  Returns t and the barycentric weights.
__device__ __forceinline__ bool wt_hit(const Shear &sh, float3 o, float3 a, float3 b, float3 c,
                                       float &t, float &b0, float &b1, float &b2) {
    float3 A = make_float3(a.x - o.x, a.y - o.y, a.z - o.z);
    float3 B = make_float3(b.x - o.x, b.y - o.y, b.z - o.z);
    float3 C = make_float3(c.x - o.x, c.y - o.y, c.z - o.z);
    float Az = sel3(A, sh.kz), Bz = sel3(B, sh.kz), Cz = sel3(C, sh.kz);
    float Ax = fmaf(-sh.sx, Az, sel3(A, sh.kx));
    float Ay = fmaf(-sh.sy, Az, sel3(A, sh.ky));
    float Bx = fmaf(-sh.sx, Bz, sel3(B, sh.kx));
    float By = fmaf(-sh.sy, Bz, sel3(B, sh.ky));
    float Cx = fmaf(-sh.sx, Cz, sel3(C, sh.kx));
    float Cy = fmaf(-sh.sy, Cz, sel3(C, sh.ky));
    float U = Cx * By - Cy * Bx;
    float V = Ax * Cy - Ay * Cx;
    float W = Bx * Ay - By * Ax;
    if ((U < 0.0f || V < 0.0f || W < 0.0f) && (U > 0.0f || V > 0.0f || W > 0.0f)) return false;
    float det = U + V + W;
    if (det == 0.0f) return false;
    float T = U * (sh.sz * Az) + V * (sh.sz * Bz) + W * (sh.sz * Cz);
    float inv = 1.0f / det;
    t = T * inv;
    b0 = U * inv;
    b1 = V * inv;
    b2 = W * inv;
    return true;
}

__device__ __forceinline__ Shear make_shear(float3 d) {
    Shear sh;
    float ax = fabsf(d.x), ay = fabsf(d.y), az = fabsf(d.z);
    sh.kz = (ax > ay) ? (ax > az ? 0 : 2) : (ay > az ? 1 : 2);
    sh.kx = sh.kz == 2 ? 0 : sh.kz + 1;
    sh.ky = sh.kx == 2 ? 0 : sh.kx + 1;
    float dz = sel3(d, sh.kz);
    if (dz < 0.0f) {
        int tmp = sh.kx;
        sh.kx = sh.ky;
        sh.ky = tmp;
    }
    sh.sx = sel3(d, sh.kx) / dz;
    sh.sy = sel3(d, sh.ky) / dz;
    sh.sz = 1.0f / dz;
    return sh;
}

// Any hit of a triangle other than `self` at t in (tmin, tmax) along the unit
// direction s from x: the occlusion test of a return segment.  Same stackless
// walk as the closest-hit query, leaving at the first accepted hit.
__device__ bool any_hit(const TraceArgs &a, int n_nodes, float3 x, float3 s, float tmin, float tmax, int self) {
    const Shear sh = make_shear(s);
    float3 id;
    id.x = 1.0f / (fabsf(s.x) > 1e-30f ? s.x : copysignf(1e-30f, s.x));
    id.y = 1.0f / (fabsf(s.y) > 1e-30f ? s.y : copysignf(1e-30f, s.y));
    id.z = 1.0f / (fabsf(s.z) > 1e-30f ? s.z : copysignf(1e-30f, s.z));
    const float3 oid = make_float3(x.x * id.x, x.y * id.y, x.z * id.z);
    int i = 0;
    while (i < n_nodes) {
        const BvhNode nd = a.nodes[i];
        float tx0 = fmaf(nd.lo[0], id.x, -oid.x), tx1 = fmaf(nd.hi[0], id.x, -oid.x);
        float ty0 = fmaf(nd.lo[1], id.y, -oid.y), ty1 = fmaf(nd.hi[1], id.y, -oid.y);
        float tz0 = fmaf(nd.lo[2], id.z, -oid.z), tz1 = fmaf(nd.hi[2], id.z, -oid.z);
        float tn = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
        float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1));
        tf *= 1.0000005f;
        const bool hit = tn <= tf && tn <= tmax;
        const int esc = nd.escape > i ? nd.escape : i + 1;
        if (!hit) {
            i = esc;
            continue;
        }
        if (nd.leaf < 0) {
            i++;
            continue;
        }
        if (nd.leaf < a.n_tris) {
            const LeafTri lt = a.tris[nd.leaf];
            float th, c0, c1, c2;
            if (__float_as_int(lt.a.w) != self &&
                wt_hit(sh, x, make_float3(lt.a.x, lt.a.y, lt.a.z), make_float3(lt.b.x, lt.b.y, lt.b.z),
                       make_float3(lt.c.x, lt.c.y, lt.c.z), th, c0, c1, c2) &&
                th > tmin && th < tmax)
                return true;
        }
        i = esc;
    }
    return false;
}

template <bool COUNT, bool SHADOW>
__global__ __launch_bounds__(256) void k_trace(TraceArgs a) {
    const int gid = blockIdx.x * blockDim.x + threadIdx.x;
    const int tile = gid >> 6, l = gid & 63;
    const int tiles_x = (a.g.nx + 7) >> 3;
    const int ix = (tile % tiles_x) * 8 + (l & 7);
    const int iy = (tile / tiles_x) * 8 + (l >> 3);
    const bool active = ix < a.g.nx && iy < a.g.ny;
    // a buffer that no BUILD for this face count has sealed is never walked:
    // every ray misses
    const int n_nodes = (a.n_nodes > 0 && a.header[1] == kBvhMagic && a.header[0] == a.n_tris) ? a.n_nodes : 0;
    unsigned long long n_q = 0, n_node = 0, n_tri = 0;
    if (active) {
        const size_t R = (size_t)a.g.nx * a.g.ny;
        const size_t r = (size_t)iy * a.g.nx + ix;
        // ray of the grid, formed in double and rounded once
        double dr[3], dw_unused;
        grid_dir_local(a.g, ix, iy, dr, &dw_unused);
        float3 d, o;
        d.x = (float)(a.rot[0] * dr[0] + a.rot[1] * dr[1] + a.rot[2] * dr[2]);
        d.y = (float)(a.rot[3] * dr[0] + a.rot[4] * dr[1] + a.rot[5] * dr[2]);
        d.z = (float)(a.rot[6] * dr[0] + a.rot[7] * dr[1] + a.rot[8] * dr[2]);
        o = make_float3((float)a.o[0], (float)a.o[1], (float)a.o[2]);
        const float3 o0 = o;   // array centre: where every return ends
        const float tmin = (float)a.g.t_min;
        int prev = -1;
        float Lprev = 0.0f;
        uint8_t anc = 0;
        bool alive = true;
        for (int k = 0; k < a.g.K; k++) {
            const size_t slot = (size_t)k * R + r;
            if (!alive) {
                a.tri[slot] = -1;
                a.t[slot] = 0.0f;
                a.u[slot] = 0.0f;
                a.v[slot] = 0.0f;
                a.flags[slot] = 0;
                continue;
            }
            n_q++;
            // per-ray shear constants of the watertight test
            const Shear sh = make_shear(d);
            // slab-test reciprocals (zero components replaced by tiny values)
            float3 id;
            id.x = 1.0f / (fabsf(d.x) > 1e-30f ? d.x : copysignf(1e-30f, d.x));
            id.y = 1.0f / (fabsf(d.y) > 1e-30f ? d.y : copysignf(1e-30f, d.y));
            id.z = 1.0f / (fabsf(d.z) > 1e-30f ? d.z : copysignf(1e-30f, d.z));
            float3 oid = make_float3(o.x * id.x, o.y * id.y, o.z * id.z);

            int best = -1, bslot = -1;
            float t1 = INFINITY, t2 = INFINITY, bb0 = 0.f, bb1 = 0.f, bb2 = 0.f;
            float tlim = INFINITY;   // box cull limit: best t plus the tie margin
            int i = 0;
            while (i < n_nodes) {
                const BvhNode nd = a.nodes[i];
                if (COUNT) n_node++;
                float tx0 = fmaf(nd.lo[0], id.x, -oid.x), tx1 = fmaf(nd.hi[0], id.x, -oid.x);
                float ty0 = fmaf(nd.lo[1], id.y, -oid.y), ty1 = fmaf(nd.hi[1], id.y, -oid.y);
                float tz0 = fmaf(nd.lo[2], id.z, -oid.z), tz1 = fmaf(nd.hi[2], id.z, -oid.z);
                float tn = fmaxf(fmaxf(fminf(tx0, tx1), fminf(ty0, ty1)), fmaxf(fminf(tz0, tz1), 0.0f));
                float tf = fminf(fminf(fmaxf(tx0, tx1), fmaxf(ty0, ty1)), fmaxf(tz0, tz1));
                tf *= 1.0000005f;
                bool hit = tn <= tf && tn <= tlim;
                // escape links always point forward; the guard keeps the walk
                // finite even for a corrupted buffer
                const int esc = nd.escape > i ? nd.escape : i + 1;
                if (!hit) {
                    i = esc;
                    continue;
                }
                if (nd.leaf < 0) {
                    i++;
                    continue;
                }
                if (nd.leaf >= a.n_tris) {
                    i = esc;
                    continue;
                }
                const LeafTri lt = a.tris[nd.leaf];
                const int fid = __float_as_int(lt.a.w);
                if ((unsigned)fid >= (unsigned)a.n_tris) {   // not a face of this mesh
                    i = esc;
                    continue;
                }
                if (COUNT) n_tri++;
                float th, c0, c1, c2;
                if (fid != prev &&
                    wt_hit(sh, o, make_float3(lt.a.x, lt.a.y, lt.a.z), make_float3(lt.b.x, lt.b.y, lt.b.z),
                           make_float3(lt.c.x, lt.c.y, lt.c.z), th, c0, c1, c2) &&
                    th > tmin) {
                    if (th < t1 || (th == t1 && fid < best)) {
                        t2 = t1;
                        t1 = th;
                        best = fid;
                        bslot = nd.leaf;
                        bb0 = c0;
                        bb1 = c1;
                        bb2 = c2;
                        tlim = t1 + 1e-6f * fmaxf(1.0f, Lprev + t1);
                    } else if (th < t2) {
                        t2 = th;
                    }
                }
                i = esc;
            }
            if (best < 0) {
                alive = false;
                a.tri[slot] = -1;
                a.t[slot] = 0.0f;
                a.u[slot] = 0.0f;
                a.v[slot] = 0.0f;
                a.flags[slot] = 0;
                continue;
            }
            const LeafTri lt = a.tris[bslot];
            float3 v0 = make_float3(lt.a.x, lt.a.y, lt.a.z);
            float3 v1 = make_float3(lt.b.x, lt.b.y, lt.b.z);
            float3 v2 = make_float3(lt.c.x, lt.c.y, lt.c.z);
            float3 e1 = make_float3(v1.x - v0.x, v1.y - v0.y, v1.z - v0.z);
            float3 e2 = make_float3(v2.x - v0.x, v2.y - v0.y, v2.z - v0.z);
            float3 N = make_float3(e1.y * e2.z - e1.z * e2.y, e1.z * e2.x - e1.x * e2.z,
                                   e1.x * e2.y - e1.y * e2.x);
            float nl = sqrtf(N.x * N.x + N.y * N.y + N.z * N.z);
            float3 nh = make_float3(N.x / nl, N.y / nl, N.z / nl);
            float dn = d.x * nh.x + d.y * nh.y + d.z * nh.z;
            float Lk = Lprev + t1;
            float delta = 1e-6f * fmaxf(1.0f, Lk);
            // distance to the line of the edge opposite vertex i: b_i |N| / |e_i|
            float3 e0 = make_float3(v2.x - v1.x, v2.y - v1.y, v2.z - v1.z);
            float l0 = sqrtf(e0.x * e0.x + e0.y * e0.y + e0.z * e0.z);
            float l1 = sqrtf(e2.x * e2.x + e2.y * e2.y + e2.z * e2.z);
            float l2 = sqrtf(e1.x * e1.x + e1.y * e1.y + e1.z * e1.z);
            float de = fminf(fabsf(bb0) * nl / l0, fminf(fabsf(bb1) * nl / l1, fabsf(bb2) * nl / l2));
            uint8_t fl = anc ? SBR_HIT_PARENT : 0;
            if (de < delta) fl |= SBR_HIT_EDGE;
            if (t2 - t1 < delta) fl |= SBR_HIT_TIE;
            if (fabsf(dn) < 1e-6f) fl |= SBR_HIT_GRAZE;
            if (t1 < 2.0f * tmin) fl |= SBR_HIT_TMIN;
            anc |= fl;
            // the hit point (barycentric, lies on the face): the return's start
            // and the next bounce's origin
            o = make_float3(bb0 * v0.x + bb1 * v1.x + bb2 * v2.x, bb0 * v0.y + bb1 * v1.y + bb2 * v2.y,
                            bb0 * v0.z + bb1 * v1.z + bb2 * v2.z);
            if (SHADOW && k > 0) {
                const float3 q = make_float3(o0.x - o.x, o0.y - o.y, o0.z - o.z);
                const float D = sqrtf(q.x * q.x + q.y * q.y + q.z * q.z);
                const float3 sd = make_float3(q.x / D, q.y / D, q.z / D);
                if (any_hit(a, n_nodes, o, sd, tmin, D - tmin, best)) fl |= SBR_HIT_OCCLUDED;
            }
            a.tri[slot] = best;
            a.t[slot] = t1;
            a.u[slot] = bb1;
            a.v[slot] = bb2;
            a.flags[slot] = fl;
            d = make_float3(d.x - 2.0f * dn * nh.x, d.y - 2.0f * dn * nh.y, d.z - 2.0f * dn * nh.z);
            float dl = 1.0f / sqrtf(d.x * d.x + d.y * d.y + d.z * d.z);
            d = make_float3(d.x * dl, d.y * dl, d.z * dl);
            prev = best;
            Lprev = Lk;
        }
    }
    if (a.counters) {
        // wavefront sums, one atomic per wave and counter
        for (int off = 32; off >= 1; off >>= 1) {
            n_q += __shfl_xor(n_q, off);
            n_node += __shfl_xor(n_node, off);
            n_tri += __shfl_xor(n_tri, off);
        }
        if ((threadIdx.x & 63) == 0) {
            atomicAdd(&a.counters[0], n_q);
            if (COUNT) {
                atomicAdd(&a.counters[1], n_node);
                atomicAdd(&a.counters[2], n_tri);
            }
        }
    }
}

}  // namespace

int trace_launch(const sbr_mesh *m, const void *bvh, const RadarDev &rd, const GridDev &gd,
                 const sbr_hits *h, uint64_t *counters, hipStream_t st) {
    BvhView bv = bvh_view(const_cast<void *>(bvh), m->nf, nullptr);
    TraceArgs a;
    a.header = bv.header;
    a.nodes = bv.nodes;
    a.tris = bv.tris;
    a.n_nodes = m->nf > 0 ? bv.n_nodes : 0;
    a.n_tris = m->nf;
    a.g = gd;
    for (int i = 0; i < 3; i++) a.o[i] = rd.o[i];
    for (int i = 0; i < 9; i++) a.rot[i] = rd.rot[i];
    a.tri = h->tri;
    a.t = h->t;
    a.u = h->u;
    a.v = h->v;
    a.flags = h->flags;
    a.counters = reinterpret_cast<unsigned long long *>(counters);
    long long tiles = (long long)((gd.nx + 7) / 8) * ((gd.ny + 7) / 8);
    long long threads = tiles * 64;
    int blocks = (int)((threads + 255) / 256);
    {
        ProfScope ps(kProfTrace, st);
        const bool shadow = (gd.options & SBR_RAYS_SHADOW) != 0;
        if (counters && shadow)
            hipLaunchKernelGGL((k_trace<true, true>), dim3(blocks), dim3(256), 0, st, a);
        else if (counters)
            hipLaunchKernelGGL((k_trace<true, false>), dim3(blocks), dim3(256), 0, st, a);
        else if (shadow)
            hipLaunchKernelGGL((k_trace<false, true>), dim3(blocks), dim3(256), 0, st, a);
        else
            hipLaunchKernelGGL((k_trace<false, false>), dim3(blocks), dim3(256), 0, st, a);
    }
    SBR_LAUNCHED();
    return SBR_OK;
}

}  // namespace sbr
