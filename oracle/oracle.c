/*
 * FP64 CPU oracle -- TEST INFRASTRUCTURE ONLY (see oracle.h).
 *
 * Plain C99 + OpenMP.  Each function states the passage of the paper it
 * follows, and where the paper is silent, the reading taken:
 *   rays          Sec. 3.2.1, Eq. (3): the Monte Carlo estimator, taken as a
 *                 deterministic tangent-plane grid with solid-angle weights
 *   closest hit   Sec. 3.2.1 (ray tracing prose): brute force over triangles
 *   reflection    Sec. 3.2.1, Eq. (1): the recursive S_r term, specular law
 *   Fresnel       Sec. 3.2.2, Eqs. (9)-(10), with eta read as the relative
 *                 refractive index sqrt(eps_c) and Snell as
 *                 sin(dt) = sin(di) / sqrt(eps_c)
 *   amplitude     Sec. 3.2.1, Eq. (1) factors, one return per bounce
 *   IF signal     Sec. 3.2.2, Eq. (8)
 *   IF adjoint    Sec. 3.2.2, Eqs. (11)-(12)
 *   radar cube    Sec. 3.4.2, Eq. (16): T as range/Doppler/angle DFTs
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

static const double C0 = 299792458.0;          /* speed of light, m/s */
static const double EPS0 = 8.8541878128e-12;   /* vacuum permittivity, F/m */
static const double TWO_PI = 6.283185307179586476925286766559;

/* ---------- small vector helpers (double) ---------- */
static double dot3(const double a[3], const double b[3]) {
    return a[0] * b[0] + a[1] * b[1] + a[2] * b[2];
}
static void sub3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[0] - b[0]; o[1] = a[1] - b[1]; o[2] = a[2] - b[2];
}
static void cross3(const double a[3], const double b[3], double o[3]) {
    o[0] = a[1] * b[2] - a[2] * b[1];
    o[1] = a[2] * b[0] - a[0] * b[2];
    o[2] = a[0] * b[1] - a[1] * b[0];
}
static double norm3(const double a[3]) { return sqrt(dot3(a, a)); }
static double dist3(const double a[3], const double b[3]) {
    double d[3]; sub3(a, b, d); return norm3(d);
}
static void vert(const orc_mesh *m, int vi, double o[3]) {
    o[0] = m->verts[3 * vi]; o[1] = m->verts[3 * vi + 1]; o[2] = m->verts[3 * vi + 2];
}
static void tri_verts(const orc_mesh *m, int f, double a[3], double b[3], double c[3]) {
    vert(m, m->faces[3 * f], a); vert(m, m->faces[3 * f + 1], b); vert(m, m->faces[3 * f + 2], c);
}
/* radar frame -> world frame, for a point */
static void to_world(const orc_radar *rd, const double p[3], double o[3]) {
    for (int i = 0; i < 3; i++)
        o[i] = rd->origin[i] + rd->rot[3 * i] * p[0] + rd->rot[3 * i + 1] * p[1] + rd->rot[3 * i + 2] * p[2];
}

/* ---------- Philox-4x32-10 (Salmon, Moraes, Dror, Shaw, SC 2011) ----------
 * Counter-based generator: ten rounds of two 32x32->64 multiplications with
 * the published constants, the key bumped by the Weyl constants each round. */
void orc_philox4x32_10(const unsigned int ctr[4], const unsigned int key[2], unsigned int out[4]) {
    unsigned int x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3], k0 = key[0], k1 = key[1];
    for (int r = 0; r < 10; r++) {
        unsigned long long p0 = 0xD2511F53ull * x0, p1 = 0xCD9E8D57ull * x2;
        unsigned int n0 = (unsigned int)(p1 >> 32) ^ x1 ^ k0, n1 = (unsigned int)p1;
        unsigned int n2 = (unsigned int)(p0 >> 32) ^ x3 ^ k1, n3 = (unsigned int)p0;
        x0 = n0; x1 = n1; x2 = n2; x3 = n3;
        k0 += 0x9E3779B9u; k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* ---------- ray launch (Eq. 3 / Eq. 4 estimator on the tangent grid) ----------
 * Without jitter the sample of cell (ix, iy) is its centre.  With jitter it is
 * uniform in the cell (stratified Monte Carlo, Eq. 4): offsets u1 - 1/2 and
 * u2 - 1/2 of the cell size from Philox-4x32-10 with counter (r, 0, 0, 0) and
 * key (seed_lo, seed_hi), u = (word >> 8) / 2^24 for the first two words. */
void orc_ray(const orc_radar *rd, const orc_grid *g, int r, double o[3], double d[3], double *domega) {
    int ix = r % g->nx, iy = r / g->nx;
    double jx = 0.5, jy = 0.5;
    if (g->jitter) {
        unsigned int ctr[4] = {(unsigned int)r, 0u, 0u, 0u}, key[2] = {g->seed_lo, g->seed_hi}, w[4];
        orc_philox4x32_10(ctr, key, w);
        jx = (double)(w[0] >> 8) / 16777216.0;
        jy = (double)(w[1] >> 8) / 16777216.0;
    }
    double u = g->tan_hx * (2.0 * (ix + jx) / g->nx - 1.0);
    double v = g->tan_hy * (2.0 * (iy + jy) / g->ny - 1.0);
    double q = 1.0 + u * u + v * v;
    double s = 1.0 / sqrt(q);
    double dr[3] = {u * s, v * s, s};
    for (int i = 0; i < 3; i++) {
        o[i] = rd->origin[i];
        d[i] = rd->rot[3 * i] * dr[0] + rd->rot[3 * i + 1] * dr[1] + rd->rot[3 * i + 2] * dr[2];
    }
    /* solid angle of one grid cell at its sample: (cell area on the z=1 plane) * cos / dist^2 */
    if (domega) *domega = (2.0 * g->tan_hx / g->nx) * (2.0 * g->tan_hy / g->ny) / (q * sqrt(q));
}

/* ---------- Moller-Trumbore, two-sided, inclusive edges (FP64) ---------- */
static int mt_hit(const double o[3], const double d[3], const double a[3], const double b[3],
                  const double c[3], double *t, double *bu, double *bv) {
    double e1[3], e2[3], nrm[3], p[3], s[3], q[3];
    sub3(b, a, e1); sub3(c, a, e2);
    cross3(e1, e2, nrm);
    if (nrm[0] == 0.0 && nrm[1] == 0.0 && nrm[2] == 0.0) return 0;  /* degenerate */
    cross3(d, e2, p);
    double det = dot3(e1, p);
    if (det == 0.0) return 0;  /* ray parallel to the plane */
    double inv = 1.0 / det;
    sub3(o, a, s);
    double u = dot3(s, p) * inv;
    if (u < 0.0 || u > 1.0) return 0;
    cross3(s, e1, q);
    double v = dot3(d, q) * inv;
    if (v < 0.0 || u + v > 1.0) return 0;
    *t = dot3(e2, q) * inv;
    *bu = u; *bv = v;
    return 1;
}

/* distance from x to the line through a and b */
static double line_dist(const double x[3], const double a[3], const double b[3]) {
    double ab[3], ax[3], cr[3];
    sub3(b, a, ab); sub3(x, a, ax); cross3(ax, ab, cr);
    return norm3(cr) / norm3(ab);
}

/* distance from x to the segment [a, b] */
static double seg_dist(const double x[3], const double a[3], const double b[3]) {
    double ab[3], ax[3];
    sub3(b, a, ab); sub3(x, a, ax);
    double s = dot3(ax, ab) / dot3(ab, ab);
    if (s < 0.0) s = 0.0;
    if (s > 1.0) s = 1.0;
    double y[3] = {a[0] + s * ab[0], a[1] + s * ab[1], a[2] + s * ab[2]};
    return dist3(x, y);
}

/* Occlusion of the segment from x (on face `self`) to the array centre O.
 * Sets *edge when the decision is within delta of changing. */
static int occluded(const orc_mesh *m, const double x[3], const double O[3], int self, double t_min,
                    double delta, int *edge) {
    double s[3];
    sub3(O, x, s);
    double D = norm3(s);
    for (int j = 0; j < 3; j++) s[j] /= D;
    int occ = 0;
    *edge = 0;
    for (int f = 0; f < m->nf; f++) {
        if (f == self) continue;
        double a[3], b[3], c[3], th, uh, vh;
        tri_verts(m, f, a, b, c);
        if (mt_hit(x, s, a, b, c, &th, &uh, &vh) && th > t_min && th < D - t_min) occ = 1;
        /* borderline: the line meets the plane near the triangle's boundary,
         * or a hit sits near the ends of the accepted interval */
        double e1[3], e2[3], N[3], av[3];
        sub3(b, a, e1); sub3(c, a, e2); cross3(e1, e2, N);
        double den = dot3(N, s);
        if (den == 0.0) continue;
        sub3(a, x, av);
        double tp = dot3(N, av) / den;
        if (tp < t_min - delta || tp > D - t_min + delta) continue;
        double y[3] = {x[0] + tp * s[0], x[1] + tp * s[1], x[2] + tp * s[2]};
        double de = seg_dist(y, a, b), d2 = seg_dist(y, b, c);
        if (d2 < de) de = d2;
        d2 = seg_dist(y, c, a);
        if (d2 < de) de = d2;
        int inside = mt_hit(x, s, a, b, c, &th, &uh, &vh);
        if (de < delta) *edge = 1;
        if (inside && (fabs(tp - t_min) < delta || fabs(tp - (D - t_min)) < delta)) *edge = 1;
    }
    return occ;
}

long long orc_trace(const orc_mesh *m, const orc_radar *rd, const orc_grid *g, const int *rays, int n,
                    int *tri, double *t_out, double *b1_out, double *b2_out, unsigned char *flags,
                    unsigned char *shadow_edge, double *cos_out) {
    const int K = g->max_bounces;
    long long queries = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : queries)
    for (int i = 0; i < n; i++) {
        int r = rays ? rays[i] : i;
        double o[3], d[3], dw;
        orc_ray(rd, g, r, o, d, &dw);
        int prev = -1;
        unsigned char anc = 0;
        double Lpath = 0.0;
        int alive = 1;
        for (int k = 0; k < K; k++) {
            size_t slot = (size_t)k * n + i;
            tri[slot] = -1;
            if (t_out) t_out[slot] = 0.0;
            if (b1_out) b1_out[slot] = 0.0;
            if (b2_out) b2_out[slot] = 0.0;
            if (flags) flags[slot] = 0;
            if (shadow_edge) shadow_edge[slot] = 0;
            if (cos_out) cos_out[slot] = 0.0;
            if (!alive) continue;
            queries++;
            /* closest hit = lexicographic minimum of (t, triangle id) */
            int best = -1;
            double bt = INFINITY, bu = 0.0, bv = 0.0, second = INFINITY;
            for (int f = 0; f < m->nf; f++) {
                if (f == prev) continue;
                double a[3], b[3], c[3], th, uh, vh;
                tri_verts(m, f, a, b, c);
                if (!mt_hit(o, d, a, b, c, &th, &uh, &vh)) continue;
                if (!(th > g->t_min)) continue;
                if (th < bt || (th == bt && f < best)) {
                    second = bt;
                    bt = th; best = f; bu = uh; bv = vh;
                } else if (th < second) {
                    second = th;
                }
            }
            if (best < 0) { alive = 0; continue; }
            double a[3], b[3], c[3], x[3], e1[3], e2[3], nn[3];
            tri_verts(m, best, a, b, c);
            for (int j = 0; j < 3; j++) x[j] = o[j] + bt * d[j];
            sub3(b, a, e1); sub3(c, a, e2); cross3(e1, e2, nn);
            double nl = norm3(nn);
            for (int j = 0; j < 3; j++) nn[j] /= nl;
            double dn = dot3(d, nn);
            Lpath += bt;
            double delta = 1e-6 * (Lpath > 1.0 ? Lpath : 1.0);
            unsigned char fl = anc ? ORC_F_PARENT : 0;
            double de = line_dist(x, a, b);
            double t2 = line_dist(x, b, c); if (t2 < de) de = t2;
            t2 = line_dist(x, c, a); if (t2 < de) de = t2;
            if (de < delta) fl |= ORC_F_EDGE;
            if (second - bt < delta) fl |= ORC_F_TIE;
            if (fabs(dn) < 1e-6) fl |= ORC_F_GRAZE;
            if (bt < 2.0 * g->t_min) fl |= ORC_F_TMIN;
            tri[slot] = best;
            if (t_out) t_out[slot] = bt;
            if (b1_out) b1_out[slot] = bu;
            if (b2_out) b2_out[slot] = bv;
            if (cos_out) cos_out[slot] = fabs(dn);
            anc |= fl;
            if (g->shadow && k > 0) {
                int edge;
                double lr = Lpath + dist3(x, rd->origin);
                if (occluded(m, x, rd->origin, best, g->t_min, 1e-6 * (lr > 1.0 ? lr : 1.0), &edge))
                    fl |= ORC_F_OCCLUDED;
                if (shadow_edge) shadow_edge[slot] = (unsigned char)edge;
            }
            if (flags) flags[slot] = fl;
            /* specular reflection, continue from the hit point */
            for (int j = 0; j < 3; j++) { o[j] = x[j]; d[j] = d[j] - 2.0 * dn * nn[j]; }
            prev = best;
        }
    }
    return queries;
}

/* ---------- Eqs. (9)-(10): Fresnel reflection coefficient ---------- */
typedef struct { double re, im; } cplx;
static cplx cmk(double re, double im) { cplx z = {re, im}; return z; }
static cplx cadd(cplx a, cplx b) { return cmk(a.re + b.re, a.im + b.im); }
static cplx csub(cplx a, cplx b) { return cmk(a.re - b.re, a.im - b.im); }
static cplx cmul(cplx a, cplx b) { return cmk(a.re * b.re - a.im * b.im, a.re * b.im + a.im * b.re); }
static cplx cdiv(cplx a, cplx b) {
    double den = b.re * b.re + b.im * b.im;
    return cmk((a.re * b.re + a.im * b.im) / den, (a.im * b.re - a.re * b.im) / den);
}
/* principal square root */
static cplx csqrt_p(cplx z) {
    double r = hypot(z.re, z.im);
    double a = sqrt(0.5 * (r + fabs(z.re)));
    if (a == 0.0) return cmk(0.0, 0.0);
    double b = 0.5 * z.im / a;
    if (z.re >= 0.0) return cmk(a, b);
    return cmk(fabs(b), z.im >= 0.0 ? a : -a);
}

void orc_fresnel(const orc_mesh *m, int mi, double fc, double cos_i, double out[2]) {
    /* a material index outside the table means a perfect conductor */
    int mode = (mi >= 0 && mi < m->n_mats) ? m->mat_mode[mi] : 0;
    if (mode == 0) { out[0] = -1.0; out[1] = 0.0; return; }
    double er = m->mat_eps_r[mi], sg = m->mat_sigma[mi];
    /* complex relative permittivity eps_c = eps_r - j sigma / (omega eps_0) */
    cplx eps = cmk(er, -sg / (TWO_PI * fc * EPS0));
    cplx nidx = csqrt_p(eps);                                      /* eta read as sqrt(eps_c) */
    double sin2_i = 1.0 - cos_i * cos_i;
    cplx sin2_t = cdiv(cmk(sin2_i, 0.0), eps);                      /* Snell: sin dt = sin di / n */
    cplx cos_t = csqrt_p(csub(cmk(1.0, 0.0), sin2_t));
    cplx ci = cmk(cos_i, 0.0);
    cplx r;
    if (mode == 1) {  /* r_s, perpendicular polarization */
        cplx nct = cmul(nidx, cos_t);
        r = cdiv(csub(ci, nct), cadd(ci, nct));
    } else {          /* r_p, parallel polarization */
        cplx nci = cmul(nidx, ci);
        r = cdiv(csub(nci, cos_t), cadd(nci, cos_t));
    }
    out[0] = r.re; out[1] = r.im;
}

/* ---------- per-path time of flight (I^t) and strength (I^s) ---------- */
/* ---------- Eqs. (6)-(7): a transform T that attaches each sample to its first hit ----------
 * Solid angle per unit of barycentric area at the point x of a triangle with
 * (unnormalised) normal N seen from o:  |N . (x - o)| / |x - o|^3. */
static double attach_density(const double N[3], const double x[3], const double o[3]) {
    double q[3];
    sub3(x, o, q);
    double r = norm3(q);
    return fabs(dot3(N, q)) / (r * r * r);
}

void orc_attach(const orc_mesh *m, const orc_radar *rd, const orc_grid *g, const int *rays, int n,
                const int *tri, double *attach) {
    for (int i = 0; i < n; i++) {
        int r = rays ? rays[i] : i;
        double *out = attach + 3 * (size_t)i;
        int f = tri[i];
        if (f < 0) { out[0] = out[1] = out[2] = 0.0; continue; }
        double o[3], d[3], dw, a[3], b[3], c[3], e1[3], e2[3], N[3], av[3], x[3], w[3], cx[3];
        orc_ray(rd, g, r, o, d, &dw);
        tri_verts(m, f, a, b, c);
        sub3(b, a, e1); sub3(c, a, e2); cross3(e1, e2, N);
        sub3(a, o, av);
        double th = dot3(N, av) / dot3(N, d);
        for (int j = 0; j < 3; j++) x[j] = o[j] + th * d[j];
        /* barycentrics of x: x - a = b1 e1 + b2 e2 */
        double nn = dot3(N, N);
        sub3(x, a, w);
        cross3(w, e2, cx);
        out[0] = dot3(cx, N) / nn;
        cross3(e1, w, cx);
        out[1] = dot3(cx, N) / nn;
        out[2] = attach_density(N, x, o);
    }
}

int orc_paths(const orc_mesh *m, const orc_radar *rd, const orc_grid *g, const orc_chirp *ch,
              const int *rays, int n, const int *tri, const unsigned char *flags, int options,
              const double *attach, int *path_ray, int *path_k, double *amp, double *tau,
              double *taudot, double *weight) {
    const int K = g->max_bounces;
    const int V = rd->n_tx * rd->n_rx;
    double txw[ORC_MAXTX][3], rxw[ORC_MAXRX][3];
    for (int t = 0; t < rd->n_tx; t++) to_world(rd, rd->tx[t], txw[t]);
    for (int q = 0; q < rd->n_rx; q++) to_world(rd, rd->rx[q], rxw[q]);
    int P = 0;
    /* sequential over rays so the path order is fixed: ray-major, then bounce */
    for (int i = 0; i < n; i++) {
        int r = rays ? rays[i] : i;
        double o[3], d[3], dw;
        orc_ray(rd, g, r, o, d, &dw);
        double O[3] = {o[0], o[1], o[2]};
        const double *att = NULL;
        double xa[3] = {0, 0, 0};
        if (attach && tri[i] >= 0) {
            /* the sample follows its first hit: fixed barycentrics on the
             * (moved) triangle, the direction through that point, and the
             * cell's solid angle scaled by |det J_T| = density / density_0 */
            att = attach + 3 * (size_t)i;
            double a[3], b[3], c[3];
            tri_verts(m, tri[i], a, b, c);
            for (int j = 0; j < 3; j++) xa[j] = a[j] + att[0] * (b[j] - a[j]) + att[1] * (c[j] - a[j]);
            double q[3], e1[3], e2[3], N[3];
            sub3(xa, O, q);
            double rq = norm3(q);
            for (int j = 0; j < 3; j++) d[j] = q[j] / rq;
            sub3(b, a, e1); sub3(c, a, e2); cross3(e1, e2, N);
            dw *= attach_density(N, xa, O) / att[2];
        }
        /* Doppler of the path: rate of change of the round trip for a rigidly
         * moving scene, 2 (u . d_1) / c */
        double tdot = 2.0 * dot3(rd->vel, d) / C0;
        double d0[3] = {d[0], d[1], d[2]};
        double x1[3] = {0, 0, 0}, xprev[3] = {O[0], O[1], O[2]};
        double Lk = 0.0, Lmid = 0.0;
        double pr_re = 1.0, pr_im = 0.0;   /* product of reflection coefficients */
        for (int k = 0; k < K; k++) {
            size_t slot = (size_t)k * n + i;
            int f = tri[slot];
            if (f < 0) break;
            double a[3], b[3], c[3], e1[3], e2[3], N[3], av[3], x[3];
            tri_verts(m, f, a, b, c);
            sub3(b, a, e1); sub3(c, a, e2); cross3(e1, e2, N);
            /* plane intersection along the current ray */
            sub3(a, o, av);
            double th = dot3(N, av) / dot3(N, d);
            for (int j = 0; j < 3; j++) x[j] = (k == 0 && att) ? xa[j] : o[j] + th * d[j];
            double nl = norm3(N), nh[3] = {N[0] / nl, N[1] / nl, N[2] / nl};
            double dn = dot3(d, nh);
            double cos_i = fabs(dn);
            double rc[2];
            orc_fresnel(m, m->mat_id ? m->mat_id[f] : 0, ch->fc, cos_i, rc);
            double nre = pr_re * rc[0] - pr_im * rc[1];
            double nim = pr_re * rc[1] + pr_im * rc[0];
            pr_re = nre; pr_im = nim;
            double seg = dist3(x, xprev);
            Lk += seg;
            if (k == 0) { x1[0] = x[0]; x1[1] = x[1]; x1[2] = x[2]; }
            else Lmid += seg;
            double Rk = dist3(x, O);
            int keep = 1;
            if (flags && (flags[slot] & ORC_F_OCCLUDED)) keep = 0;
            if ((options & ORC_DROP_FLAGGED) && flags && (flags[slot] & ~ORC_F_OCCLUDED)) keep = 0;
            if ((options & ORC_EXIT_ONLY) && k + 1 < K && tri[slot + n] >= 0) keep = 0;
            if (keep) {
                /* I^s = d_omega * prod r_j * cos(theta_k) / (L_k R_k), times the
                 * medium's attenuation exp(-a (L_k + R_k)) */
                double s = dw * cos_i / (Lk * Rk) * exp(-rd->atten * (Lk + Rk));
                if (rd->n_tx_gain != 0.0 || rd->n_rx_gain != 0.0) {
                    /* F G of Eq. 1: cos^n to boresight (third column of rot) */
                    double zb[3] = {rd->rot[2], rd->rot[5], rd->rot[8]}, q[3];
                    sub3(x, O, q);
                    double ct = dot3(d0, zb), cr = dot3(q, zb) / norm3(q);
                    s *= pow(ct > 0.0 ? ct : 0.0, rd->n_tx_gain) * pow(cr > 0.0 ? cr : 0.0, rd->n_rx_gain);
                }
                amp[2 * P] = pr_re * s;
                amp[2 * P + 1] = pr_im * s;
                /* I^t per virtual antenna: TX -> x_1 -> ... -> x_k -> RX */
                for (int t = 0; t < rd->n_tx; t++)
                    for (int q = 0; q < rd->n_rx; q++) {
                        double len = dist3(x1, txw[t]) + Lmid + dist3(rxw[q], x);
                        tau[(size_t)P * V + t * rd->n_rx + q] = len / C0;
                    }
                taudot[P] = tdot;
                if (weight) weight[P] = dw;
                path_ray[P] = i;
                path_k[P] = k + 1;
                P++;
            }
            for (int j = 0; j < 3; j++) {
                o[j] = x[j]; xprev[j] = x[j];
                d[j] = d[j] - 2.0 * dn * nh[j];
            }
        }
    }
    return P;
}

/* ---------- Eq. (8), IF signal by direct summation ---------- */
void orc_synth(int P, const double *amp, const double *tau, const double *taudot, int V,
               const orc_chirp *ch, const int *rows, int n_rows, double *out) {
    const int C = ch->n_chirps, S = ch->n_samples;
    if (!rows) n_rows = V * C;
#pragma omp parallel for collapse(2) schedule(static)
    for (int ri = 0; ri < n_rows; ri++) {
        for (int s = 0; s < S; s++) {
            int row = rows ? rows[ri] : ri;
            int v = row / C, c = row % C;
            double ts = s / ch->fs;                       /* sample time from the ramp start */
            double re = 0.0, im = 0.0;
            for (int p = 0; p < P; p++) {
                double tp = tau[(size_t)p * V + v] + c * ch->t_chirp * taudot[p];
                double ph = TWO_PI * (ch->slope * ts * tp + ch->fc * tp);
                double cs = cos(ph), sn = sin(ph);
                re += amp[2 * p] * cs - amp[2 * p + 1] * sn;
                im += amp[2 * p] * sn + amp[2 * p + 1] * cs;
            }
            out[((size_t)ri * S + s) * 2] = re;
            out[((size_t)ri * S + s) * 2 + 1] = im;
        }
    }
}

/* ---------- Eqs. (11)-(12), adjoint of Eq. (8) ----------
 * With G = dL/dRe S + i dL/dIm S and any real parameter q of the path,
 * dL/dq = Re(conj(G) dS/dq).  dS/dI^t = 2 pi j (mu t + fc) I^s e^{j phi}
 * (Eq. 11) and dS/dI^s = e^{j phi} (Eq. 12). */
void orc_synth_adjoint(int P, const double *amp, const double *tau, const double *taudot, int V,
                       const orc_chirp *ch, const double *G, double *amp_bar, double *tau_bar,
                       double *taudot_bar) {
    const int C = ch->n_chirps, S = ch->n_samples;
#pragma omp parallel for schedule(dynamic, 4)
    for (int p = 0; p < P; p++) {
        double ab_re = 0.0, ab_im = 0.0, tdb = 0.0;
        for (int v = 0; v < V; v++) {
            double tb = 0.0;
            for (int c = 0; c < C; c++) {
                double tp = tau[(size_t)p * V + v] + c * ch->t_chirp * taudot[p];
                for (int s = 0; s < S; s++) {
                    double ts = s / ch->fs;
                    double ph = TWO_PI * (ch->slope * ts * tp + ch->fc * tp);
                    double e_re = cos(ph), e_im = sin(ph);
                    double g_re = G[(((size_t)v * C + c) * S + s) * 2];
                    double g_im = G[(((size_t)v * C + c) * S + s) * 2 + 1];
                    /* Eq. (12): dS/dA = e^{j phi}; dL/dRe A = Re(conj G e), dL/dIm A = Re(conj G j e) */
                    ab_re += g_re * e_re + g_im * e_im;
                    ab_im += g_re * (-e_im) + g_im * e_re;
                    /* Eq. (11): dS/dtau = 2 pi j (mu t + fc) A e^{j phi} */
                    double w = TWO_PI * (ch->slope * ts + ch->fc);
                    double ae_re = amp[2 * p] * e_re - amp[2 * p + 1] * e_im;
                    double ae_im = amp[2 * p] * e_im + amp[2 * p + 1] * e_re;
                    double ds_re = -w * ae_im, ds_im = w * ae_re;
                    double dq = g_re * ds_re + g_im * ds_im;
                    tb += dq;
                    tdb += dq * c * ch->t_chirp;
                }
            }
            tau_bar[(size_t)p * V + v] = tb;
        }
        amp_bar[2 * p] = ab_re;
        amp_bar[2 * p + 1] = ab_im;
        if (taudot_bar) taudot_bar[p] = tdb;
    }
}

/* ---------- Eq. (16) T = range, Doppler, angle DFTs (naive) ---------- */
static double window_val(int window, int i, int N) {
    if (window == 1 && N > 1) return 0.5 - 0.5 * cos(TWO_PI * i / (N - 1));
    return 1.0;
}
/* exp(sign * 2 pi j * (k mod N) / N) */
static void twiddle(long long k, int N, int sign, double *re, double *im) {
    long long q = k % N;
    double a = TWO_PI * (double)q / (double)N;
    *re = cos(a); *im = sign * sin(a);
}

void orc_radar_cube(const double *in, int V, int C, int S, int Na, int window, int dir, double *out) {
    orc_radar_cube2(in, V, 1, C, S, Na, 1, window, dir, out);
}

void orc_radar_cube2(const double *in, int Vx, int Vy, int C, int S, int Nax, int Nay, int window, int dir,
                     double *out) {
    const int V = Vx * Vy, Na = Nax * Nay;
    size_t plane = (size_t)C * S;
    if (dir == 0) {
        double *y1 = (double *)calloc((size_t)V * plane * 2, sizeof(double));
        double *y2 = (double *)calloc((size_t)V * plane * 2, sizeof(double));
        /* range: over s */
#pragma omp parallel for collapse(2)
        for (int vc = 0; vc < V * C; vc++)
            for (int r = 0; r < S; r++) {
                double re = 0.0, im = 0.0;
                for (int s = 0; s < S; s++) {
                    double w = window_val(window, s, S), tr, ti;
                    twiddle((long long)r * s, S, -1, &tr, &ti);
                    double xr = w * in[((size_t)vc * S + s) * 2], xi = w * in[((size_t)vc * S + s) * 2 + 1];
                    re += xr * tr - xi * ti; im += xr * ti + xi * tr;
                }
                y1[((size_t)vc * S + r) * 2] = re; y1[((size_t)vc * S + r) * 2 + 1] = im;
            }
        /* Doppler: over c */
#pragma omp parallel for collapse(3)
        for (int v = 0; v < V; v++)
            for (int dd = 0; dd < C; dd++)
                for (int r = 0; r < S; r++) {
                    double re = 0.0, im = 0.0;
                    for (int c = 0; c < C; c++) {
                        double w = window_val(window, c, C), tr, ti;
                        twiddle((long long)dd * c, C, -1, &tr, &ti);
                        size_t ix = ((size_t)v * plane + (size_t)c * S + r) * 2;
                        double xr = w * y1[ix], xi = w * y1[ix + 1];
                        re += xr * tr - xi * ti; im += xr * ti + xi * tr;
                    }
                    size_t ox = ((size_t)v * plane + (size_t)dd * S + r) * 2;
                    y2[ox] = re; y2[ox + 1] = im;
                }
        /* angle: over the array grid (vy, vx), zero-padded to (Nay, Nax);
         * v = vy Vx + vx in, a = ay Nax + ax out */
#pragma omp parallel for collapse(2)
        for (int a = 0; a < Na; a++)
            for (size_t e = 0; e < plane; e++) {
                int ax = a % Nax, ay = a / Nax;
                double re = 0.0, im = 0.0;
                for (int v = 0; v < V; v++) {
                    int vx = v % Vx, vy = v / Vx;
                    double tr, ti, ur, ui;
                    twiddle((long long)ax * vx, Nax, -1, &tr, &ti);
                    twiddle((long long)ay * vy, Nay, -1, &ur, &ui);
                    double wr = tr * ur - ti * ui, wi = tr * ui + ti * ur;
                    size_t ix = ((size_t)v * plane + e) * 2;
                    re += y2[ix] * wr - y2[ix + 1] * wi; im += y2[ix] * wi + y2[ix + 1] * wr;
                }
                out[((size_t)a * plane + e) * 2] = re; out[((size_t)a * plane + e) * 2 + 1] = im;
            }
        free(y1); free(y2);
    } else {
        double *z2 = (double *)calloc((size_t)V * plane * 2, sizeof(double));
        double *z1 = (double *)calloc((size_t)V * plane * 2, sizeof(double));
        /* angle adjoint: only the V populated inputs receive gradient */
#pragma omp parallel for collapse(2)
        for (int v = 0; v < V; v++)
            for (size_t e = 0; e < plane; e++) {
                int vx = v % Vx, vy = v / Vx;
                double re = 0.0, im = 0.0;
                for (int a = 0; a < Na; a++) {
                    int ax = a % Nax, ay = a / Nax;
                    double tr, ti, ur, ui;
                    twiddle((long long)ax * vx, Nax, +1, &tr, &ti);
                    twiddle((long long)ay * vy, Nay, +1, &ur, &ui);
                    double wr = tr * ur - ti * ui, wi = tr * ui + ti * ur;
                    size_t ix = ((size_t)a * plane + e) * 2;
                    re += in[ix] * wr - in[ix + 1] * wi; im += in[ix] * wi + in[ix + 1] * wr;
                }
                z2[((size_t)v * plane + e) * 2] = re; z2[((size_t)v * plane + e) * 2 + 1] = im;
            }
        /* Doppler adjoint */
#pragma omp parallel for collapse(3)
        for (int v = 0; v < V; v++)
            for (int c = 0; c < C; c++)
                for (int r = 0; r < S; r++) {
                    double re = 0.0, im = 0.0;
                    for (int dd = 0; dd < C; dd++) {
                        double tr, ti;
                        twiddle((long long)dd * c, C, +1, &tr, &ti);
                        size_t ix = ((size_t)v * plane + (size_t)dd * S + r) * 2;
                        re += z2[ix] * tr - z2[ix + 1] * ti; im += z2[ix] * ti + z2[ix + 1] * tr;
                    }
                    double w = window_val(window, c, C);
                    size_t ox = ((size_t)v * plane + (size_t)c * S + r) * 2;
                    z1[ox] = w * re; z1[ox + 1] = w * im;
                }
        /* range adjoint */
#pragma omp parallel for collapse(2)
        for (int vc = 0; vc < V * C; vc++)
            for (int s = 0; s < S; s++) {
                double re = 0.0, im = 0.0;
                for (int r = 0; r < S; r++) {
                    double tr, ti;
                    twiddle((long long)r * s, S, +1, &tr, &ti);
                    size_t ix = ((size_t)vc * S + r) * 2;
                    re += z1[ix] * tr - z1[ix + 1] * ti; im += z1[ix] * ti + z1[ix + 1] * tr;
                }
                double w = window_val(window, s, S);
                out[((size_t)vc * S + s) * 2] = w * re; out[((size_t)vc * S + s) * 2 + 1] = w * im;
            }
        free(z1); free(z2);
    }
}

/* ---------- detections -> 3D points (Sec. 4: radars output point clouds) ----------
 * Range bin r of an S-sample chirp: beat frequency r f_s / S = mu tau, R = c tau / 2.
 * Doppler bin d of C chirps: d / C cycles per chirp = f_c T_c taudot, v = c taudot / 2.
 * Angle bin a of the zero-padded array DFT (sign -1) over lambda/2 spacing:
 * the element phase step is -pi u, so u = -2 a_s / N with a_s the signed bin. */
static double signed_bin(int a, int N) { return (a >= (N + 1) / 2) ? (double)(a - N) : (double)a; }

void orc_cloud(const int *points, int n, const orc_radar *rd, const orc_chirp *ch, int Nax, int Nay,
               double *out) {
    const int S = ch->n_samples, C = ch->n_chirps;
    for (int i = 0; i < n; i++) {
        int rb = points[4 * i], db = points[4 * i + 1], a = points[4 * i + 2];
        double R = C0 * (rb * ch->fs / ((double)S * ch->slope)) / 2.0;
        double ax = a % Nax, ay = a / Nax;
        double ux = -2.0 * signed_bin((int)ax, Nax) / Nax;
        double uy = Nay > 1 ? -2.0 * signed_bin((int)ay, Nay) / Nay : 0.0;
        double uz2 = 1.0 - ux * ux - uy * uy;
        double u[3] = {ux, uy, uz2 > 0.0 ? sqrt(uz2) : 0.0};
        double p[3] = {R * u[0], R * u[1], R * u[2]}, w[3];
        to_world(rd, p, w);
        double tdot = signed_bin(db, C) / ((double)C * ch->fc * ch->t_chirp);
        out[4 * i] = w[0];
        out[4 * i + 1] = w[1];
        out[4 * i + 2] = w[2];
        out[4 * i + 3] = C0 * tdot / 2.0;
    }
}

/* ---------- angle peaks of detected range-Doppler cells ----------
 * A cell's angle spectrum q[a] = |X[a][d][r]|^2 over the (circular) angle grid
 * (ring for a linear array, torus of Nay x Nax for a planar one): a is a peak
 * when q[a] >= rel * max_a q, q[a] > q[n] for every neighbour n with a lower
 * index and q[a] >= q[n] for the others (plateaus give their first cell). */
static double cell_q(const double *cube, size_t plane, size_t e, int a) {
    size_t ix = ((size_t)a * plane + e) * 2;
    return cube[ix] * cube[ix] + cube[ix + 1] * cube[ix + 1];
}

int orc_angle_peaks(const double *cube, int Nax, int Nay, int C, int S, const int *det, int n, double rel,
                    int *out, int max_out) {
    const size_t plane = (size_t)C * S;
    const int Na = Nax * Nay;
    int cnt = 0;
    for (int i = 0; i < n; i++) {
        const int r = det[4 * i], d = det[4 * i + 1];
        const size_t e = (size_t)d * S + r;
        double qmax = 0.0;
        for (int a = 0; a < Na; a++) {
            double q = cell_q(cube, plane, e, a);
            if (q > qmax) qmax = q;
        }
        for (int a = 0; a < Na; a++) {
            const double q = cell_q(cube, plane, e, a);
            if (!(q >= rel * qmax) || q <= 0.0) continue;
            const int ax = a % Nax, ay = a / Nax;
            int peak = 1;
            for (int dy = (Nay > 1 ? -1 : 0); dy <= (Nay > 1 ? 1 : 0) && peak; dy++)
                for (int dx = -1; dx <= 1 && peak; dx++) {
                    if (dx == 0 && dy == 0) continue;
                    const int bx = (ax + dx + Nax) % Nax, by = (ay + dy + Nay) % Nay;
                    const int b = by * Nax + bx;
                    if (b == a) continue;
                    const double qb = cell_q(cube, plane, e, b);
                    if (b < a ? !(q > qb) : !(q >= qb)) peak = 0;
                }
            if (!peak) continue;
            if (cnt < max_out) {
                out[4 * cnt] = r; out[4 * cnt + 1] = d; out[4 * cnt + 2] = a; out[4 * cnt + 3] = 0;
            }
            cnt++;
        }
    }
    return cnt;
}

/* ---------- textbook square-law cell-averaging CFAR ---------- */
int orc_cfar(const double *cube, int Na, int C, int S, int guard, int train, double pfa,
             unsigned char *status, int *argmax, double *power, double *ratio) {
    size_t plane = (size_t)C * S;
    double *pm = (double *)calloc(plane, sizeof(double));
    for (size_t e = 0; e < plane; e++) {
        double acc = 0.0;
        for (int a = 0; a < Na; a++) {
            double re = cube[((size_t)a * plane + e) * 2], im = cube[((size_t)a * plane + e) * 2 + 1];
            acc += re * re + im * im;
        }
        pm[e] = acc;
    }
    int w = guard + train, cnt = 0;
    for (int d = 0; d < C; d++)
        for (int r = 0; r < S; r++) {
            size_t e = (size_t)d * S + r;
            double sum = 0.0;
            int nt = 0;
            for (int dd = -w; dd <= w; dd++)
                for (int rr = -w; rr <= w; rr++) {
                    if (abs(dd) <= guard && abs(rr) <= guard) continue;
                    int r2 = r + rr;
                    if (r2 < 0 || r2 >= S) continue;                  /* range truncated */
                    int d2 = ((d + dd) % C + C) % C;                   /* Doppler circular */
                    sum += pm[(size_t)d2 * S + r2];
                    nt++;
                }
            int am = 0;
            double best = -1.0;
            for (int a = 0; a < Na; a++) {
                size_t ix = ((size_t)a * plane + e) * 2;
                double q = cube[ix] * cube[ix] + cube[ix + 1] * cube[ix + 1];
                if (q > best) { best = q; am = a; }   /* ties: lowest index */
            }
            unsigned char st = 0;
            double rt = 0.0;
            if (nt > 0) {
                double mean = sum / nt;
                double alpha = nt * (pow(pfa, -1.0 / nt) - 1.0);
                double thr = alpha * mean;
                if (pm[e] > thr) { st = 1; cnt++; }
                if (fabs(pm[e] - thr) <= 1e-6 * thr) st |= 2;
                rt = thr > 0.0 ? pm[e] / thr : 0.0;
            }
            if (ratio) ratio[e] = rt;
            if (status) status[e] = st;
            if (argmax) argmax[e] = am;
            if (power) power[e] = pm[e];
        }
    free(pm);
    return cnt;
}
