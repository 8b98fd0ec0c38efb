/*
 * FP64 CPU oracle for the differentiable shooting-and-bouncing-rays (SBR)
 * mmWave radar simulator of "Differentiable Radio Frequency Ray Tracing for
 * Millimeter-Wave Sensing" (DiffSBR, arXiv 2311.13182).
 *
 * TEST INFRASTRUCTURE ONLY.  This library is the slow, plain, obviously
 * correct definition that the HIP path is checked against.  Only the test
 * suite, the smoke check and the CPU-baseline leg of the benchmark may load
 * it.  It shares no code, header, table or helper with the HIP library.
 *
 * Everything is double precision.  Brute-force O(rays x triangles) closest
 * hit, direct per-path summation of the IF signal, naive O(N^2) DFTs.
 *
 * Units: metres, seconds, hertz.  Radar frame: x = array axis, y = up,
 * z = boresight.  Virtual antenna index v = t * n_rx + m.
 *
 * Parity status (what pins each function; the tests under tests/ hold them):
 *   orc_ray            closed-form solid angle of the grid, boresight symmetry;
 *                      jitter: Philox known-answer vectors, unbiased solid angle
 *   orc_trace          independent NumPy brute force, trihedral and plate
 *                      closed forms, energy invariant; shadow test: no
 *                      occlusion inside a convex room, independent NumPy
 *                      segment test with occluders, no inheritance
 *   orc_paths (exit)   exit-only == last record of each ray of the full model
 *   orc_paths          plate normal incidence (tau = 2R/c), trihedral
 *                      point-reflection identity, Fresnel special cases;
 *                      per-antenna legs of k >= 2 paths: the angle DFT of
 *                      a two-plate double bounce peaks at the first hit's
 *                      azimuth for a TX line and at the last hit's for an
 *                      RX line (a TX<->RX leg swap moves both peaks)
 *   orc_attach         summed attached weights vs the closed-form solid angle
 *                      of a triangle (Van Oosterom-Strackee) and its
 *                      derivative; attached estimator == fixed one at theta_0;
 *                      dense re-traced grid (loose)
 *   orc_fresnel        normal incidence, grazing, passivity, conductor limit
 *   orc_synth          single-path geometric sequence and Dirichlet kernel,
 *                      range / Doppler / angle peak bins, 24 GHz ranging
 *                      radar's plate at its 2R mu / c bin
 *   orc_synth_adjoint  central differences of orc_synth
 *   orc_radar_cube     numpy.fft, dot-product (adjoint) identity (1D and 2D
 *                      arrays)
 *   orc_cfar           injected targets, brute force on tiny maps
 *   orc_angle_peaks    independent NumPy local-maximum search, planted peaks
 *   orc_cloud          bins of a synthesised point target map back to its
 *                      position and velocity within one resolution cell
 */
#ifndef SBR_ORACLE_H
#define SBR_ORACLE_H

#ifdef __cplusplus
extern "C" {
#endif

#define ORC_MAXK 8
#define ORC_MAXTX 20
#define ORC_MAXRX 20

typedef struct {
    int nv, nf;
    const double *verts;     /* [nv][3] world frame, metres                    */
    const int *faces;        /* [nf][3] vertex indices                          */
    const int *mat_id;       /* [nf] material index, or NULL: material 0        */
    int n_mats;              /* 0: every face is a perfect electric conductor   */
    const int *mat_mode;     /* [n_mats] 0 conductor (r = -1), 1 TE r_s, 2 TM r_p */
    const double *mat_eps_r; /* [n_mats] relative permittivity                  */
    const double *mat_sigma; /* [n_mats] conductivity, S/m                      */
} orc_mesh;

typedef struct {
    double origin[3];   /* array centre, world frame                          */
    double rot[9];      /* radar -> world rotation, row-major                  */
    int n_tx, n_rx;
    double tx[ORC_MAXTX][3];  /* radar frame                                   */
    double rx[ORC_MAXRX][3];  /* radar frame                                   */
    double vel[3];      /* rigid scene velocity, world frame, m/s              */
    double atten;       /* amplitude attenuation of the medium, 1/m: each path's
                           I^s carries exp(-atten (L_k + R_k)) (Eq. 5's A)      */
    double n_tx_gain, n_rx_gain;  /* directional gains F, G of Eq. 1: cos^n of
                           the angle to boresight of the outgoing ray (F) and of
                           the return from the last hit (G); 0 = isotropic      */
} orc_radar;

typedef struct {
    double fc;          /* carrier, Hz                                         */
    double slope;       /* mu = B / T, Hz/s                                    */
    double fs;          /* ADC rate, Hz                                        */
    double t_chirp;     /* chirp repetition period, s                         */
    int n_samples, n_chirps;
} orc_chirp;

typedef struct {
    int nx, ny;
    double tan_hx, tan_hy;   /* half-width of the tangent-plane grid           */
    int max_bounces;
    double t_min;            /* minimum accepted hit distance, metres          */
    int shadow;              /* 1: test the return segment of every hit after
                                the first for occlusion (any hit strictly
                                between it and the array centre)              */
    int jitter;              /* 1: stratified Monte Carlo sample per cell      */
    unsigned int seed_lo, seed_hi;   /* Philox key of the jitter              */
} orc_grid;

/* hit flags, one byte per (bounce, ray) */
#define ORC_F_EDGE     1   /* hit point within delta_k of an edge line          */
#define ORC_F_TIE      2   /* second-closest candidate within delta_k            */
#define ORC_F_GRAZE    4   /* |d . n| < 1e-6                                     */
#define ORC_F_TMIN     8   /* t < 2 t_min                                        */
#define ORC_F_PARENT  16   /* an earlier bounce of the same ray is flagged       */
#define ORC_F_OCCLUDED 32  /* return segment to the array centre is blocked      */

/* orc_paths options */
#define ORC_DROP_FLAGGED 1 /* skip records with any flag other than OCCLUDED     */
#define ORC_EXIT_ONLY    2 /* only the last hit of each ray returns              */

/* Philox-4x32-10 counter-based generator (Salmon et al., SC 2011). */
void orc_philox4x32_10(const unsigned int ctr[4], const unsigned int key[2], unsigned int out[4]);

/* Ray r = iy * nx + ix of the grid: origin, unit direction, solid-angle weight
 * (cell centre, or with g->jitter a Philox-drawn point of the cell). */
void orc_ray(const orc_radar *rd, const orc_grid *g, int r,
             double o[3], double d[3], double *domega);

/* Brute-force closest hit for every bounce of the listed rays.
 * rays: [n] ray indices (NULL = all rays 0..nx*ny-1, then n must be nx*ny).
 * Outputs are [K][n] with K = g->max_bounces: tri (-1 = none), t, barycentric
 * weights of vertices 1 and 2, flags.  Any output pointer may be NULL except tri.
 * With g->shadow the return of every hit after the first (the first one's
 * return retraces its incoming, unobstructed ray) is tested: a hit of another
 * triangle with t in (t_min, D - t_min) along the segment of length D to the
 * array centre sets ORC_F_OCCLUDED (not inherited by later bounces).
 * shadow_edge ([K][n], NULL-able): 1 where that decision is borderline -- some
 * other triangle meets the segment's line within delta_k of its boundary, or
 * a hit lies within delta_k of the segment's ends.
 * cos_i ([K][n], NULL-able): |d . n| of each hit, the cosine of its incidence
 * angle (0 where there is none).
 * Returns the number of closest-hit queries issued (a ray's final miss counts). */
long long orc_trace(const orc_mesh *m, const orc_radar *rd, const orc_grid *g,
                    const int *rays, int n, int *tri, double *t, double *b1,
                    double *b2, unsigned char *flags, unsigned char *shadow_edge,
                    double *cos_i);

/* Reflection coefficient of material `mi` at incidence cosine cos_i (in [0,1]).
 * out[0] = real part, out[1] = imaginary part. */
void orc_fresnel(const orc_mesh *m, int mi, double fc, double cos_i, double out[2]);

/* Path quantities from frozen hit triangle IDs (FP64 plane intersections).
 * One path per (ray, bounce) with a hit, in ray-major then bounce order.
 * Records flagged ORC_F_OCCLUDED never return.  options: ORC_DROP_FLAGGED
 * skips records with any other flag bit; ORC_EXIT_ONLY keeps only the last
 * hit of each ray (classic exit-ray SBR), and none if that one is skipped.
 * Outputs sized for K*n paths: path_ray [P] (index into `rays`), path_k [P]
 * (1-based bounce), amp [P][2], tau [P][V] (seconds), taudot [P] (s/s).
 * Returns P. */
int orc_paths(const orc_mesh *m, const orc_radar *rd, const orc_grid *g,
              const orc_chirp *ch, const int *rays, int n, const int *tri,
              const unsigned char *flags, int options, const double *attach,
              int *path_ray, int *path_k, double *amp, double *tau, double *taudot,
              double *weight);

/* Reparameterisation of Eqs. (6)-(7) that attaches every sample to its first
 * hit.  For each of the n rays whose first hit triangle tri[i] (bounce-0 row
 * of the hit ids) exists: attach[i] = (b1, b2, D0) with x = a + b1 (b - a) +
 * b2 (c - a) the hit point and D0 = |N . (x - o)| / |x - o|^3 the solid angle
 * per unit barycentric area there.  Given to orc_paths (with the geometry
 * moved), the first hit stays at (b1, b2) of its triangle, the ray turns to
 * pass through it, and the cell weight is multiplied by |det J_T| = D / D0;
 * weight (NULL-able, [P]) receives that weight per path.  Misses: zeros. */
void orc_attach(const orc_mesh *m, const orc_radar *rd, const orc_grid *g,
                const int *rays, int n, const int *tri, double *attach);

/* IF signal by direct summation over paths.  rows: [n_rows] indices v*C + c
 * (NULL = every row, n_rows = V*C).  out: [n_rows][S][2]. */
void orc_synth(int P, const double *amp, const double *tau, const double *taudot,
               int V, const orc_chirp *ch, const int *rows, int n_rows, double *out);

/* Adjoint of orc_synth.  G = dL/dRe S + i dL/dIm S, [V][C][S][2].
 * amp_bar [P][2] (dL/dRe A + i dL/dIm A), tau_bar [P][V], taudot_bar [P]. */
void orc_synth_adjoint(int P, const double *amp, const double *tau,
                       const double *taudot, int V, const orc_chirp *ch,
                       const double *G, double *amp_bar, double *tau_bar,
                       double *taudot_bar);

/* Range -> Doppler -> angle DFT cube.  dir 0: in [V][C][S][2] -> out [Na][C][S][2].
 * dir 1 (conjugate transpose): in [Na][C][S][2] -> out [V][C][S][2].
 * window 0 rectangular, 1 symmetric Hann on the range and Doppler axes. */
void orc_radar_cube(const double *in, int V, int C, int S, int Na, int window,
                    int dir, double *out);

/* The same for a planar array whose virtual antennas form a Vy x Vx grid
 * (v = vy * Vx + vx): the angle stage is the 2D DFT over (vy, vx), zero-padded
 * to (Nay, Nax), output angle index a = ay * Nax + ax.  Vy = Nay = 1 is
 * orc_radar_cube. */
void orc_radar_cube2(const double *in, int Vx, int Vy, int C, int S, int Nax, int Nay,
                     int window, int dir, double *out);

/* Cell-averaging CFAR on P[d][r] = sum_a |X[a][d][r]|^2 (X is [Na][C][S][2]).
 * Doppler axis circular, range axis truncated; alpha = N_t (pfa^(-1/N_t) - 1).
 * Per cell of the [C][S] map: status bit 0 = detected (P > alpha * mean),
 * bit 1 = borderline (|P - alpha*mean| <= 1e-6 alpha*mean); argmax over a
 * (lowest index on ties); power P; ratio P / (alpha * mean).  Any output may
 * be NULL.  Returns the number of detections. */
int orc_cfar(const double *cube, int Na, int C, int S, int guard, int train,
             double pfa, unsigned char *status, int *argmax, double *power,
             double *ratio);

/* Angle peaks of detected range-Doppler cells (several scatterers per cell,
 * as a radar's angle search reports them).  cube [Nay*Nax][C][S][2]; det
 * [n][4] (range bin, Doppler bin, ...); rel: a peak holds at least rel of the
 * cell's largest angle power.  Peaks are local maxima over the circular angle
 * grid (ring if Nay = 1, else the 8-neighbourhood on the Nay x Nax torus);
 * equal neighbours keep the lower index.  out [max_out][4] = (range bin,
 * Doppler bin, angle index, 0), detection-major then angle ascending.
 * Returns the number of peaks (may exceed max_out). */
int orc_angle_peaks(const double *cube, int Nax, int Nay, int C, int S, const int *det, int n,
                    double rel, int *out, int max_out);

/* Detections -> points.  points: [n][4] (range bin, Doppler bin, angle index
 * a = ay * Nax + ax, unused) as orc_cfar's cells give them; Nay = 1 for a
 * linear array along the radar x axis (elevation unknown: points in the
 * radar's x-z plane), else a planar lambda/2 grid (vy along y).  out [n][4]:
 * world x, y, z and radial velocity (m/s, positive = receding). */
void orc_cloud(const int *points, int n, const orc_radar *rd, const orc_chirp *ch, int Nax,
               int Nay, double *out);

#ifdef __cplusplus
}
#endif
#endif
