/*
 * libsbr -- differentiable shooting-and-bouncing-rays (SBR) mmWave radar
 * simulator for AMD Instinct MI355X (gfx950).
 *
 * Implements the forward simulation and backpropagation of "Differentiable
 * Radio Frequency Ray Tracing for Millimeter-Wave Sensing" (DiffSBR,
 * arXiv 2311.13182): ray launch, BVH closest-hit tracing with specular
 * multi-bounce (Sec. 3.2.1, Eqs. 1-3), per-path time of flight I^t and
 * strength I^s with Fresnel reflection (Sec. 3.2.2, Eqs. 9-10), the FMCW IF
 * signal (Eq. 8), the signal-to-image map T of the spatial loss (Sec. 3.4.2,
 * Eq. 16), and the adjoint chain from dL/dIF to mesh vertices (Eqs. 11-13).
 *
 * Conventions shared by every entry point
 *   - Units: metres, seconds, hertz (SI).
 *   - Radar frame: x = array axis, y = up, z = boresight.  sbr_radar.rot maps
 *     radar-frame vectors to the world frame (row-major 3x3).
 *   - Ray grid: ray r = iy * nx + ix looks along (u, v, 1)/|(u, v, 1)| with
 *     u = tan_half_x * (2 (ix + 0.5) / nx - 1), v likewise in y; its Monte
 *     Carlo weight (Eq. 3) is the cell solid angle
 *     (2 tan_half_x / nx)(2 tan_half_y / ny) / (1 + u^2 + v^2)^(3/2).
 *     With SBR_RAYS_JITTER in sbr_rays.options the offset 0.5 becomes a
 *     per-ray uniform draw from Philox-4x32-10 (key seed_lo, seed_hi); the
 *     weight stays the cell's, evaluated at the drawn (u, v).
 *   - Virtual antenna v = t * n_rx + m (TX t, RX m).
 *   - Complex arrays are interleaved float pairs (re, im), C-contiguous.
 *   - Memory: every pointer inside the structs below and every array argument
 *     is DEVICE memory owned by the caller, except the structs themselves and
 *     the sbr_material table, which are host memory read during the call.
 *     The library never allocates or frees; size queries say how much scratch
 *     to pass.  Scratch content is not preserved between calls.
 *   - Streams: `stream` is a hipStream_t (NULL = default stream).  Every call
 *     only enqueues work on it and returns; results are ready when the stream
 *     is.  Calls on one stream run in order.
 *   - Errors: 0 on success, a negative sbr_status otherwise; no C++ exception
 *     crosses the ABI.  sbr_last_error() gives the calling thread's message.
 *     Argument checks happen before anything is enqueued.
 */
#ifndef SBR_H
#define SBR_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    SBR_OK = 0,
    SBR_E_ARG = -1,          /* null pointer, bad size, bounds exceeded          */
    SBR_E_HIP = -2,          /* HIP launch or API failure (message has the text) */
    SBR_E_SCRATCH = -3,      /* scratch or BVH buffer too small (message: bytes) */
    SBR_E_UNSUPPORTED = -4
} sbr_status;

#define SBR_MAX_BOUNCES 8
#define SBR_MAX_TX 20
#define SBR_MAX_RX 20
#define SBR_MAX_VIRTUAL 400
#define SBR_MAX_MATERIALS 64

/* Triangle mesh (Sec. 3.1: surface mesh representation).  Device arrays. */
typedef struct {
    const float *verts;      /* [nv][3] world frame, metres                      */
    int32_t nv;
    const int32_t *faces;    /* [nf][3] vertex indices, each in [0, nv)           */
    int32_t nf;
    const uint16_t *mat_id;  /* [nf] material table index (>= n_mats: conductor), or NULL */
} sbr_mesh;

/* Reflection model of one material (Sec. 3.2.2, Eqs. 9-10).  mode 0: perfect
 * conductor, r = -1; mode 1: r_s (TE); mode 2: r_p (TM), with complex
 * relative permittivity eps_c = eps_r - j sigma / (2 pi fc eps_0), refractive
 * index n = sqrt(eps_c) and Snell's law sin(dt) = sin(di) / n.  Host memory. */
typedef struct {
    int32_t mode;
    int32_t reserved;
    double eps_r;
    double sigma;            /* S/m */
} sbr_material;

/* Radar pose and MIMO array (Sec. 3.2: part of the scene parameters Theta). */
typedef struct {
    double origin[3];        /* array centre, world frame                        */
    double rot[9];           /* radar -> world rotation, row-major               */
    int32_t n_tx, n_rx;      /* n_tx <= 20, n_rx <= 20 (n_tx * n_rx <= 400)      */
    double tx[SBR_MAX_TX][3];/* radar frame                                      */
    double rx[SBR_MAX_RX][3];/* radar frame                                      */
    double velocity[3];      /* rigid scene velocity, world frame, m/s (Doppler) */
    double attenuation;      /* amplitude attenuation of the medium, 1/m (>= 0): each
                                path's I^s carries exp(-attenuation (L_k + R_k)), the
                                attenuation function A of Sec. 3.2.1, Eqs. 4-5      */
    double tx_gain_exp;      /* F of Eq. 1: TX gain cos^n of the outgoing ray's angle
                                to boresight (third column of rot); 0 = isotropic   */
    double rx_gain_exp;      /* G of Eq. 1: RX gain cos^n of the angle to boresight of
                                the direction from the array centre to the last hit */
} sbr_radar;

/* FMCW chirp (Eq. 8: fc, mu = B / T).  Sample s is taken at t = s / fs from
 * the start of the ramp; chirp c starts c * t_chirp after chirp 0. */
typedef struct {
    double fc;               /* carrier, Hz            */
    double slope;            /* mu, Hz/s               */
    double fs;               /* ADC sample rate, Hz    */
    double t_chirp;          /* chirp period, s        */
    int32_t n_samples;       /* S >= 1                 */
    int32_t n_chirps;        /* C >= 1                 */
} sbr_chirp;

/* Ray grid (the samples of Eq. 3) and bounce limit. */
typedef struct {
    int32_t nx, ny;          /* nx * ny <= 2^26                                  */
    double tan_half_x, tan_half_y;
    int32_t max_bounces;     /* K, 1..8                                          */
    int32_t options;         /* SBR_RAYS_* bits (0 = none)                       */
    double t_min;            /* hits closer than this are ignored, metres        */
    uint32_t seed_lo, seed_hi;   /* Philox key of SBR_RAYS_JITTER                */
} sbr_rays;

/* sbr_rays.options */
#define SBR_RAYS_SHADOW 1    /* sbr_trace tests the return of every hit after the
                                first (whose return retraces its own incoming ray)
                                for occlusion: a hit of another triangle at
                                t in (t_min, D - t_min) along the segment of length D
                                from the hit point to the array centre sets
                                SBR_HIT_OCCLUDED.  Any-hit traversal, early exit. */
#define SBR_RAYS_JITTER 2    /* stratified Monte Carlo sampling (Sec. 3.2.1, Eq. 4):
                                the sample of cell (ix, iy) is uniform in the cell
                                instead of its centre, offsets (u1 - 1/2, u2 - 1/2)
                                cells with u = (w >> 8) / 2^24 of the first two words
                                of Philox-4x32-10 (Salmon et al., SC 2011) at counter
                                (iy * nx + ix, 0, 0, 0), key (seed_lo, seed_hi); the
                                weight is the cell's solid-angle density at the
                                sample.  Every entry point given the same sbr_rays
                                draws the same samples. */

/* Closest-hit records, structure of arrays, each [K][nx*ny] (device). */
typedef struct {
    int32_t *tri;            /* original face index, -1 = no hit (ray ended)     */
    float *t;                /* hit distance along the bounce's unit direction   */
    float *u;                /* barycentric weight of face vertex 1              */
    float *v;                /* barycentric weight of face vertex 2              */
    uint8_t *flags;          /* SBR_HIT_* bits                                   */
} sbr_hits;

/* Hit flags.  With delta_k = 1e-6 m * max(1, path length to hit k / 1 m):   */
#define SBR_HIT_EDGE   1u    /* hit point within delta_k of an edge line          */
#define SBR_HIT_TIE    2u    /* another candidate hit within delta_k of t          */
#define SBR_HIT_GRAZE  4u    /* |d . n| < 1e-6                                     */
#define SBR_HIT_TMIN   8u    /* t < 2 t_min                                        */
#define SBR_HIT_PARENT 16u   /* an earlier bounce of this ray is flagged (bits 1-8) */
#define SBR_HIT_OCCLUDED 32u /* return segment blocked (SBR_RAYS_SHADOW); this record
                                returns no path, later bounces of the ray still do;
                                not inherited through SBR_HIT_PARENT               */

/* sbr_synth_if / sbr_backward flags */
#define SBR_DROP_FLAGGED 1   /* a record with a flag other than SBR_HIT_OCCLUDED
                                ends the ray's paths (it and later bounces)         */
#define SBR_EXIT_ONLY 4      /* only the last hit of each ray returns (classic SBR
                                exit ray); none if that record is skipped           */
#define SBR_ATTACHED 2       /* sbr_backward only: differentiate the reparameterised
                                estimator of Sec. 3.2.1 Eqs. 6-7 in which every sample
                                follows its first hit (fixed barycentrics on the moving
                                triangle, ray turned through it, cell weight times
                                |det J_T| = D / D_0 with D = |N . (x - o)| / |x - o|^3);
                                moving silhouettes then contribute.  The forward
                                signal is the same; without the flag the gradient is
                                the pathwise one with fixed ray directions. */
#define SBR_PATHS_IN_SCRATCH 16 /* sbr_backward only: skip the path stage (FP64
                                path records and their ray-major compaction) and
                                use the records already in `scratch`.  The caller
                                vouches that the last call that wrote this scratch
                                was an sbr_synth_if with the same mesh, materials,
                                radar, rays, hits, chirp and SBR_DROP_FLAGGED /
                                SBR_EXIT_ONLY flags (both entry points lay the
                                records out alike); the library cannot check this.
                                It saves recomputing identical records when a
                                backward pass follows its forward pass.            */
#define SBR_DIRECT_SUMS 8    /* sum Eq. 8 (sbr_synth_if) and the per-path series of
                                Eqs. 11-12 (sbr_backward) directly over paths and
                                samples rather than by the non-uniform FFT forms
                                described at those entry points; chirps of fewer
                                than 16 or more than 1024 samples always use the
                                direct sums                                        */

/* scratch-size queries */
#define SBR_OP_BUILD_BVH 0
#define SBR_OP_SYNTH 1
#define SBR_OP_BACKWARD 2
#define SBR_OP_RADAR_CUBE 3
#define SBR_OP_CFAR 4

/* Bytes of the BVH buffer for nf triangles. */
size_t sbr_bvh_bytes(int32_t nf);

/* Scratch bytes an operation needs.  Pointers that the operation does not
 * depend on may be NULL (BUILD_BVH: mesh; SYNTH/BACKWARD: rays, radar, chirp;
 * RADAR_CUBE and CFAR: chirp + radar give V, C, S; n_angle is taken as 64 or
 * V, whichever is larger).  Returns 0 for bad arguments. */
size_t sbr_scratch_bytes(int32_t op, const sbr_mesh *mesh, const sbr_rays *rays,
                         const sbr_radar *radar, const sbr_chirp *chirp);

/* Build (mode 0) or refit (mode 1) the bounding volume hierarchy of a mesh.
 * BUILD sorts triangles by 30-bit Morton code of their centroids, forms the
 * binary radix tree (Karras, HPG 2012), computes boxes bottom-up and lays
 * nodes out in depth-first order with escape links for stackless traversal.
 * REFIT keeps the tree of the last BUILD of this buffer (same faces, new
 * vertex positions) and recomputes boxes and triangle data.  A BUILD seals
 * the buffer with its face count; a REFIT of a buffer that no BUILD for
 * mesh->nf faces has sealed changes nothing but sets the buffer's int32
 * word 2 to 1, and sbr_trace reports every ray of such a buffer as a miss.
 * bvh: device buffer of at least sbr_bvh_bytes(nf).  The BVH is not part of
 * the paper's method; it accelerates the closest-hit queries of Sec. 3.2.1. */
int sbr_build_bvh(const sbr_mesh *mesh, void *bvh, size_t bvh_bytes, int32_t mode,
                  void *scratch, size_t scratch_bytes, void *stream);

/* Ray tracing forward simulation (Sec. 3.2.1): launch the grid from the radar
 * origin, find the closest hit of each ray (minimum of (t, face index), the
 * previous face excluded, t > t_min, two-sided, degenerate faces never hit),
 * reflect specularly about the face normal (recursive term of Eq. 1) and
 * repeat up to K bounces or the first miss.  Writes out->* for all K*R
 * records.  counters: NULL or device uint64[3] that receives += (closest-hit
 * queries issued incl. the final miss, BVH nodes tested, triangles tested). */
int sbr_trace(const sbr_mesh *mesh, const void *bvh, const sbr_radar *radar,
              const sbr_rays *rays, const sbr_hits *out, uint64_t *counters, void *stream);

/* IF signal synthesis (Eq. 8).  For every (ray, bounce) hit -- minus
 * occluded records, flagged ones with SBR_DROP_FLAGGED and all but the last
 * with SBR_EXIT_ONLY -- one path returns to every virtual antenna:
 *   I^s = d_omega * prod_j r_j * cos(theta_k) / (L_k R_k)
 *   I^t_v(c) = (|x_1 - tx_t| + sum_{j=2..k} |x_j - x_{j-1}| + |rx_m - x_k|) / c0
 *              + c * t_chirp * 2 (velocity . d_1) / c0
 * with hit points x_j recomputed in double precision from the face indices,
 * L_k the unfolded path length, R_k = |x_k - origin|, theta_k the incidence
 * angle at the last hit and r_j the material reflection coefficients.
 *   if_cube[v][c][s] = sum_paths I^s exp(2 pi j (slope s / fs + fc) I^t_v(c))
 * Each row if_cube[v][c][.] is a finite Fourier series in s whose terms sit at
 * the paths' beat frequencies.  For 16 <= S <= 1024 it is formed by a type-1
 * non-uniform FFT: every path's term is spread onto a 2S-point grid with 7
 * exponential-of-semicircle kernel taps, each contribution rounded to an
 * integer (a power-of-two scale between 2^18 and 2^19 over the largest
 * max(|Re I^s|, |Im I^s|) of its chunk of paths; the chunks depend only on the
 * call's sizes) and accumulated exactly in 64-bit integers, so the result
 * does not depend on the order of the additions; one DFT per row and the
 * kernel's deconvolution follow.  The kernel's error is below 1e-6 of
 * sum_paths |I^s| per sample; each tap's rounding adds at most 2^-19 of that
 * largest component of its chunk.
 * With SBR_DIRECT_SUMS, or for other S, the sum is taken directly.
 * if_cube: device float [V][C][S][2], overwritten.  mats: host array of
 * n_mats (<= 64) entries, or NULL / 0 for all-conductor.  A hit id outside
 * [0, nf) ends its ray like a miss (no face outside the mesh is read). */
int sbr_synth_if(const sbr_mesh *mesh, const sbr_material *mats, int32_t n_mats,
                 const sbr_radar *radar, const sbr_rays *rays, const sbr_hits *hits,
                 const sbr_chirp *chirp, int32_t flags, float *if_cube,
                 void *scratch, size_t scratch_bytes, void *stream);

/* The signal-to-image map T of the spatial multi-antenna loss (Eq. 16):
 * range, Doppler and angle DFTs,
 *   X[a][d][r] = sum_{v,c,s} w(s) w(c) S[v][c][s] e^{-2 pi j (r s/S + d c/C + a v/Na)}
 * (v zero-padded to n_angle >= V, no normalisation, no shift; window 0 =
 * rectangular, 1 = symmetric Hann on the range and Doppler axes).
 * direction 0: in [V][C][S][2] -> out [Na][C][S][2].  direction 1 applies the
 * conjugate transpose: in [Na][C][S][2] -> out [V][C][S][2] (the gradient of
 * a real loss with respect to S, given its gradient with respect to X).
 * FP32 throughout: power-of-two range and Doppler lengths run as FFTs, other
 * lengths as dense contractions with the DFT matrix on the matrix cores;
 * results agree with the direct sum to FP32 rounding, not bit for bit across
 * shapes.  V, C, S and n_angle are each at most 4096; scratch:
 * sbr_scratch_bytes(SBR_OP_RADAR_CUBE, ...) for n_angle = max(64, V), else
 * sbr_radar_cube_2d_bytes(V, 1, C, S, n_angle, 1). */
int sbr_radar_cube(const float *in, int32_t V, int32_t C, int32_t S, int32_t n_angle,
                   int32_t window, int32_t direction, float *out, void *scratch,
                   size_t scratch_bytes, void *stream);

/* sbr_radar_cube without a scratch argument, for callers that cannot
 * allocate device memory (code under HIP graph capture, tight serving loops,
 * harnesses that forbid hipMalloc): the staging buffers are a file-scope
 * device array of SBR_NOALLOC_SCRATCH_BYTES that each GPU the library runs on
 * holds until the process ends; nothing is allocated or freed.  Arguments,
 * result and limits as sbr_radar_cube, and sizes whose staging
 * (sbr_scratch_bytes(SBR_OP_RADAR_CUBE, ...) for that n_angle) exceeds the
 * array are refused with SBR_E_SCRATCH before anything is enqueued.  All
 * calls on one GPU share its array: calls that overlap on one GPU (other
 * streams, other threads) race and must be ordered by the caller. */
#define SBR_NOALLOC_SCRATCH_BYTES (64 << 20)
int sbr_radar_cube_noalloc(const float *in, int32_t V, int32_t C, int32_t S, int32_t n_angle, int32_t window,
                           int32_t direction, float *out, void *stream);

/* The same map T for a planar array (Sec. 4's 20 TX x 20 RX class of radar):
 * the virtual antennas form a Vy x Vx grid, v = vy * Vx + vx (for example TX
 * t along one axis and RX m along the other: vy = t, vx = m).  Range and
 * Doppler as above; the angle stage is the 2D DFT over (vy, vx) zero-padded
 * to (n_ay, n_ax), output angle index a = ay * n_ax + ax.
 * direction 0: in [Vy*Vx][C][S][2] -> out [n_ay*n_ax][C][S][2]; direction 1
 * applies the conjugate transpose.  Needs n_ax >= Vx, n_ay >= Vy and fewer
 * than 2^31 cells per cube; scratch: sbr_radar_cube_2d_bytes(...) bytes.
 * With Vy = n_ay = 1 it equals sbr_radar_cube. */
int sbr_radar_cube_2d(const float *in, int32_t Vx, int32_t Vy, int32_t C, int32_t S,
                      int32_t n_ax, int32_t n_ay, int32_t window, int32_t direction,
                      float *out, void *scratch, size_t scratch_bytes, void *stream);

/* Scratch bytes of sbr_radar_cube_2d; 0 for invalid sizes. */
size_t sbr_radar_cube_2d_bytes(int32_t Vx, int32_t Vy, int32_t C, int32_t S, int32_t n_ax,
                               int32_t n_ay);

/* Radar point cloud from the cube: square-law cell-averaging CFAR on
 * P[d][r] = sum_a |X[a][d][r]|^2 with a (2(guard+train)+1)^2 window minus the
 * (2 guard+1)^2 guard cells, Doppler axis circular, range axis truncated,
 * threshold alpha * mean with alpha = N_t (pfa^(-1/N_t) - 1).
 * cube: device [Na][C][S][2].  points: device int32 [max_points][4] =
 * (range bin, Doppler bin, argmax_a |X|^2 (lowest on ties), 0) in row-major
 * (d, r) order; ratio: device float [max_points] = P / threshold, or NULL;
 * n_points: device int32, total detections (may exceed max_points).
 * Sizes: Na <= 65536, C and S <= 4096, guard + train < 4096; scratch:
 * sbr_scratch_bytes(SBR_OP_CFAR, ...). */
int sbr_cfar(const float *cube, int32_t Na, int32_t C, int32_t S, int32_t guard,
             int32_t train, double pfa, int32_t *points, float *ratio, int32_t max_points,
             int32_t *n_points, void *scratch, size_t scratch_bytes, void *stream);

/* Angle peaks of detected range-Doppler cells, the several scatterers per
 * cell a radar's angle search reports.  For each detection i < min(*n_det,
 * max_det) (det: device int32 [max_det][4] as sbr_cfar writes them) its angle
 * spectrum q[a] = |X[a][d][r]|^2 (cube [n_ay*n_ax][C][S][2]) is searched for
 * local maxima over the circular angle grid (ring if n_ay = 1, else the
 * 8-neighbourhood on the n_ay x n_ax torus; among equal neighbours the lower
 * index wins) holding at least rel (0..1) of the cell's largest q.  points:
 * device int32 [max_points][4] = (range bin, Doppler bin, angle index, 0),
 * detection-major, angle ascending; n_points: device int32 total (may exceed
 * max_points).  scratch: sbr_angle_peaks_bytes(max_det, n_ax, n_ay). */
int sbr_angle_peaks(const float *cube, int32_t n_ax, int32_t n_ay, int32_t C, int32_t S,
                    const int32_t *det, const int32_t *n_det, int32_t max_det, float rel,
                    int32_t *points, int32_t max_points, int32_t *n_points, void *scratch,
                    size_t scratch_bytes, void *stream);

/* Scratch bytes of sbr_angle_peaks; 0 for invalid sizes. */
size_t sbr_angle_peaks_bytes(int32_t max_det, int32_t n_ax, int32_t n_ay);

/* Radar point cloud: CFAR detections to world points (Sec. 4: the radars
 * output point clouds; Fig. 1 initialises the scene from them).  points:
 * device int32 [max_points][4] as sbr_cfar writes them; n_points: device
 * int32 count (entries past min(count, max_points) are written as NaN).
 * Range bin r -> R = c r f_s / (2 mu S) from the array centre; Doppler bin d
 * -> radial velocity c d_s / (2 C f_c t_chirp) (positive = receding); angle
 * index a = ay * n_ax + ax of the cube over a lambda/2 array -> direction
 * cosines u_x = -2 ax_s / n_ax and, for n_ay > 1 (planar array,
 * sbr_radar_cube_2d), u_y = -2 ay_s / n_ay, else u_y = 0 (a linear array
 * along x measures no elevation); a_s is the signed bin.  out: device float
 * [max_points][4] = world x, y, z, radial velocity. */
int sbr_cloud(const int32_t *points, const int32_t *n_points, int32_t max_points,
              const sbr_radar *radar, const sbr_chirp *chirp, int32_t n_ax, int32_t n_ay,
              float *out, void *stream);

/* Gradients with respect to scene parameters other than the vertices (the
 * material, pose and dynamics entries of Theta, Sec. 3.2).  Device arrays,
 * accumulated (+=); either pointer may be NULL. */
typedef struct {
    float *materials;        /* [n_mats][2]: dL/d eps_r, dL/d sigma per table entry */
    float *radar;            /* [6]: dL/d origin (world x, y, z), dL/d velocity (x, y, z) */
    float *rot;              /* [9]: dL/d rot, row-major like sbr_radar.rot (the full
                                3x3 matrix; project onto a rotation parameterisation
                                outside, e.g. dL/d omega = axial part of G R^T) */
    float *attenuation;      /* [1]: dL/d sbr_radar.attenuation (Eq. 5)          */
} sbr_param_grads;

/* Backpropagation (Sec. 3.2.2 Eqs. 11-12, Sec. 3.3 Eq. 13): given
 * grad_if = dL/dRe S + i dL/dIm S ([V][C][S][2], device), ADD dL/dverts to
 * grad_verts ([nv][3], device).  The gradient is the pathwise derivative of
 * the fixed-grid estimator: each path's geometry is recomputed per bounce
 * from the hit records (nothing of the forward synthesis is stored) and the
 * reverse sweep runs through path lengths, ray-plane intersections,
 * reflections, normals and Fresnel coefficients.  Per path, antenna v and
 * chirp c the adjoint needs two finite Fourier series of the gradient row
 * G[v][c][.] at the path's beat frequency g: P(g) = sum_s conj(G_s)
 * e^{2 pi j s g} (Eq. 12) and the same sum weighted by fc + (slope/fs) s
 * (Eq. 11).  For 16 <= S <= 1024 they are evaluated by a type-2 non-uniform
 * FFT (one 2S-point transform per row, shared by all paths, then 7 kernel taps
 * per path; exponential-of-semicircle kernel), whose error is below 1e-6 of
 * sum_s |weighted G_s| at every g; with SBR_DIRECT_SUMS, or for other S, by
 * direct summation.  Arguments as for sbr_synth_if; hits and flags must be
 * those the forward used (plus SBR_ATTACHED, and SBR_PATHS_IN_SCRATCH when
 * the scratch still holds that forward's path records).  params: NULL,
 * or where to ADD the gradients of the material table (Eqs. 9-10 through
 * eps_c), of the radar origin (ray origins, TX and RX positions, return
 * distances), of the radar rotation (ray directions, TX and RX positions,
 * Doppler direction) and of the scene velocity (Doppler term of I^t). */
int sbr_backward(const sbr_mesh *mesh, const sbr_material *mats, int32_t n_mats,
                 const sbr_radar *radar, const sbr_rays *rays, const sbr_hits *hits,
                 const sbr_chirp *chirp, int32_t flags, const float *grad_if,
                 float *grad_verts, const sbr_param_grads *params, void *scratch,
                 size_t scratch_bytes, void *stream);

/* Number of paths the last sbr_synth_if / sbr_backward found is left in the
 * first int32 of their scratch buffer (device) once the stream reaches it. */

/* ---- Batched entry points (serving many simulations on one device) ------
 * Not part of the paper's method: they run several independent requests'
 * Eq. 8 synthesis, or Eqs. 11-13 adjoints, as one launch, so small requests
 * fill the device together.  Each request carries exactly the arguments of
 * sbr_synth_if (if_cube) or sbr_backward (grad_if, grad_verts, params), with
 * its own scratch of the size those calls need; requests must not share
 * scratch, outputs or (for the backward) grad_verts.  A request's launch
 * shapes depend only on its own sizes, so its IF cube is bit-identical to
 * sbr_synth_if's and its gradients equal sbr_backward's up to the order of
 * floating-point atomics. */
#define SBR_MAX_BATCH 1024

typedef struct {
    const sbr_mesh *mesh;
    const sbr_material *mats;       /* host, n_mats entries, or NULL          */
    int32_t n_mats;
    int32_t flags;                  /* as for sbr_synth_if / sbr_backward     */
    const sbr_radar *radar;
    const sbr_rays *rays;
    const sbr_hits *hits;
    const sbr_chirp *chirp;
    float *if_cube;                 /* synthesis: [V][C][S][2], overwritten   */
    const float *grad_if;           /* backward: dL/dRe S + i dL/dIm S        */
    float *grad_verts;              /* backward: [nv][3], accumulated (+=)     */
    const sbr_param_grads *params;  /* backward: NULL or where to add them    */
    void *scratch;                  /* device, >= sbr_scratch_bytes of the op */
    size_t scratch_bytes;
} sbr_request;

/* Bytes of the device table a batched call of n (1..SBR_MAX_BATCH) requests
 * needs; 0 for other n. */
size_t sbr_batch_table_bytes(int32_t n_requests);

/* sbr_synth_if for each of reqs[0..n) (host array), enqueued on `stream`:
 * every request's path stage, then ONE launch per sample-run length over the
 * synthesis blocks of all requests -- a device table (written by the call
 * into `table`, device memory of sbr_batch_table_bytes(n) bytes, not to be
 * reused until the stream has passed this call) gives each block its request
 * -- then each request's fixed-order reduction into its if_cube.  Every
 * request is checked before anything is enqueued; the error message names
 * the first bad one. */
int sbr_synth_if_batched(const sbr_request *reqs, int32_t n, void *table, size_t table_bytes, void *stream);

/* sbr_backward for each of reqs[0..n): every request's path stage, ONE
 * work-queue launch of the synthesis adjoint (Eqs. 11-12) whose items --
 * (antenna group, path tile) of every request, counted on the device -- are
 * mapped to their request through the device table, then each request's
 * geometry adjoint (Eq. 13).  Table and checks as sbr_synth_if_batched. */
int sbr_backward_batched(const sbr_request *reqs, int32_t n, void *table, size_t table_bytes, void *stream);

/* Loss of the inverse problem (Sec. 3.4.1, Eq. 14) and its gradient, the
 * entry point of the backward pass.  n complex elements, device arrays.
 * mode 0 (IF loss):      L = sum |a - b|^2,                 grad = 2 (a - b)
 * mode 1 (heatmap loss, the MSE of Eq. 16 on the image |X|^2, with a = X and
 *   b = the target heatmap H as float [n]): L = mean (|a|^2 - H)^2,
 *   grad = 4 (|a|^2 - H) a / n
 * grad: device float [n][2] = dL/dRe a + i dL/dIm a (overwritten; may be NULL);
 * loss: device float[1] (overwritten; may be NULL).  The sum is reduced in a
 * fixed order (deterministic): per-block partials in double, then one block.
 * scratch: device buffer of SBR_LOSS_SCRATCH_BYTES for those partials
 * (needed only when loss is not NULL). */
#define SBR_LOSS_SCRATCH_BYTES 8192
int sbr_loss_grad(int32_t mode, const float *a, const float *b, int64_t n, float *grad,
                  float *loss, void *scratch, size_t scratch_bytes, void *stream);

/* Kernel timing for benchmarks.  sbr_profile(1) starts bracketing, with HIP
 * events on the launching stream, every IF synthesis (id 0: all kernels of
 * one request's Eq. 8 stage), synthesis adjoint (id 1: all kernels of one
 * request's Eqs. 11-12 stage), trace kernel (id 2), and within the
 * non-uniform FFT forms the spreading kernel of the synthesis (id 3) and the
 * tap kernel of the adjoint (id 4);
 * sbr_profile(0) stops; sbr_profile(2) discards what was recorded.
 * sbr_profile_read waits for the recorded events of one kernel id and returns
 * the summed milliseconds and the number of launches, then discards them. */
int sbr_profile(int32_t op);
int sbr_profile_read(int32_t kernel, double *total_ms, int64_t *launches);

/* Message describing the calling thread's last error ("" if none). */
const char *sbr_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
