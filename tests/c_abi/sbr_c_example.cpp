// A caller of libsbr that uses nothing but the C ABI and the HIP runtime:
// no Python, no PyTorch.  It reads a scene written by the test suite, builds
// the BVH, traces, synthesizes the IF cube and its range/Doppler/angle image,
// and writes both back.
//
// Input file (little-endian): int32 nv, nf; float32 verts[nv][3]; int32
// faces[nf][3]; sbr_radar; sbr_rays; sbr_chirp (the structs of sbr.h, as laid
// out by this compiler).  Output file: float32 cube[V][C][S][2] then
// float32 image[n_angle][C][S][2], n_angle = 64.
#include <hip/hip_runtime.h>
#include <stdio.h>
#include <stdlib.h>
#include <vector>

#include "sbr.h"

#define CHECK_HIP(x)                                                               \
    do {                                                                           \
        hipError_t e_ = (x);                                                       \
        if (e_ != hipSuccess) {                                                    \
            fprintf(stderr, "HIP error %s at %s:%d\n", hipGetErrorString(e_), __FILE__, __LINE__); \
            return 2;                                                              \
        }                                                                          \
    } while (0)
#define CHECK_SBR(x)                                                               \
    do {                                                                           \
        int r_ = (x);                                                              \
        if (r_ != SBR_OK) {                                                        \
            fprintf(stderr, "sbr error %d: %s (%s:%d)\n", r_, sbr_last_error(), __FILE__, __LINE__); \
            return 3;                                                              \
        }                                                                          \
    } while (0)

template <typename T>
static bool rd(FILE *f, T *p, size_t n) { return fread(p, sizeof(T), n, f) == n; }

int main(int argc, char **argv) {
    if (argc != 3) {
        fprintf(stderr, "usage: %s scene.bin out.bin\n", argv[0]);
        return 1;
    }
    FILE *f = fopen(argv[1], "rb");
    if (!f) return 1;
    int32_t nv = 0, nf = 0;
    if (!rd(f, &nv, 1) || !rd(f, &nf, 1) || nv <= 0 || nf <= 0) return 1;
    std::vector<float> verts((size_t)nv * 3);
    std::vector<int32_t> faces((size_t)nf * 3);
    sbr_radar radar;
    sbr_rays rays;
    sbr_chirp chirp;
    if (!rd(f, verts.data(), verts.size()) || !rd(f, faces.data(), faces.size()) || !rd(f, &radar, 1) ||
        !rd(f, &rays, 1) || !rd(f, &chirp, 1))
        return 1;
    fclose(f);

    const int R = rays.nx * rays.ny, K = rays.max_bounces;
    const int V = radar.n_tx * radar.n_rx, C = chirp.n_chirps, S = chirp.n_samples, Na = 64;
    float *d_verts, *d_t, *d_u, *d_v, *d_cube, *d_img;
    int32_t *d_faces, *d_tri;
    uint8_t *d_flags;
    CHECK_HIP(hipMalloc(&d_verts, verts.size() * sizeof(float)));
    CHECK_HIP(hipMalloc(&d_faces, faces.size() * sizeof(int32_t)));
    CHECK_HIP(hipMemcpy(d_verts, verts.data(), verts.size() * sizeof(float), hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(d_faces, faces.data(), faces.size() * sizeof(int32_t), hipMemcpyHostToDevice));
    CHECK_HIP(hipMalloc(&d_tri, (size_t)K * R * sizeof(int32_t)));
    CHECK_HIP(hipMalloc(&d_t, (size_t)K * R * sizeof(float)));
    CHECK_HIP(hipMalloc(&d_u, (size_t)K * R * sizeof(float)));
    CHECK_HIP(hipMalloc(&d_v, (size_t)K * R * sizeof(float)));
    CHECK_HIP(hipMalloc(&d_flags, (size_t)K * R));
    CHECK_HIP(hipMalloc(&d_cube, (size_t)V * C * S * 2 * sizeof(float)));
    CHECK_HIP(hipMalloc(&d_img, (size_t)Na * C * S * 2 * sizeof(float)));

    sbr_mesh mesh = {d_verts, nv, d_faces, nf, nullptr};
    sbr_hits hits = {d_tri, d_t, d_u, d_v, d_flags};
    size_t bvh_bytes = sbr_bvh_bytes(nf);
    size_t scratch = sbr_scratch_bytes(SBR_OP_BUILD_BVH, &mesh, nullptr, nullptr, nullptr);
    size_t s2 = sbr_scratch_bytes(SBR_OP_SYNTH, &mesh, &rays, &radar, &chirp);
    size_t s3 = sbr_scratch_bytes(SBR_OP_RADAR_CUBE, nullptr, &rays, &radar, &chirp);
    if (s2 > scratch) scratch = s2;
    if (s3 > scratch) scratch = s3;
    if (bvh_bytes == 0 || scratch == 0) {
        fprintf(stderr, "size query failed: %s\n", sbr_last_error());
        return 3;
    }
    void *d_bvh, *d_scratch;
    CHECK_HIP(hipMalloc(&d_bvh, bvh_bytes));
    CHECK_HIP(hipMalloc(&d_scratch, scratch));
    hipStream_t s;
    CHECK_HIP(hipStreamCreate(&s));
    CHECK_SBR(sbr_build_bvh(&mesh, d_bvh, bvh_bytes, 0, d_scratch, scratch, s));
    CHECK_SBR(sbr_trace(&mesh, d_bvh, &radar, &rays, &hits, nullptr, s));
    CHECK_SBR(sbr_synth_if(&mesh, nullptr, 0, &radar, &rays, &hits, &chirp, SBR_DROP_FLAGGED, d_cube, d_scratch,
                           scratch, s));
    CHECK_SBR(sbr_radar_cube(d_cube, V, C, S, Na, 0, 0, d_img, d_scratch, scratch, s));
    CHECK_HIP(hipStreamSynchronize(s));

    std::vector<float> cube((size_t)V * C * S * 2), img((size_t)Na * C * S * 2);
    CHECK_HIP(hipMemcpy(cube.data(), d_cube, cube.size() * sizeof(float), hipMemcpyDeviceToHost));
    CHECK_HIP(hipMemcpy(img.data(), d_img, img.size() * sizeof(float), hipMemcpyDeviceToHost));
    FILE *o = fopen(argv[2], "wb");
    if (!o) return 1;
    fwrite(cube.data(), sizeof(float), cube.size(), o);
    fwrite(img.data(), sizeof(float), img.size(), o);
    fclose(o);
    CHECK_HIP(hipStreamDestroy(s));
    void *bufs[] = {d_verts, d_faces, d_tri, d_t, d_u, d_v, d_flags, d_cube, d_img, d_bvh, d_scratch};
    for (void *b : bufs) CHECK_HIP(hipFree(b));
    printf("ok V=%d C=%d S=%d\n", V, C, S);
    return 0;
}
