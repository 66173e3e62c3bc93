/* A plain C11 consumer of the library: only include/mcl.h and the HIP runtime's
 * C API, no Python and no torch.  It runs one filter update through the
 * single-filter calls (sensor update, normalisation, resampling), then the same
 * filter and a second one (another sigma and update count) as one tick captured
 * into a graph and replayed, frees the map while the replay may still run (the
 * release is deferred), checks that an invalid call reports its error, and
 * writes every output to files for the test to compare with the oracle.
 *
 * usage: mcl_consumer DIR NX NY NZ VOXEL OX OY OZ TAU K N SIGMA SEED
 *   DIR/map.bin     int16 [NZ][NY][NX] (x fastest)
 *   DIR/points.bin  float32 [3][K]
 *   DIR/poses.bin   float32 [12][N]
 * writes DIR/<set>_{logw,w,wq,lz,idx,pout}.bin for set = single, tick0, tick1. */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "mcl.h"

#define CHECK_HIP(x)                                                          \
    do {                                                                      \
        hipError_t e_ = (x);                                                  \
        if (e_ != hipSuccess) {                                               \
            fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, hipGetErrorString(e_)); \
            exit(1);                                                          \
        }                                                                     \
    } while (0)

#define CHECK_MCL(x)                                                          \
    do {                                                                      \
        mcl_status s_ = (x);                                                  \
        if (s_ != MCL_OK) {                                                   \
            fprintf(stderr, "%s:%d: status %d: %s\n", __FILE__, __LINE__, (int)s_, mcl_last_error()); \
            exit(1);                                                          \
        }                                                                     \
    } while (0)

static void *read_file(const char *dir, const char *name, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s", dir, name);
    FILE *f = fopen(path, "rb");
    if (!f) {
        fprintf(stderr, "cannot open %s\n", path);
        exit(1);
    }
    void *p = malloc(bytes ? bytes : 1);
    if (!p || fread(p, 1, bytes, f) != bytes) {
        fprintf(stderr, "short read of %s\n", path);
        exit(1);
    }
    fclose(f);
    return p;
}

static void write_device(const char *dir, const char *set, const char *name, const void *dev, size_t bytes) {
    char path[4096];
    snprintf(path, sizeof path, "%s/%s_%s.bin", dir, set, name);
    void *h = malloc(bytes);
    if (!h) exit(1);
    CHECK_HIP(hipMemcpy(h, dev, bytes, hipMemcpyDeviceToHost));
    FILE *f = fopen(path, "wb");
    if (!f || fwrite(h, 1, bytes, f) != bytes) {
        fprintf(stderr, "cannot write %s\n", path);
        exit(1);
    }
    fclose(f);
    free(h);
}

typedef struct {
    float *logw, *pout;
    double *w, *lz;
    uint64_t *wq;
    int32_t *idx;
} outputs;

static void alloc_outputs(outputs *o, int N) {
    CHECK_HIP(hipMalloc((void **)&o->logw, (size_t)N * 4));
    CHECK_HIP(hipMalloc((void **)&o->w, (size_t)N * 8));
    CHECK_HIP(hipMalloc((void **)&o->wq, (size_t)N * 8));
    CHECK_HIP(hipMalloc((void **)&o->lz, 8));
    CHECK_HIP(hipMalloc((void **)&o->idx, (size_t)N * 4));
    CHECK_HIP(hipMalloc((void **)&o->pout, (size_t)12 * N * 4));
}

static void write_outputs(const char *dir, const char *set, const outputs *o, int N) {
    write_device(dir, set, "logw", o->logw, (size_t)N * 4);
    write_device(dir, set, "w", o->w, (size_t)N * 8);
    write_device(dir, set, "wq", o->wq, (size_t)N * 8);
    write_device(dir, set, "lz", o->lz, 8);
    write_device(dir, set, "idx", o->idx, (size_t)N * 4);
    write_device(dir, set, "pout", o->pout, (size_t)12 * N * 4);
}

static mcl_filter_job job_for(mcl_map map, const float *pts, int K, const float *poses, int N, float sigma,
                              uint64_t seed, uint64_t tick, const outputs *o) {
    mcl_filter_job j;
    memset(&j, 0, sizeof j);
    j.map = map;
    j.points = pts;
    j.K = K;
    j.poses = poses;
    j.N = N;
    j.sigma = sigma;
    j.logw = o->logw;
    j.w = o->w;
    j.wq = o->wq;
    j.log_z = o->lz;
    j.seed = seed;
    j.tick = tick;
    j.idx = o->idx;
    j.poses_out = o->pout;
    j.lookup = MCL_LOOKUP_NEAREST;
    j.score = MCL_SCORE_PRODUCT;
    return j;
}

int main(int argc, char **argv) {
    if (argc != 14) {
        fprintf(stderr, "usage: %s DIR NX NY NZ VOXEL OX OY OZ TAU K N SIGMA SEED\n", argv[0]);
        return 2;
    }
    const char *dir = argv[1];
    mcl_map_desc desc;
    desc.nx = atoi(argv[2]);
    desc.ny = atoi(argv[3]);
    desc.nz = atoi(argv[4]);
    desc.voxel = strtof(argv[5], NULL);
    desc.origin[0] = strtof(argv[6], NULL);
    desc.origin[1] = strtof(argv[7], NULL);
    desc.origin[2] = strtof(argv[8], NULL);
    desc.tau = strtof(argv[9], NULL);
    desc.dtype = MCL_TSDF_I16;
    const int K = atoi(argv[10]), N = atoi(argv[11]);
    const float sigma = strtof(argv[12], NULL);
    const uint64_t seed = strtoull(argv[13], NULL, 10);

    const size_t nvox = (size_t)desc.nx * desc.ny * desc.nz;
    int16_t *hmap = (int16_t *)read_file(dir, "map.bin", nvox * 2);
    float *hpts = (float *)read_file(dir, "points.bin", (size_t)3 * K * 4);
    float *hposes = (float *)read_file(dir, "poses.bin", (size_t)12 * N * 4);

    hipStream_t s;
    CHECK_HIP(hipStreamCreate(&s));
    mcl_map map = NULL;
    CHECK_MCL(mcl_map_upload(&desc, hmap, s, &map));

    float *pts, *poses;
    CHECK_HIP(hipMalloc((void **)&pts, (size_t)3 * K * 4));
    CHECK_HIP(hipMalloc((void **)&poses, (size_t)12 * N * 4));
    CHECK_HIP(hipMemcpy(pts, hpts, (size_t)3 * K * 4, hipMemcpyHostToDevice));
    CHECK_HIP(hipMemcpy(poses, hposes, (size_t)12 * N * 4, hipMemcpyHostToDevice));

    /* single-filter calls */
    outputs one, t0, t1;
    alloc_outputs(&one, N);
    alloc_outputs(&t0, N);
    alloc_outputs(&t1, N);
    CHECK_MCL(mcl_sensor_update(map, pts, K, poses, N, sigma, one.logw, s));
    CHECK_MCL(mcl_normalize(one.logw, N, one.w, one.wq, one.lz, s));
    CHECK_MCL(mcl_resample(one.wq, N, seed, 0, one.idx, poses, one.pout, s));

    /* an argument error is reported, not raised */
    if (mcl_sensor_update(NULL, pts, K, poses, N, sigma, one.logw, s) != MCL_EINVAL || !mcl_last_error()[0]) {
        fprintf(stderr, "a NULL map was not refused\n");
        return 1;
    }

    /* the same filter and a second one as a tick, captured then replayed */
    mcl_filter_job jobs[2];
    jobs[0] = job_for(map, pts, K, poses, N, sigma, seed, 0, &t0);
    jobs[1] = job_for(map, pts, K, poses, N, 1.5f * sigma, seed + 1, 1, &t1);
    CHECK_MCL(mcl_tick(jobs, 2, MCL_TICK_GRAPH, s));
    CHECK_HIP(hipStreamSynchronize(s));
    CHECK_HIP(hipMemsetAsync(t0.logw, 0, (size_t)N * 4, s));
    CHECK_HIP(hipMemsetAsync(t1.idx, 0, (size_t)N * 4, s));
    CHECK_MCL(mcl_tick(jobs, 2, MCL_TICK_GRAPH, s));
    /* released once the work enqueued on the map has completed */
    CHECK_MCL(mcl_map_free(map));
    CHECK_HIP(hipStreamSynchronize(s));

    write_outputs(dir, "single", &one, N);
    write_outputs(dir, "tick0", &t0, N);
    write_outputs(dir, "tick1", &t1, N);
    CHECK_HIP(hipStreamDestroy(s));
    free(hmap);
    free(hpts);
    free(hposes);
    printf("ok\n");
    return 0;
}
