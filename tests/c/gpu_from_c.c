/* The C ABI used from plain C99 on the GPU, with no Python and no torch:
 * device memory from hipMalloc, a stream of the caller's own, and the
 * library's entry points in the order a C or Fortran PIC code would call
 * them.  Writes the outputs as raw little-endian arrays into the directory
 * argv[1], where the test compares them with the oracle:
 *   f32.bin   vx, vy, vz (float, n each) of kappa_sample, FP32 mode
 *   f64.bin   vx, vy, vz (double, n each) of kappa_sample, FP64 mode
 *   plan.bin  vx, vy, vz (float, total each) of kappa_plan_launch
 *   grad.bin  dLoss/dkappa, dLoss/dtheta (double) of kappa_sample_backward
 *   g.bin     the upstream gradient gx, gy, gz (float, n each) it was given
 * and checks on its own that the plan's graph replay equals its direct
 * launch bit for bit.  Prints "ok" and exits 0 when every call succeeded. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <hip/hip_runtime_api.h>

#include "kappa.h"

#define N 100003u /* ragged: not a multiple of any vector width */

static int hip_ok(hipError_t e, const char *what)
{
    if (e != hipSuccess) {
        printf("FAIL %s: %s\n", what, hipGetErrorString(e));
        return 0;
    }
    return 1;
}

static int kappa_ok(kappa_status s, const char *what)
{
    if (s != KAPPA_OK) {
        printf("FAIL %s: %s (%s)\n", what, kappa_status_string(s), kappa_last_error());
        return 0;
    }
    return 1;
}

static int dump(const char *dir, const char *name, void *const *dev, size_t nbuf, size_t bytes)
{
    char path[4096];
    size_t k;
    FILE *f;
    void *host = malloc(bytes);
    if (!host) return 0;
    snprintf(path, sizeof path, "%s/%s", dir, name);
    f = fopen(path, "wb");
    if (!f) {
        free(host);
        return 0;
    }
    for (k = 0; k < nbuf; ++k) {
        if (!hip_ok(hipMemcpy(host, dev[k], bytes, hipMemcpyDeviceToHost), "hipMemcpy to host") ||
            fwrite(host, 1, bytes, f) != bytes) {
            fclose(f);
            free(host);
            return 0;
        }
    }
    fclose(f);
    free(host);
    return 1;
}

int main(int argc, char **argv)
{
    hipStream_t stream;
    void *f32[3], *f64[3], *pv[3], *pg[3], *g[3], *grad, *ws;
    float *gh;
    size_t k, ws_bytes;
    uint64_t total = 0;
    kappa_plan plan = NULL;
    kappa_segment segs[3];
    int ok = 1;
    if (argc < 2) return 2;
    if (!hip_ok(hipSetDevice(0), "hipSetDevice") || !hip_ok(hipStreamCreate(&stream), "hipStreamCreate")) return 1;
    for (k = 0; k < 3; ++k) {
        ok = ok && hip_ok(hipMalloc(&f32[k], N * sizeof(float)), "hipMalloc");
        ok = ok && hip_ok(hipMalloc(&f64[k], N * sizeof(double)), "hipMalloc");
        ok = ok && hip_ok(hipMalloc(&g[k], N * sizeof(float)), "hipMalloc");
    }
    if (!ok) return 1;

    /* one species, both precisions */
    ok = ok && kappa_ok(kappa_sample(3.0, 1.0, N, 5, 17, 3, KAPPA_FP32, f32[0], f32[1], f32[2], stream), "FP32");
    ok = ok && kappa_ok(kappa_sample(6.0, 0.5, N, 8, 0, 0, KAPPA_FP64, f64[0], f64[1], f64[2], stream), "FP64");

    /* three species with drifts in one batched launch, direct and through the plan's graph */
    memset(segs, 0, sizeof segs);
    segs[0].kappa = 2.0;  segs[0].theta = 1.0; segs[0].count = 40000; segs[0].seg_id = 0;
    segs[1].kappa = 4.1;  segs[1].theta = 0.7; segs[1].count = 1;     segs[1].seg_id = 1;
    segs[2].kappa = 10.0; segs[2].theta = 2.0; segs[2].count = 33333; segs[2].seg_id = 2;
    segs[0].drift[0] = 0.25; segs[2].drift[1] = -0.5; segs[2].drift[2] = 0.125;
    ok = ok && kappa_ok(kappa_plan_create(segs, 3, 4, KAPPA_FP32, &plan), "kappa_plan_create");
    ok = ok && kappa_ok(kappa_plan_total(plan, &total), "kappa_plan_total");
    for (k = 0; ok && k < 3; ++k) {
        ok = ok && hip_ok(hipMalloc(&pv[k], total * sizeof(float)), "hipMalloc");
        ok = ok && hip_ok(hipMalloc(&pg[k], total * sizeof(float)), "hipMalloc");
    }
    ok = ok && kappa_ok(kappa_plan_launch(plan, pv[0], pv[1], pv[2], stream), "kappa_plan_launch");
    ok = ok && kappa_ok(kappa_plan_graph_launch(plan, pg[0], pg[1], pg[2], stream), "kappa_plan_graph_launch");
    ok = ok && kappa_ok(kappa_plan_graph_launch(plan, pg[0], pg[1], pg[2], stream), "graph replay");

    /* the reparameterisation gradient for a deterministic upstream gradient */
    gh = (float *)malloc(3 * N * sizeof(float));
    if (!gh) return 1;
    for (k = 0; k < 3 * N; ++k) gh[k] = (float)sin(0.37 * (double)k + 0.1);
    for (k = 0; ok && k < 3; ++k)
        ok = hip_ok(hipMemcpy(g[k], gh + k * N, N * sizeof(float), hipMemcpyHostToDevice), "hipMemcpy to device");
    free(gh);
    ws_bytes = kappa_backward_workspace_bytes(N);
    ok = ok && hip_ok(hipMalloc(&grad, 2 * sizeof(double)), "hipMalloc") && hip_ok(hipMalloc(&ws, ws_bytes), "hipMalloc");
    ok = ok && kappa_ok(kappa_sample_backward(2.5, 1.3, N, 2, 0, 0, KAPPA_FP32, g[0], g[1], g[2], grad, ws, ws_bytes,
                                              stream), "kappa_sample_backward");
    ok = ok && hip_ok(hipStreamSynchronize(stream), "hipStreamSynchronize");
    if (!ok) return 1;

    /* graph replay against direct launch, bit for bit */
    {
        float *a = (float *)malloc(total * sizeof(float)), *b = (float *)malloc(total * sizeof(float));
        if (!a || !b) return 1;
        for (k = 0; ok && k < 3; ++k) {
            ok = hip_ok(hipMemcpy(a, pv[k], total * sizeof(float), hipMemcpyDeviceToHost), "copy") &&
                 hip_ok(hipMemcpy(b, pg[k], total * sizeof(float), hipMemcpyDeviceToHost), "copy");
            if (ok && memcmp(a, b, total * sizeof(float)) != 0) {
                printf("FAIL graph replay differs from direct launch in component %u\n", (unsigned)k);
                ok = 0;
            }
        }
        free(a);
        free(b);
    }
    ok = ok && dump(argv[1], "f32.bin", f32, 3, N * sizeof(float));
    ok = ok && dump(argv[1], "f64.bin", f64, 3, N * sizeof(double));
    ok = ok && dump(argv[1], "plan.bin", pv, 3, total * sizeof(float));
    ok = ok && dump(argv[1], "grad.bin", &grad, 1, 2 * sizeof(double));
    ok = ok && dump(argv[1], "g.bin", g, 3, N * sizeof(float));
    ok = ok && kappa_ok(kappa_plan_destroy(plan), "kappa_plan_destroy");
    for (k = 0; k < 3; ++k) {
        hipFree(f32[k]);
        hipFree(f64[k]);
        hipFree(g[k]);
        hipFree(pv[k]);
        hipFree(pg[k]);
    }
    hipFree(grad);
    hipFree(ws);
    hipStreamDestroy(stream);
    if (!ok) return 1;
    printf("ok %llu plan particles\n", (unsigned long long)total);
    return 0;
}
