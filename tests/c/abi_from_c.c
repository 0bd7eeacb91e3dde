/* The C ABI used from plain C99 (no HIP headers): the header compiles on its
 * own, the library links, and calls that need no GPU behave as documented. */
#include <math.h>
#include <stdio.h>
#include <string.h>

#include "kappa.h"

static int failures = 0;

static void expect(int cond, const char *what)
{
    if (!cond) {
        printf("FAIL %s\n", what);
        ++failures;
    }
}

int main(void)
{
    double p[KAPPA_NPARAMS];
    expect(kappa_params(3.0, p) == KAPPA_OK, "kappa_params(3)");
    expect(fabs(p[KAPPA_P_KSTAR] - 2.5) < 1e-15, "kappa* = kappa - 1/2");
    expect(kappa_params(1.5, p) == KAPPA_EINVAL, "kappa = 3/2 rejected");
    expect(kappa_params(INFINITY, p) == KAPPA_OK && p[KAPPA_P_C] == 0.079, "Maxwell limit");
    expect(strncmp(kappa_status_string(KAPPA_ERANGE), "KAPPA_ERANGE", 12) == 0, "status string");
    expect(kappa_sample(3.0, 1.0, 0, 0, 0, 0, KAPPA_FP32, NULL, NULL, NULL, NULL) == KAPPA_OK, "n = 0 is a no-op");
    expect(kappa_sample(3.0, -1.0, 10, 0, 0, 0, KAPPA_FP32, NULL, NULL, NULL, NULL) == KAPPA_EINVAL,
           "theta <= 0 rejected");
    expect(kappa_last_error()[0] != '\0', "last error set");
    kappa_segment seg = {3.0, 1.0, {0.0, 0.0, 0.0}, 10, 0, 0};
    kappa_plan plan = NULL;
    expect(kappa_plan_create(&seg, 0, 1, KAPPA_FP32, &plan) == KAPPA_ERANGE, "empty segment table rejected");
    expect(kappa_plan_destroy(NULL) == KAPPA_OK, "destroy(NULL)");
    expect(kappa_backward_workspace_bytes(1u << 20) % 256 == 0, "workspace size is a multiple of 256");
    printf("%s %s\n", failures ? "FAILED" : "ok", kappa_version());
    return failures != 0;
}
