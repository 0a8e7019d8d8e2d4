/* Drives every call of the C reference (oracle/lb_oracle.c) on small
 * lattices, including its argument checks, for a build with
 * -fsanitize=address,undefined: any out-of-bounds access, use of freed
 * memory, leak or undefined behaviour ends the run with an error.
 * Test infrastructure only.  Exit status 0 when every call returned what
 * the header promises and the conserved sums held. */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include "lb.h"

int lb_oracle_set_threads(int n);

static int failures = 0;
#define EXPECT(cond)                                                     \
    do {                                                                 \
        if (!(cond)) {                                                   \
            fprintf(stderr, "%s:%d: %s\n", __FILE__, __LINE__, #cond);   \
            ++failures;                                                  \
        }                                                                \
    } while (0)

static lb_params params(int nx, int ny, int nz, int model) {
    lb_params p = {.nx = nx, .ny = ny, .nz = nz, .model = model, .storage = LB_F64, .collision = LB_BGK,
                   .tau_f = 0.9, .A = -0.0625, .B = 0.0625, .kappa = 0.04, .mobility = 0.45, .gamma = 1.0,
                   .rho0 = 1.0};
    return p;
}

static void run(int nx, int ny, int nz, int model) {
    lb_params p = params(nx, ny, nz, model);
    size_t bytes = 0;
    EXPECT(lb_workspace_bytes(&p, &bytes) == LB_OK && bytes > 0);
    void* ws = malloc(bytes);
    lb_ctx* c = NULL;
    EXPECT(lb_create(&p, ws, bytes - 8, NULL, &c) == LB_ENOMEM && c == NULL);
    EXPECT(lb_create(&p, NULL, bytes, NULL, &c) == LB_EINVAL);
    EXPECT(lb_create(&p, ws, bytes, NULL, &c) == LB_OK && c != NULL);
    EXPECT(lb_set_stream(c, NULL) == LB_OK);
    const size_t n = (size_t)nx * ny * nz;
    double* rho = malloc(n * sizeof(double));
    double* u = malloc(3 * n * sizeof(double));
    double* phi = malloc(n * sizeof(double));
    for (size_t s = 0; s < n; ++s) {
        rho[s] = 1.0 + 0.01 * sin(0.7 * (double)s);
        for (int a = 0; a < 3; ++a) u[a * n + s] = 0.01 * cos(0.3 * (double)(s + 5 * a));
        phi[s] = 0.05 * sin(1.3 * (double)s);
    }
    const int bin = model == LB_BINARY;
    EXPECT(lb_init_equilibrium(c, rho, u, bin ? NULL : phi) == LB_EINVAL);
    EXPECT(lb_init_equilibrium(c, rho, u, bin ? phi : NULL) == LB_OK);
    double s0[5], s1[5];
    EXPECT(lb_conserved_sums(c, s0) == LB_OK);
    EXPECT(lb_collide(c) == LB_OK);
    EXPECT(lb_propagate(c) == LB_OK);
    EXPECT(lb_step(c, -1) == LB_EINVAL);
    EXPECT(lb_step(c, 0) == LB_OK);
    EXPECT(lb_step(c, 3) == LB_OK);
    EXPECT(lb_conserved_sums(c, s1) == LB_OK);
    for (int k = 0; k < 5; ++k) EXPECT(fabs(s1[k] - s0[k]) <= 1e-12 * (1.0 + fabs(s0[k])));
    EXPECT(lb_moments(c, rho, u, bin ? phi : NULL) == LB_OK);
    if (!bin) EXPECT(lb_moments(c, rho, u, phi) == LB_EINVAL);
    double* f = malloc(19 * n * sizeof(double));
    double* g = malloc(19 * n * sizeof(double));
    EXPECT(lb_get_state(c, f, bin ? g : NULL) == LB_OK);
    EXPECT(lb_get_state(c, f, bin ? NULL : g) == LB_EINVAL);
    EXPECT(lb_set_state(c, f, bin ? g : NULL) == LB_OK);
    EXPECT(lb_get_state(NULL, f, NULL) == LB_EINVAL);
    EXPECT(lb_destroy(c) == LB_OK);
    free(f);
    free(g);
    free(rho);
    free(u);
    free(phi);
    free(ws);
}

int main(void) {
    lb_params bad = params(0, 4, 4, LB_SINGLE);
    size_t bytes = 0;
    EXPECT(lb_workspace_bytes(&bad, &bytes) == LB_EINVAL);
    bad = params(4, 4, 4, LB_BINARY);
    bad.tau_f = 0.5;
    EXPECT(lb_workspace_bytes(&bad, &bytes) == LB_EINVAL);
    bad = params(4, 4, 4, LB_BINARY);
    bad.collision = LB_TRT;
    EXPECT(lb_workspace_bytes(&bad, &bytes) == LB_ENOTSUP);
    EXPECT(lb_workspace_bytes(NULL, &bytes) == LB_EINVAL);
    EXPECT(lb_destroy(NULL) == LB_OK);
    EXPECT(lb_strerror(LB_EINVAL) != NULL && lb_strerror(12345) != NULL);
    for (int threads = 1; threads <= 2; ++threads) {
        lb_oracle_set_threads(threads);
        run(5, 4, 3, LB_SINGLE);
        run(5, 4, 3, LB_BINARY);
        run(1, 1, 2, LB_BINARY);
        run(7, 1, 1, LB_SINGLE);
    }
    if (failures) fprintf(stderr, "%d check(s) failed\n", failures);
    return failures ? 1 : 0;
}
