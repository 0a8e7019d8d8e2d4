/* Plain-C use of liblb (include/lb.h): a binary-fluid spinodal quench on a
 * small periodic lattice, driven without Python.  Device memory and the
 * stream come from the HIP runtime's C API; the library itself only takes
 * pointers and sizes.
 *
 *   lb_example NX NY NZ STEPS OUT
 *
 * The initial fields are rho = 1, u = 0 and
 * phi = 0.05 sin(2 pi (x/nx + 2 y/ny)) cos(2 pi 3 z/nz) (FP64).  After STEPS
 * steps the program writes rho[N], u[3N] and phi[N] (canonical layout, FP64,
 * native byte order) to the file OUT, prints the conserved sums before and
 * after, and exits 0 if mass and sum phi are conserved to rounding, every
 * value is finite and the library refuses a bad parameter set. */

#include <math.h>
#include <stdio.h>
#include <stdlib.h>

#include <hip/hip_runtime_api.h>

#include "lb.h"

#define HIP_OK(call)                                                              \
    do {                                                                          \
        hipError_t e_ = (call);                                                   \
        if (e_ != hipSuccess) {                                                   \
            fprintf(stderr, "HIP error %s at line %d\n", hipGetErrorString(e_), __LINE__); \
            return 2;                                                             \
        }                                                                         \
    } while (0)

#define LB_OK_(call)                                                              \
    do {                                                                          \
        int s_ = (call);                                                          \
        if (s_ != LB_OK) {                                                        \
            fprintf(stderr, "%s failed: %s\n", #call, lb_strerror(s_));           \
            return 3;                                                             \
        }                                                                         \
    } while (0)

int main(int argc, char** argv) {
    if (argc != 6) {
        fprintf(stderr, "usage: %s NX NY NZ STEPS OUT\n", argv[0]);
        return 1;
    }
    const int nx = atoi(argv[1]), ny = atoi(argv[2]), nz = atoi(argv[3]), steps = atoi(argv[4]);
    const size_t n = (size_t)nx * ny * nz;

    lb_params p = {0};
    p.nx = nx; p.ny = ny; p.nz = nz;
    p.model = LB_BINARY; p.storage = LB_F64; p.vvl = 1; p.collision = LB_BGK;
    p.tau_f = 1.0; p.A = -0.0625; p.B = 0.0625; p.kappa = 0.04; p.mobility = 0.45; p.gamma = 1.0;
    p.rho0 = 1.0; p.phi0 = 0.0; p.tau_minus = 1.0; p.tau_bulk = 1.0; p.tau_ghost_even = 1.0; p.tau_ghost_odd = 1.0;

    /* the library checks what it is given */
    lb_params bad = p;
    bad.tau_f = 0.5;
    size_t bytes = 0;
    if (lb_workspace_bytes(&bad, &bytes) != LB_EINVAL) {
        fprintf(stderr, "tau_f = 0.5 was accepted\n");
        return 4;
    }
    LB_OK_(lb_workspace_bytes(&p, &bytes));

    hipStream_t stream;
    HIP_OK(hipStreamCreate(&stream));
    void* ws = NULL;
    HIP_OK(hipMalloc(&ws, bytes));
    lb_ctx* ctx = NULL;
    LB_OK_(lb_create(&p, ws, bytes, (void*)stream, &ctx));

    double* h = (double*)malloc(5 * n * sizeof(double));   /* rho, u (3), phi */
    if (!h) return 5;
    const double two_pi = 6.283185307179586;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                const size_t s = (size_t)x + (size_t)nx * ((size_t)y + (size_t)ny * z);
                h[s] = 1.0;
                h[n + s] = h[2 * n + s] = h[3 * n + s] = 0.0;
                h[4 * n + s] = 0.05 * sin(two_pi * ((double)x / nx + 2.0 * y / ny)) * cos(two_pi * 3.0 * z / nz);
            }
    double* d = NULL;      /* rho | u | phi | sums (5) */
    HIP_OK(hipMalloc((void**)&d, (5 * n + 5) * sizeof(double)));
    HIP_OK(hipMemcpy(d, h, 5 * n * sizeof(double), hipMemcpyHostToDevice));
    double* rho = d;
    double* u = d + n;
    double* phi = d + 4 * n;
    double* sums = d + 5 * n;

    double s0[5], s1[5];
    LB_OK_(lb_init_equilibrium(ctx, rho, u, phi));
    LB_OK_(lb_conserved_sums(ctx, sums));
    HIP_OK(hipMemcpyAsync(s0, sums, sizeof s0, hipMemcpyDeviceToHost, stream));
    LB_OK_(lb_step(ctx, steps));
    LB_OK_(lb_conserved_sums(ctx, sums));
    HIP_OK(hipMemcpyAsync(s1, sums, sizeof s1, hipMemcpyDeviceToHost, stream));
    LB_OK_(lb_moments(ctx, rho, u, phi));
    HIP_OK(hipMemcpyAsync(h, d, 5 * n * sizeof(double), hipMemcpyDeviceToHost, stream));
    HIP_OK(hipStreamSynchronize(stream));

    int ok = 1;
    for (size_t k = 0; k < 5 * n; ++k) ok &= isfinite(h[k]) != 0;
    ok &= fabs(s1[0] - s0[0]) <= 1e-12 * fabs(s0[0]);
    ok &= fabs(s1[4] - s0[4]) <= 1e-12 * (double)n;
    printf("mass %.17g -> %.17g  sum phi %.17g -> %.17g  %s\n", s0[0], s1[0], s0[4], s1[4], ok ? "ok" : "FAILED");

    FILE* out = fopen(argv[5], "wb");
    if (!out || fwrite(h, sizeof(double), 5 * n, out) != 5 * n) return 6;
    fclose(out);

    LB_OK_(lb_destroy(ctx));
    HIP_OK(hipFree(d));
    HIP_OK(hipFree(ws));
    HIP_OK(hipStreamDestroy(stream));
    free(h);
    return ok ? 0 : 7;
}
