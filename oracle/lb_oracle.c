/* Plain FP64 CPU reference behind the library's C calling convention, with
 * HOST pointers: the same calls as liblb.so, computed by straightforward
 * loops over the lattice, one phase at a time.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product path links or loads
 * this library; it shares no code, tables or constants with the HIP
 * library or with the numpy reference (oracle/lb_oracle.py), and the tests
 * check the two references against each other.
 *
 * What is computed (the paper prints no formula; these are stated textbook
 * readings, as in the numpy reference):
 *  - D3Q19 velocities, rest first, then |c|^2 in {1, 2} in lexicographic
 *    order of (cx, cy, cz); weights 1/3, 1/18, 1/36; c_s^2 = 1/3.
 *  - Single fluid (Section IV's lattice-Boltzmann collision): BGK relaxation
 *    to f^eq_i = w_i rho [1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u].
 *  - Binary fluid (Section II-A: LB hydrodynamics coupled to a free-energy
 *    order parameter whose gradients are finite differences): phi = sum g,
 *    central-difference gradient and 7-point Laplacian (periodic),
 *    mu = A phi + B phi^3 - kappa lap phi, the chemical stress
 *    P_ab = [A/2 phi^2 + 3B/4 phi^4 - kappa phi lap - kappa/2 |grad|^2] delta
 *           + kappa d_a phi d_b phi
 *    in f^eq_i = w_i {rho E_i + 9/2 [c.P.c - tr P / 3]} and
 *    g^eq_i = w_i {phi E_i + 9/2 (Gamma mu - phi/3)(|c|^2 - 1)}, E_i the bracket
 *    above; f relaxes with tau_f, g with tau_g = mobility/Gamma + 1/2.
 *  - A step is collide, then propagate f_i(s + c_i) <- f*_i(s) (periodic).
 * Only LB_F64 storage and LB_BGK collision (other settings: LB_ENOTSUP), and
 * only the core calls (create, init, collide, propagate, step, moments,
 * conserved sums, get/set state, destroy).  Layout: canonical, distribution
 * i of site s = x + nx (y + ny z) at [i*N + s].
 *
 * Threads: built with OpenMP, the loops over sites (and over z planes in the
 * stencils and the propagation) are shared among threads.  Every value is
 * computed by the same expression whatever thread computes it, and the
 * conserved sums are taken serially in site order, so results do not depend
 * on the thread count (bitwise).  lb_oracle_set_threads chooses the count. */

#include <math.h>
#include <stddef.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* The library's C calling convention, declared here on its own (this file
 * includes nothing of the library): the parameter record, field for field
 * in the library's order, and the status and selector values it uses.
 * The tests compile the library header's README example against this file
 * and drive it through the same calls as the GPU library, which fails on
 * any layout mismatch. */
typedef struct lb_params {
    int32_t nx, ny, nz, model, storage, vvl, collision, binary_step;
    double tau_f, A, B, kappa, mobility, gamma, rho0, phi0;
    double tau_minus, tau_bulk, tau_ghost_even, tau_ghost_odd;
} lb_params;
typedef struct lb_ctx lb_ctx;

enum { LB_OK = 0, LB_EINVAL = -1, LB_ENOMEM = -2, LB_EDEVICE = -3, LB_ENOTSUP = -4 };
enum { LB_SINGLE = 0, LB_BINARY = 1 };
enum { LB_F64 = 0 };
enum { LB_BGK = 0 };
enum { LB_STEP_AUTO = 0, LB_STEP_TWO_PASS = 2 };

#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 19

/* Number of threads for the loops below (n <= 0: all the host offers);
 * returns the count that will be used.  Not part of lb.h. */
int lb_oracle_set_threads(int n) {
#ifdef _OPENMP
    if (n <= 0) n = omp_get_num_procs();
    omp_set_num_threads(n);
    return n;
#else
    (void)n;
    return 1;
#endif
}

static int CV[NQ][3];
static double WT[NQ];
static int tables_ready = 0;

static void make_tables(void) {
    if (tables_ready) return;
    int k = 0;
    CV[k][0] = CV[k][1] = CV[k][2] = 0;
    WT[k++] = 1.0 / 3.0;
    for (int x = -1; x <= 1; ++x)
        for (int y = -1; y <= 1; ++y)
            for (int z = -1; z <= 1; ++z) {
                const int c2 = x * x + y * y + z * z;
                if (c2 == 1 || c2 == 2) {
                    CV[k][0] = x; CV[k][1] = y; CV[k][2] = z;
                    WT[k++] = c2 == 1 ? 1.0 / 18.0 : 1.0 / 36.0;
                }
            }
    tables_ready = 1;
}

struct lb_ctx {
    lb_params p;
    size_t n;
    double *f, *g, *tmp;          /* state (19N each) and a propagation buffer */
    double *phi, *lap, *grad;     /* N, N, 3N */
};

static int bad_tau(double t) { return !(isfinite(t) && t > 0.5); }

static int check(const lb_params* p) {
    if (!p) return LB_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return LB_EINVAL;
    if ((int64_t)p->nx * p->ny * p->nz >= ((int64_t)1 << 29)) return LB_EINVAL;
    if (p->model != LB_SINGLE && p->model != LB_BINARY) return LB_EINVAL;
    if (p->binary_step < LB_STEP_AUTO || p->binary_step > LB_STEP_TWO_PASS || bad_tau(p->tau_f)) return LB_EINVAL;
    if (p->model == LB_BINARY &&
        (!isfinite(p->A) || !isfinite(p->B) || !(p->kappa >= 0.0) || !(p->mobility > 0.0) || !(p->gamma > 0.0)))
        return LB_EINVAL;
    if (p->storage != LB_F64 || p->collision != LB_BGK) return LB_ENOTSUP;
    return LB_OK;
}

static size_t sites(const lb_params* p) { return (size_t)p->nx * p->ny * p->nz; }

int lb_workspace_bytes(const lb_params* p, size_t* bytes) {
    int rc = check(p);
    if (rc) return rc;
    if (!bytes) return LB_EINVAL;
    *bytes = (3 * NQ + 5) * sites(p) * sizeof(double);
    return LB_OK;
}

int lb_create(const lb_params* p, void* workspace, size_t bytes, void* stream, lb_ctx** out) {
    (void)stream;
    if (!out) return LB_EINVAL;
    *out = NULL;
    size_t need = 0;
    int rc = lb_workspace_bytes(p, &need);
    if (rc) return rc;
    if (!workspace) return LB_EINVAL;
    if (bytes < need) return LB_ENOMEM;
    make_tables();
    lb_ctx* c = (lb_ctx*)malloc(sizeof(lb_ctx));
    if (!c) return LB_ENOMEM;
    c->p = *p;
    c->n = sites(p);
    double* w = (double*)workspace;
    c->f = w;
    c->g = w + NQ * c->n;
    c->tmp = w + 2 * NQ * c->n;
    c->phi = w + 3 * NQ * c->n;
    c->lap = c->phi + c->n;
    c->grad = c->lap + c->n;
    memset(workspace, 0, need);
    *out = c;
    return LB_OK;
}

int lb_set_stream(lb_ctx* c, void* stream) {
    (void)stream;
    return c ? LB_OK : LB_EINVAL;
}

int lb_destroy(lb_ctx* c) {
    free(c);
    return LB_OK;
}

const char* lb_strerror(int status) {
    switch (status) {
        case LB_OK: return "ok";
        case LB_EINVAL: return "invalid argument";
        case LB_ENOMEM: return "workspace too small";
        case LB_EDEVICE: return "device error";
        case LB_ENOTSUP: return "not supported by this reference";
    }
    return "unknown status";
}

/* a + d wrapped into [0, n), for a in [0, n) and d in {-1, 0, 1} */
static int wrap(int a, int d, int n) {
    a += d;
    return a < 0 ? a + n : (a >= n ? a - n : a);
}

/* index of (x + dx, y + dy, z + dz), periodic; dx, dy, dz in {-1, 0, 1} */
static size_t nb(const lb_params* p, int x, int y, int z, int dx, int dy, int dz) {
    x = wrap(x, dx, p->nx);
    y = wrap(y, dy, p->ny);
    z = wrap(z, dz, p->nz);
    return (size_t)x + (size_t)p->nx * ((size_t)y + (size_t)p->ny * z);
}

/* central-difference gradient and 7-point Laplacian of c->phi */
static void stencils(lb_ctx* c) {
    const lb_params* p = &c->p;
#pragma omp parallel for schedule(static)
    for (int z = 0; z < p->nz; ++z)
        for (int y = 0; y < p->ny; ++y)
            for (int x = 0; x < p->nx; ++x) {
                const size_t s = nb(p, x, y, z, 0, 0, 0);
                const double xm = c->phi[nb(p, x, y, z, -1, 0, 0)], xp = c->phi[nb(p, x, y, z, 1, 0, 0)];
                const double ym = c->phi[nb(p, x, y, z, 0, -1, 0)], yp = c->phi[nb(p, x, y, z, 0, 1, 0)];
                const double zm = c->phi[nb(p, x, y, z, 0, 0, -1)], zp = c->phi[nb(p, x, y, z, 0, 0, 1)];
                c->grad[s] = 0.5 * (xp - xm);
                c->grad[c->n + s] = 0.5 * (yp - ym);
                c->grad[2 * c->n + s] = 0.5 * (zp - zm);
                c->lap[s] = xm + xp + ym + yp + zm + zp - 6.0 * c->phi[s];
            }
}

/* phi = sum g, then its stencils */
static void phi_fields(lb_ctx* c, const double* g) {
#pragma omp parallel for schedule(static)
    for (size_t s = 0; s < c->n; ++s) {
        double a = 0.0;
        for (int i = 0; i < NQ; ++i) a += g[i * c->n + s];
        c->phi[s] = a;
    }
    stencils(c);
}

/* equilibria of one site; P (3x3) may be NULL (single fluid) */
static void equilibria(double rho, const double u[3], const double P[3][3], double phi, double mu,
                       const lb_params* p, double feq[NQ], double geq[NQ]) {
    const double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    const double trP = P ? P[0][0] + P[1][1] + P[2][2] : 0.0;
    for (int i = 0; i < NQ; ++i) {
        const double cu = CV[i][0] * u[0] + CV[i][1] * u[1] + CV[i][2] * u[2];
        const double E = 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * uu;
        double stress = 0.0;
        if (P) {
            double cPc = 0.0;
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) cPc += CV[i][a] * CV[i][b] * P[a][b];
            stress = 4.5 * (cPc - trP / 3.0);
        }
        feq[i] = WT[i] * (rho * E + stress);
        if (geq) {
            const int c2 = CV[i][0] * CV[i][0] + CV[i][1] * CV[i][1] + CV[i][2] * CV[i][2];
            geq[i] = WT[i] * (phi * E + 4.5 * (p->gamma * mu - phi / 3.0) * (c2 - 1));
        }
    }
}

static void stress_and_mu(const lb_ctx* c, size_t s, double P[3][3], double* mu) {
    const lb_params* p = &c->p;
    const double ph = c->phi[s], lp = c->lap[s];
    const double G[3] = {c->grad[s], c->grad[c->n + s], c->grad[2 * c->n + s]};
    const double GG = G[0] * G[0] + G[1] * G[1] + G[2] * G[2];
    const double iso = 0.5 * p->A * ph * ph + 0.75 * p->B * ph * ph * ph * ph - p->kappa * ph * lp - 0.5 * p->kappa * GG;
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) P[a][b] = p->kappa * G[a] * G[b] + (a == b ? iso : 0.0);
    *mu = p->A * ph + p->B * ph * ph * ph - p->kappa * lp;
}

static void moments_of(const double* f, size_t n, size_t s, double* rho, double u[3]) {
    double r = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int i = 0; i < NQ; ++i) {
        const double v = f[i * n + s];
        r += v;
        for (int a = 0; a < 3; ++a) j[a] += CV[i][a] * v;
    }
    *rho = r;
    for (int a = 0; a < 3; ++a) u[a] = j[a] / r;
}

int lb_init_equilibrium(lb_ctx* c, const double* rho, const double* u, const double* phi) {
    if (!c || !rho || !u) return LB_EINVAL;
    const int bin = c->p.model == LB_BINARY;
    if (bin != (phi != NULL)) return LB_EINVAL;
    if (bin) {
        memcpy(c->phi, phi, c->n * sizeof(double));
        stencils(c);
    }
#pragma omp parallel for schedule(static)
    for (size_t s = 0; s < c->n; ++s) {
        const double us[3] = {u[s], u[c->n + s], u[2 * c->n + s]};
        double feq[NQ], geq[NQ], P[3][3], mu = 0.0;
        if (bin) stress_and_mu(c, s, P, &mu);
        equilibria(rho[s], us, bin ? P : NULL, bin ? c->phi[s] : 0.0, mu, &c->p, feq, bin ? geq : NULL);
        for (int i = 0; i < NQ; ++i) {
            c->f[i * c->n + s] = feq[i];
            if (bin) c->g[i * c->n + s] = geq[i];
        }
    }
    return LB_OK;
}

int lb_collide(lb_ctx* c) {
    if (!c) return LB_EINVAL;
    const int bin = c->p.model == LB_BINARY;
    const double of = 1.0 / c->p.tau_f;
    const double og = 1.0 / (c->p.mobility / c->p.gamma + 0.5);
    if (bin) phi_fields(c, c->g);
#pragma omp parallel for schedule(static)
    for (size_t s = 0; s < c->n; ++s) {
        double rho, u[3], feq[NQ], geq[NQ], P[3][3], mu = 0.0;
        moments_of(c->f, c->n, s, &rho, u);
        if (bin) stress_and_mu(c, s, P, &mu);
        equilibria(rho, u, bin ? P : NULL, bin ? c->phi[s] : 0.0, mu, &c->p, feq, bin ? geq : NULL);
        for (int i = 0; i < NQ; ++i) {
            double* fi = &c->f[i * c->n + s];
            *fi = *fi - of * (*fi - feq[i]);
            if (bin) {
                double* gi = &c->g[i * c->n + s];
                *gi = *gi - og * (*gi - geq[i]);
            }
        }
    }
    return LB_OK;
}

static void stream_one(lb_ctx* c, double* a) {
    const lb_params* p = &c->p;
    for (int i = 0; i < NQ; ++i)
#pragma omp parallel for schedule(static)
        for (int z = 0; z < p->nz; ++z)
            for (int y = 0; y < p->ny; ++y)
                for (int x = 0; x < p->nx; ++x)
                    c->tmp[i * c->n + nb(p, x, y, z, CV[i][0], CV[i][1], CV[i][2])] =
                        a[i * c->n + nb(p, x, y, z, 0, 0, 0)];
    memcpy(a, c->tmp, NQ * c->n * sizeof(double));
}

int lb_propagate(lb_ctx* c) {
    if (!c) return LB_EINVAL;
    stream_one(c, c->f);
    if (c->p.model == LB_BINARY) stream_one(c, c->g);
    return LB_OK;
}

int lb_step(lb_ctx* c, int32_t nsteps) {
    if (!c || nsteps < 0) return LB_EINVAL;
    for (int32_t k = 0; k < nsteps; ++k) {
        lb_collide(c);
        lb_propagate(c);
    }
    return LB_OK;
}

int lb_moments(lb_ctx* c, double* rho, double* u, double* phi) {
    if (!c) return LB_EINVAL;
    if (phi && c->p.model != LB_BINARY) return LB_EINVAL;
#pragma omp parallel for schedule(static)
    for (size_t s = 0; s < c->n; ++s) {
        double r, us[3];
        moments_of(c->f, c->n, s, &r, us);
        if (rho) rho[s] = r;
        if (u)
            for (int a = 0; a < 3; ++a) u[a * c->n + s] = us[a];
        if (phi) {
            double a = 0.0;
            for (int i = 0; i < NQ; ++i) a += c->g[i * c->n + s];
            phi[s] = a;
        }
    }
    return LB_OK;
}

int lb_conserved_sums(lb_ctx* c, double* out) {
    if (!c || !out) return LB_EINVAL;
    for (int k = 0; k < 5; ++k) out[k] = 0.0;
    for (size_t s = 0; s < c->n; ++s)
        for (int i = 0; i < NQ; ++i) {
            const double v = c->f[i * c->n + s];
            out[0] += v;
            for (int a = 0; a < 3; ++a) out[1 + a] += CV[i][a] * v;
            if (c->p.model == LB_BINARY) out[4] += c->g[i * c->n + s];
        }
    return LB_OK;
}

int lb_get_state(lb_ctx* c, void* f, void* g) {
    if (!c || !f) return LB_EINVAL;
    if ((c->p.model == LB_BINARY) != (g != NULL)) return LB_EINVAL;
    memcpy(f, c->f, NQ * c->n * sizeof(double));
    if (g) memcpy(g, c->g, NQ * c->n * sizeof(double));
    return LB_OK;
}

int lb_set_state(lb_ctx* c, const void* f, const void* g) {
    if (!c || !f) return LB_EINVAL;
    if ((c->p.model == LB_BINARY) != (g != NULL)) return LB_EINVAL;
    memcpy(c->f, f, NQ * c->n * sizeof(double));
    if (g) memcpy(c->g, g, NQ * c->n * sizeof(double));
    return LB_OK;
}
