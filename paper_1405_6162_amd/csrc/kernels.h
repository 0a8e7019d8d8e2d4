// gfx950 kernels of the D3Q19 lattice-Boltzmann update.
//
// One lattice site per lane; every distribution is stored structure-of-arrays
// (direction-major, x fastest), so each of the 19 (binary: 38) direction
// streams is a coalesced HBM stream.  The update is bandwidth bound (well
// under one flop per byte), so there is no MFMA here: the design goal is to
// move each distribution value through HBM once per step.
//
// State convention.  A buffer either holds the state itself ("direct") or a
// post-collision field whose propagation is still pending; in the second
// case the pre-collision value at s in direction i is read from s - c_i
// (pull).  The fused step kernel reads a pending buffer with the pull
// gather, collides in registers and writes the post-collision values at s:
// one read and one write of every value per step.
#pragma once

#include "d3q19.h"

namespace lbk {

constexpr int MODEL_SINGLE = 0;
constexpr int MODEL_BINARY = 1;

template <class T>
struct CollParams {
    T omega_f, omega_g;        // 1/tau_f, 1/tau_g
    T A, B, kappa, gamma;      // free energy and mobility parameter
    T rho0, phi0;              // deviation references (0 for FP64 storage)
};

// ---------------------------------------------------------------------------
// Per-site physics shared by the collision kernels (compute type T).
// ---------------------------------------------------------------------------

// c_i . u for a compile-time direction.
template <int I, class T>
__device__ __forceinline__ T cdot(T ux, T uy, T uz) {
    T r = T(0);
    if constexpr (cx(I) > 0) r = r + ux;
    if constexpr (cx(I) < 0) r = r - ux;
    if constexpr (cy(I) > 0) r = r + uy;
    if constexpr (cy(I) < 0) r = r - uy;
    if constexpr (cz(I) > 0) r = r + uz;
    if constexpr (cz(I) < 0) r = r - uz;
    return r;
}

// Binary-fluid quantities at one site from phi, its gradient and Laplacian:
// mu = A phi + B phi^3 - kappa lap, and the two pieces of the chemical stress
// that enter the equilibrium, iso = A/2 phi^2 + 3B/4 phi^4 - kappa phi lap
// - kappa/2 |grad phi|^2 and kappa |grad phi|^2 / 3.
template <class T>
struct FreeEnergy {
    T phi, gx, gy, gz, mu, iso, k3;
    __device__ __forceinline__ FreeEnergy(T phi_, T gx_, T gy_, T gz_, T lap, const CollParams<T>& cp)
        : phi(phi_), gx(gx_), gy(gy_), gz(gz_) {
        const T phi2 = phi * phi;
        const T gsq = gx * gx + gy * gy + gz * gz;
        mu = cp.A * phi + cp.B * phi2 * phi - cp.kappa * lap;
        iso = T(0.5) * cp.A * phi2 + T(0.75) * cp.B * phi2 * phi2 - cp.kappa * phi * lap
              - T(0.5) * cp.kappa * gsq;
        k3 = cp.kappa * gsq / T(3);
    }
    // 9/2 [c_i.P.c_i - tr(P)/3] for direction I.
    template <int I>
    __device__ __forceinline__ T stress_term(const CollParams<T>& cp) const {
        const T cg = cdot<I>(gx, gy, gz);
        if constexpr (csq(I) == 0) return T(4.5) * (-iso - k3);
        else if constexpr (csq(I) == 1) return T(4.5) * (cp.kappa * cg * cg - k3);
        else return T(4.5) * (iso + cp.kappa * cg * cg - k3);
    }
    // 9/2 (gamma mu - phi/3)(|c_i|^2 - 1) for direction I.
    template <int I>
    __device__ __forceinline__ T mobility_term(const CollParams<T>& cp) const {
        if constexpr (csq(I) == 1) return T(0);
        else {
            const T m = T(4.5) * (cp.gamma * mu - phi / T(3));
            return csq(I) == 0 ? -m : m;
        }
    }
};

// ---------------------------------------------------------------------------
// Order parameter: phi(s) = phi0 + sum_i e_i, e = g - w phi0 (deviation).
// ---------------------------------------------------------------------------

template <class S, bool GATHER>
__global__ __launch_bounds__(TPB) void k_phi(const S* __restrict__ g, typename Compute<S>::T* __restrict__ phi,
                                             Geo geo, typename Compute<S>::T phi0) {
    using T = typename Compute<S>::T;
    const Site st = site_of_thread(geo);
    if (!st.active) return;
    T acc = T(0);
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        acc = acc + load_as<T>(g + i * geo.dstride + src_offset<i, GATHER>(st, geo));
    });
    phi[offset_at<0, 0, 0>(st, geo)] = phi0 + acc;
}

// ---------------------------------------------------------------------------
// Collision (GATHER = false: in place on a direct buffer) or fused pull-stream
// + collision (GATHER = true: pending src buffer -> direct dst buffer).
// The binary model stages the phi tile of this z plane (with a one-site halo
// in x and y) in LDS for the gradient and Laplacian; the two z neighbours are
// read straight from the phi field.
// ---------------------------------------------------------------------------

template <int MODEL, class S, bool GATHER>
__global__ __launch_bounds__(TPB) void k_collide(const S* fsrc, const S* gsrc, S* fdst, S* gdst,
                                                 const typename Compute<S>::T* __restrict__ phi, Geo geo,
                                                 CollParams<typename Compute<S>::T> cp) {
    using T = typename Compute<S>::T;
    const Site st = site_of_thread(geo);

    T phic = T(0), gx = T(0), gy = T(0), gz = T(0), lap = T(0);
    if constexpr (MODEL == MODEL_BINARY) {
        __shared__ T tile[TY + 2][TX + 2];
        const int x0 = (int)blockIdx.x * TX - 1;
        const int y0 = (int)blockIdx.y * TY - 1;
        const uint32_t zoff = (uint32_t)st.z * geo.plane;
        for (int k = threadIdx.y * TX + threadIdx.x; k < (TX + 2) * (TY + 2); k += TPB) {
            const int lx = k % (TX + 2), ly = k / (TX + 2);
            int xx = (x0 + lx) % geo.nx;
            int yy = (y0 + ly) % geo.ny;
            xx += xx < 0 ? geo.nx : 0;
            yy += yy < 0 ? geo.ny : 0;
            tile[ly][lx] = phi[zoff + (uint32_t)yy * (uint32_t)geo.nx + (uint32_t)xx];
        }
        __syncthreads();
        if (!st.active) return;
        const int lx = threadIdx.x + 1, ly = threadIdx.y + 1;
        phic = tile[ly][lx];
        const T pxm = tile[ly][lx - 1], pxp = tile[ly][lx + 1];
        const T pym = tile[ly - 1][lx], pyp = tile[ly + 1][lx];
        const T pzm = phi[offset_at<0, 0, -1>(st, geo)];
        const T pzp = phi[offset_at<0, 0, 1>(st, geo)];
        gx = T(0.5) * (pxp - pxm);
        gy = T(0.5) * (pyp - pym);
        gz = T(0.5) * (pzp - pzm);
        lap = (pxp + pxm) + (pyp + pym) + (pzp + pzm) - T(6) * phic;
    } else {
        if (!st.active) return;
    }

    const uint32_t off = offset_at<0, 0, 0>(st, geo);

    T f[Q];
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        f[i] = load_as<T>(fsrc + i * geo.dstride + src_offset<i, GATHER>(st, geo));
    });
    T g[Q];
    if constexpr (MODEL == MODEL_BINARY) {
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            g[i] = load_as<T>(gsrc + i * geo.dstride + src_offset<i, GATHER>(st, geo));
        });
    }

    // Moments (deviation form: rho = rho0 + sum d_i, j = sum d_i c_i).
    T drho = T(0), jx = T(0), jy = T(0), jz = T(0);
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        drho = drho + f[i];
        if constexpr (cx(i) > 0) jx = jx + f[i];
        if constexpr (cx(i) < 0) jx = jx - f[i];
        if constexpr (cy(i) > 0) jy = jy + f[i];
        if constexpr (cy(i) < 0) jy = jy - f[i];
        if constexpr (cz(i) > 0) jz = jz + f[i];
        if constexpr (cz(i) < 0) jz = jz - f[i];
    });
    const T rho = cp.rho0 + drho;
    const T ux = jx / rho, uy = jy / rho, uz = jz / rho;
    const T usq = ux * ux + uy * uy + uz * uz;

    if constexpr (MODEL == MODEL_BINARY) {
        const FreeEnergy<T> fe(phic, gx, gy, gz, lap, cp);
        const T dphi = phic - cp.phi0;
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const T cu = cdot<i>(ux, uy, uz);
            const T base = T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq;
            const T feq = weight<T>(i) * (drho + rho * base + fe.template stress_term<i>(cp));
            const T geq = weight<T>(i) * (dphi + phic * base + fe.template mobility_term<i>(cp));
            store_as(fdst + i * geo.dstride + off, f[i] - cp.omega_f * (f[i] - feq));
            store_as(gdst + i * geo.dstride + off, g[i] - cp.omega_g * (g[i] - geq));
        });
    } else {
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const T cu = cdot<i>(ux, uy, uz);
            const T base = T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq;
            const T feq = weight<T>(i) * (drho + rho * base);
            store_as(fdst + i * geo.dstride + off, f[i] - cp.omega_f * (f[i] - feq));
        });
    }
}

// ---------------------------------------------------------------------------
// Stand-alone propagation (pull): dst_i(s) = src_i(s - c_i).  Also used to
// materialise a pending buffer into caller memory of another stride.
// ---------------------------------------------------------------------------

template <class S>
__global__ __launch_bounds__(TPB) void k_stream(const S* __restrict__ src, S* __restrict__ dst, Geo geo,
                                                int64_t dst_stride) {
    const Site st = site_of_thread(geo);
    if (!st.active) return;
    const uint32_t off = offset_at<0, 0, 0>(st, geo);
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        dst[i * dst_stride + off] = src[i * geo.dstride + src_offset<i, true>(st, geo)];
    });
}

// ---------------------------------------------------------------------------
// Equilibrium initialisation (FP64 arithmetic, stored in S as deviations).
// ---------------------------------------------------------------------------

template <int MODEL, class S>
__global__ __launch_bounds__(TPB) void k_init(const double* __restrict__ rho_in, const double* __restrict__ u_in,
                                              const double* __restrict__ phi_in, S* __restrict__ f,
                                              S* __restrict__ g, Geo geo, CollParams<double> cp) {
    const Site st = site_of_thread(geo);
    if (!st.active) return;
    const uint32_t off = offset_at<0, 0, 0>(st, geo);
    const double rho = rho_in[off];
    const double ux = u_in[off], uy = u_in[geo.nsite + off], uz = u_in[2 * (size_t)geo.nsite + off];
    const double usq = ux * ux + uy * uy + uz * uz;
    const double drho = rho - cp.rho0;
    if constexpr (MODEL == MODEL_BINARY) {
        const double p = phi_in[off];
        const double pxm = phi_in[offset_at<-1, 0, 0>(st, geo)], pxp = phi_in[offset_at<1, 0, 0>(st, geo)];
        const double pym = phi_in[offset_at<0, -1, 0>(st, geo)], pyp = phi_in[offset_at<0, 1, 0>(st, geo)];
        const double pzm = phi_in[offset_at<0, 0, -1>(st, geo)], pzp = phi_in[offset_at<0, 0, 1>(st, geo)];
        const double lap = (pxp + pxm) + (pyp + pym) + (pzp + pzm) - 6.0 * p;
        const FreeEnergy<double> fe(p, 0.5 * (pxp - pxm), 0.5 * (pyp - pym), 0.5 * (pzp - pzm), lap, cp);
        const double dphi = p - cp.phi0;
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double cu = cdot<i>(ux, uy, uz);
            const double base = 3.0 * cu + 4.5 * cu * cu - 1.5 * usq;
            store_as(f + i * geo.dstride + off, weight<double>(i) * (drho + rho * base + fe.template stress_term<i>(cp)));
            store_as(g + i * geo.dstride + off, weight<double>(i) * (dphi + p * base + fe.template mobility_term<i>(cp)));
        });
    } else {
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double cu = cdot<i>(ux, uy, uz);
            const double base = 3.0 * cu + 4.5 * cu * cu - 1.5 * usq;
            store_as(f + i * geo.dstride + off, weight<double>(i) * (drho + rho * base));
        });
    }
}

// ---------------------------------------------------------------------------
// Moments of the current state in FP64 (pending buffers are read by pull).
// ---------------------------------------------------------------------------

template <int MODEL, class S, bool GATHER>
__global__ __launch_bounds__(TPB) void k_moments(const S* __restrict__ f, const S* __restrict__ g,
                                                 double* __restrict__ rho_out, double* __restrict__ u_out,
                                                 double* __restrict__ phi_out, Geo geo, double rho0, double phi0) {
    const Site st = site_of_thread(geo);
    if (!st.active) return;
    const uint32_t off = offset_at<0, 0, 0>(st, geo);
    double drho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const double v = load_as<double>(f + i * geo.dstride + src_offset<i, GATHER>(st, geo));
        drho = drho + v;
        if constexpr (cx(i) > 0) jx = jx + v;
        if constexpr (cx(i) < 0) jx = jx - v;
        if constexpr (cy(i) > 0) jy = jy + v;
        if constexpr (cy(i) < 0) jy = jy - v;
        if constexpr (cz(i) > 0) jz = jz + v;
        if constexpr (cz(i) < 0) jz = jz - v;
    });
    const double rho = rho0 + drho;
    if (rho_out) rho_out[off] = rho;
    if (u_out) {
        u_out[off] = jx / rho;
        u_out[geo.nsite + off] = jy / rho;
        u_out[2 * (size_t)geo.nsite + off] = jz / rho;
    }
    if constexpr (MODEL == MODEL_BINARY) {
        if (phi_out) {
            double acc = 0.0;
            static_for<0, Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                acc = acc + load_as<double>(g + i * geo.dstride + src_offset<i, GATHER>(st, geo));
            });
            phi_out[off] = phi0 + acc;
        }
    }
}

// ---------------------------------------------------------------------------
// Deterministic reductions: per-block tree in LDS, then one block summing the
// block partials in index order.
// ---------------------------------------------------------------------------

__device__ __forceinline__ int block_linear() {
    return (int)(blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z));
}

// Tree sum over the block of K values per thread, in a fixed order; on return
// sh[k][0] holds the block total of value k (visible to every thread).
template <int K>
__device__ __forceinline__ void block_tree_sum(const double (&v)[K], double (*sh)[TPB]) {
    const int t = threadIdx.y * TX + threadIdx.x;
#pragma unroll
    for (int k = 0; k < K; ++k) sh[k][t] = v[k];
    __syncthreads();
    for (int half = TPB / 2; half > 0; half >>= 1) {
        if (t < half) {
#pragma unroll
            for (int k = 0; k < K; ++k) sh[k][t] = sh[k][t] + sh[k][t + half];
        }
        __syncthreads();
    }
}

// Local sums of the stored values (streaming permutes values, so the sums of
// a pending buffer equal those of the state it stands for, up to the order
// of the additions).
template <int MODEL, class S>
__global__ __launch_bounds__(TPB) void k_sums_partial(const S* __restrict__ f, const S* __restrict__ g, Geo geo,
                                                      double* __restrict__ partial) {
    __shared__ double sh[5][TPB];
    const Site st = site_of_thread(geo);
    double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    if (st.active) {
        const uint32_t off = offset_at<0, 0, 0>(st, geo);
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double a = load_as<double>(f + i * geo.dstride + off);
            v[0] = v[0] + a;
            if constexpr (cx(i) != 0) v[1] = v[1] + cx(i) * a;
            if constexpr (cy(i) != 0) v[2] = v[2] + cy(i) * a;
            if constexpr (cz(i) != 0) v[3] = v[3] + cz(i) * a;
            if constexpr (MODEL == MODEL_BINARY) v[4] = v[4] + load_as<double>(g + i * geo.dstride + off);
        });
    }
    block_tree_sum<5>(v, sh);
    const int t = threadIdx.y * TX + threadIdx.x;
    if (t < 5) partial[8 * (size_t)block_linear() + t] = sh[t][0];
}

// out[k] = base[k] + sum_b partial[8 b + k], k < K; one block of TPB threads.
template <int K>
__global__ __launch_bounds__(TPB) void k_sums_final(const double* __restrict__ partial, int nblocks, double* out,
                                                    double base0, double base4, int accumulate) {
    __shared__ double sh[K][TPB];
    const int t = threadIdx.y * TX + threadIdx.x;
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = 0.0;
    for (int b = t; b < nblocks; b += TPB) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = v[k] + partial[8 * (size_t)b + k];
    }
    block_tree_sum<K>(v, sh);
    if (t == 0) {
        for (int k = 0; k < K; ++k) {
            double r = sh[k][0];
            if (k == 0) r = base0 + r;
            if (k == 4) r = base4 + r;
            out[k] = accumulate ? out[k] + r : r;
        }
    }
}

// ---------------------------------------------------------------------------
// Adjoint of one single-fluid FP64 step (canonical layout, stride N).
// lambda*_i(s) = lambda^{n+1}_i(s + c_i) is the transpose of the pull.
// ---------------------------------------------------------------------------

__global__ __launch_bounds__(TPB) void k_adjoint(const double* __restrict__ fn, const double* __restrict__ lam_next,
                                                 double* __restrict__ lam_n, double* __restrict__ partial, Geo geo,
                                                 double omega) {
    __shared__ double sh[1][TPB];
    const Site st = site_of_thread(geo);
    double dw[1] = {0.0};
    if (st.active) {
        const uint32_t off = offset_at<0, 0, 0>(st, geo);
        double f[Q], ls[Q];
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            f[i] = fn[i * geo.dstride + off];
            ls[i] = lam_next[i * geo.dstride + offset_at<cx(i), cy(i), cz(i)>(st, geo)];
        });
        double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0;
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            rho = rho + f[i];
            if constexpr (cx(i) > 0) jx = jx + f[i];
            if constexpr (cx(i) < 0) jx = jx - f[i];
            if constexpr (cy(i) > 0) jy = jy + f[i];
            if constexpr (cy(i) < 0) jy = jy - f[i];
            if constexpr (cz(i) > 0) jz = jz + f[i];
            if constexpr (cz(i) < 0) jz = jz - f[i];
        });
        const double ux = jx / rho, uy = jy / rho, uz = jz / rho;
        const double usq = ux * ux + uy * uy + uz * uz;
        // S = sum_i lambda*_i f^eq_i / rho = sum_i lambda*_i w_i E_i;
        // T_a = rho sum_i lambda*_i w_i (3 c_ia + 9 (c_i.u) c_ia - 3 u_a).
        double Ssum = 0.0, lw = 0.0, tx = 0.0, ty = 0.0, tz = 0.0, dom = 0.0;
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double cu = cdot<i>(ux, uy, uz);
            const double E = 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq;
            const double lwi = ls[i] * weight<double>(i);
            Ssum = Ssum + lwi * E;
            lw = lw + lwi;
            const double h = lwi * (3.0 + 9.0 * cu);
            if constexpr (cx(i) > 0) tx = tx + h;
            if constexpr (cx(i) < 0) tx = tx - h;
            if constexpr (cy(i) > 0) ty = ty + h;
            if constexpr (cy(i) < 0) ty = ty - h;
            if constexpr (cz(i) > 0) tz = tz + h;
            if constexpr (cz(i) < 0) tz = tz - h;
            dom = dom + ls[i] * (weight<double>(i) * rho * E - f[i]);
        });
        // T_a / rho = tx - 3 u_a lw
        const double Tx = tx - 3.0 * ux * lw, Ty = ty - 3.0 * uy * lw, Tz = tz - 3.0 * uz * lw;
        const double TU = Tx * ux + Ty * uy + Tz * uz;
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double tc = cdot<i>(Tx, Ty, Tz);
            lam_n[i * geo.dstride + off] = (1.0 - omega) * ls[i] + omega * (Ssum + tc - TU);
        });
        dw[0] = dom;
    }
    block_tree_sum<1>(dw, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0) partial[8 * (size_t)block_linear()] = sh[0][0];
}

}  // namespace lbk
