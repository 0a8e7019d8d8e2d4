// gfx950 kernels of the D3Q19 lattice-Boltzmann update.
//
// Every distribution is stored structure-of-arrays (direction-major, x
// fastest; the paper's lattice-field layout, Section III-B), and each lane
// updates TZ sites of one (x, y) column, so each of the 19 (binary: 38)
// direction streams is a coalesced HBM stream.  The update is bandwidth
// bound (well under one flop per byte), so there is no MFMA here: the design
// goal is to move each distribution value through HBM once per step.
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

// Collision of f: BGK, two-relaxation-time, or multiple-relaxation-time.
constexpr int COLL_BGK = 0;
constexpr int COLL_TRT = 1;
constexpr int COLL_MRT = 2;

template <class T>
struct CollParams {
    T omega_f, omega_g;        // 1/tau_f, 1/tau_g
    T A, B, kappa, gamma;      // free energy and mobility parameter
    T rho0, phi0;              // deviation references (0 for FP64 storage)
    T omega_m;                 // 1/tau_minus: odd part (TRT), energy flux (MRT)
    T omega_b, omega_ge, omega_go;   // MRT: energy (bulk), even ghosts, odd ghosts
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

// Load the 19 populations of one site (pulled from s - c_i when GATHER) from
// direction arrays `stride` elements apart (default: the lattice's own).
template <class P, bool GATHER, class S, class T>
__device__ __forceinline__ void load_site(const S* src, const Site& st, const Geo& geo, T (&v)[Q],
                                          int64_t stride = -1) {
    const int64_t ds = stride < 0 ? geo.dstride : stride;
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        v[i] = static_cast<T>(ldg<P::nt_load>(src + i * ds, src_offset<i, GATHER>(st, geo)));
    });
}

// Density deviation and momentum of 19 populations (deviation form:
// rho = rho0 + sum d_i, j = sum d_i c_i), summed in A, returned in T.
template <class A, class T>
__device__ __forceinline__ void moments_in(const T (&f)[Q], T& drho, T& jx, T& jy, T& jz) {
    A r = A(0), x = A(0), y = A(0), z = A(0);
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const A v = static_cast<A>(f[i]);
        r = r + v;
        if constexpr (cx(i) > 0) x = x + v;
        if constexpr (cx(i) < 0) x = x - v;
        if constexpr (cy(i) > 0) y = y + v;
        if constexpr (cy(i) < 0) y = y - v;
        if constexpr (cz(i) > 0) z = z + v;
        if constexpr (cz(i) < 0) z = z - v;
    });
    drho = static_cast<T>(r); jx = static_cast<T>(x); jy = static_cast<T>(y); jz = static_cast<T>(z);
}

template <class T>
__device__ __forceinline__ void moments_of(const T (&f)[Q], T& drho, T& jx, T& jy, T& jz) {
    moments_in<T>(f, drho, jx, jy, jz);
}

// phi = phi0 + sum_i e_i of 19 values already in registers, summed in A.
template <class A, class T>
__device__ __forceinline__ T phi_sum(const T (&e)[Q], T phi0) {
    A acc = A(0);
#pragma unroll
    for (int i = 0; i < Q; ++i) acc = acc + static_cast<A>(e[i]);
    return static_cast<T>(static_cast<A>(phi0) + acc);
}

// ---------------------------------------------------------------------------
// Order parameter: phi(s) = phi0 + sum_i e_i, e = g - w phi0 (deviation).
// ---------------------------------------------------------------------------

template <class P, class S, bool GATHER>
__global__ __launch_bounds__(P::TPB) void k_phi(const S* __restrict__ g, typename Compute<S>::T* __restrict__ phi,
                                                Geo geo, typename Compute<S>::T phi0) {
    using T = typename Compute<S>::T;
    const Column col = column_of_thread<P>(geo);
#pragma unroll
    for (int v = 0; v < P::TZ; ++v) {
        const Site st = site_at(col, v, geo);
        if (!st.active) continue;
        using A = typename Accum<S>::T;
        A acc = A(0);
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            acc = acc + static_cast<A>(static_cast<T>(ldg<P::nt_load>(g + i * geo.dstride, src_offset<i, GATHER>(st, geo))));
        });
        phi[canon_at<0, 0, 0>(st, geo)] = static_cast<T>(static_cast<A>(phi0) + acc);
    }
}

// ---------------------------------------------------------------------------
// Collision (GATHER = false: in place on a direct buffer) or fused pull-stream
// + collision (GATHER = true: pending src buffer -> direct dst buffer).
// The binary model stages the phi tile of the block (TX x TY x TZ sites plus
// a one-site halo on every side) in LDS; the gradient and Laplacian read
// their six neighbours from there.
// ---------------------------------------------------------------------------

// TRT: the parts of f - f^eq even and odd under c -> -c relax with omega_f
// and omega_m.  MRT: TRT for the shear stresses (even) and the energy fluxes
// (odd), and seven more moments of the orthogonal basis with their own rates
// -- the energy e (omega_b), the even ghosts eps, pi_xx, pi_ww (omega_ge) and
// the odd ghosts m_x, m_y, m_z (omega_go) -- applied as a correction
// (omega_k - its TRT rate) times the moment's projection.  neq = f - f^eq.
template <class P, int COLL, class S, class T>
__device__ __forceinline__ void relax_moments_store(const T (&f)[Q], const T (&neq)[Q], S* fdst, uint32_t off,
                                                    int64_t ds, const CollParams<T>& cp) {
    T a[7] = {T(0), T(0), T(0), T(0), T(0), T(0), T(0)};
    if constexpr (COLL == COLL_MRT) {
        static_for<0, 7>([&](auto K) {
            constexpr int k = decltype(K)::value;
            constexpr int m = mrt_extra(k);
            T acc = T(0);
            static_for<0, Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int c = mrt_poly(m, i);
                if constexpr (c != 0) acc = acc + T(c) * neq[i];
            });
            // k = 0: e (bulk); 1-3: eps, pi_xx, pi_ww (even ghosts); 4-6: m (odd ghosts)
            const T dw = k == 0 ? cp.omega_b - cp.omega_f : (k < 4 ? cp.omega_ge - cp.omega_f : cp.omega_go - cp.omega_m);
            a[k] = dw * acc / T(mrt_norm(m));
        });
    }
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        constexpr int o = opp(i);
        T corr = T(0);
        if constexpr (COLL == COLL_MRT) {
            static_for<0, 7>([&](auto K) {
                constexpr int k = decltype(K)::value;
                constexpr int c = mrt_poly(mrt_extra(k), i);
                if constexpr (c != 0) corr = corr + T(c) * a[k];
            });
        }
        const T np = T(0.5) * (neq[i] + neq[o]);
        const T nm = T(0.5) * (neq[i] - neq[o]);
        stg<P::nt_store>(fdst + i * ds, off, static_cast<S>(f[i] - cp.omega_f * np - cp.omega_m * nm - corr));
    });
}

template <class P, int COLL = COLL_BGK, class S, class T>
__device__ __forceinline__ void relax_single(const T (&f)[Q], S* fdst, uint32_t off, const Geo& geo,
                                             const CollParams<T>& cp, int64_t stride = -1) {
    const int64_t ds = stride < 0 ? geo.dstride : stride;
    T drho, jx, jy, jz;
    moments_in<typename Accum<S>::T>(f, drho, jx, jy, jz);
    const T rho = cp.rho0 + drho;
    const T ux = jx / rho, uy = jy / rho, uz = jz / rho;
    const T usq = ux * ux + uy * uy + uz * uz;
    if constexpr (COLL != COLL_BGK) {
        T neq[Q];
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const T cu = cdot<i>(ux, uy, uz);
            neq[i] = f[i] - weight<T>(i) * (drho + rho * (T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq));
        });
        relax_moments_store<P, COLL>(f, neq, fdst, off, ds, cp);
    } else {
        // every post-collision value before the first store (measured 1.3%
        // faster than storing each as it is computed)
        T out[Q];
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const T cu = cdot<i>(ux, uy, uz);
            const T base = T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq;
            const T feq = weight<T>(i) * (drho + rho * base);
            out[i] = f[i] - cp.omega_f * (f[i] - feq);
        });
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            stg<P::nt_store>(fdst + i * ds, off, static_cast<S>(out[i]));
        });
    }
}

// Binary collision of one site: g relaxes with omega_g (BGK); f with BGK, or
// with TRT / MRT around the same f^eq (relax_moments_store).
template <class P, int COLL = COLL_BGK, class S, class T>
__device__ __forceinline__ void relax_binary(const T (&f)[Q], const T (&g)[Q], S* fdst, S* gdst, uint32_t off,
                                             const Geo& geo, const CollParams<T>& cp, T phic, T gx, T gy, T gz,
                                             T lap) {
    T drho, jx, jy, jz;
    moments_in<typename Accum<S>::T>(f, drho, jx, jy, jz);
    const T rho = cp.rho0 + drho;
    const T ux = jx / rho, uy = jy / rho, uz = jz / rho;
    const T usq = ux * ux + uy * uy + uz * uz;
    const FreeEnergy<T> fe(phic, gx, gy, gz, lap, cp);
    const T dphi = phic - cp.phi0;
    if constexpr (COLL != COLL_BGK) {
        T neq[Q];
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const T cu = cdot<i>(ux, uy, uz);
            const T base = T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq;
            neq[i] = f[i] - weight<T>(i) * (drho + rho * base + fe.template stress_term<i>(cp));
            const T geq = weight<T>(i) * (dphi + phic * base + fe.template mobility_term<i>(cp));
            stg<P::nt_store>(gdst + i * geo.dstride, off, static_cast<S>(g[i] - cp.omega_g * (g[i] - geq)));
        });
        relax_moments_store<P, COLL>(f, neq, fdst, off, geo.dstride, cp);
        return;
    }
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const T cu = cdot<i>(ux, uy, uz);
        const T base = T(3) * cu + T(4.5) * cu * cu - T(1.5) * usq;
        const T feq = weight<T>(i) * (drho + rho * base + fe.template stress_term<i>(cp));
        const T geq = weight<T>(i) * (dphi + phic * base + fe.template mobility_term<i>(cp));
        stg<P::nt_store>(fdst + i * geo.dstride, off, static_cast<S>(f[i] - cp.omega_f * (f[i] - feq)));
        stg<P::nt_store>(gdst + i * geo.dstride, off, static_cast<S>(g[i] - cp.omega_g * (g[i] - geq)));
    });
}

template <class P, int MODEL, class S, bool GATHER, int COLL = COLL_BGK>
__global__ __launch_bounds__(P::TPB) void k_collide(const S* fsrc, const S* gsrc, S* fdst, S* gdst,
                                                    const typename Compute<S>::T* __restrict__ phi, Geo geo,
                                                    CollParams<typename Compute<S>::T> cp) {
    using T = typename Compute<S>::T;
    const Column col = column_of_thread<P>(geo);
    if constexpr (MODEL == MODEL_BINARY) {
        constexpr int TX = P::TX, TY = P::TY, TZ = P::TZ;
        constexpr int LX = TX + 2, LY = TY + 2, LZ = TZ + 2;
        __shared__ T tile[LZ][LY][LX];
        for (int k = threadIdx.x; k < LX * LY * LZ; k += P::TPB) {
            const int lx = k % LX, ly = (k / LX) % LY, lz = k / (LX * LY);
            int xx = (col.x0 - 1 + lx) % geo.nx;
            int yy = (col.y0 - 1 + ly) % geo.ny;
            int zz = (col.z0 - 1 + lz) % geo.nz;
            xx += xx < 0 ? geo.nx : 0;
            yy += yy < 0 ? geo.ny : 0;
            zz += zz < 0 ? geo.nz : 0;
            tile[lz][ly][lx] = phi[(uint32_t)zz * geo.plane + (uint32_t)yy * (uint32_t)geo.nx + (uint32_t)xx];
        }
        __syncthreads();
        const int lx = col.x - col.x0 + 1, ly = col.y - col.y0 + 1;
#pragma unroll
        for (int v = 0; v < TZ; ++v) {
            const Site st = site_at(col, v, geo);
            if (!st.active) continue;
            const int lz = v + 1;
            const T phic = tile[lz][ly][lx];
            const T pxm = tile[lz][ly][lx - 1], pxp = tile[lz][ly][lx + 1];
            const T pym = tile[lz][ly - 1][lx], pyp = tile[lz][ly + 1][lx];
            const T pzm = tile[lz - 1][ly][lx], pzp = tile[lz + 1][ly][lx];
            const T gx = T(0.5) * (pxp - pxm);
            const T gy = T(0.5) * (pyp - pym);
            const T gz = T(0.5) * (pzp - pzm);
            const T lap = (pxp + pxm) + (pyp + pym) + (pzp + pzm) - T(6) * phic;
            T f[Q], g[Q];
            load_site<P, GATHER>(fsrc, st, geo, f);
            load_site<P, GATHER>(gsrc, st, geo, g);
            relax_binary<P, COLL>(f, g, fdst, gdst, offset_at<0, 0, 0>(st, geo), geo, cp, phic, gx, gy, gz, lap);
        }
    } else {
#pragma unroll
        for (int v = 0; v < P::TZ; ++v) {
            const Site st = site_at(col, v, geo);
            if (!st.active) continue;
            T f[Q];
            load_site<P, GATHER>(fsrc, st, geo, f);
            relax_single<P, COLL>(f, fdst, offset_at<0, 0, 0>(st, geo), geo, cp);
        }
    }
}

// Single-fluid collision from an array of one layout (geo) into an array of
// another (dgeo), used to record each step's post-collision field into
// canonical caller memory.
template <class P, class S, bool GATHER, int COLL = COLL_BGK>
__global__ __launch_bounds__(P::TPB) void k_collide_single_strided(const S* fsrc, S* fdst, Geo geo, Geo dgeo,
                                                                   CollParams<typename Compute<S>::T> cp) {
    using T = typename Compute<S>::T;
    const Column col = column_of_thread<P>(geo);
#pragma unroll
    for (int v = 0; v < P::TZ; ++v) {
        const Site st = site_at(col, v, geo);
        if (!st.active) continue;
        T f[Q];
        load_site<P, GATHER>(fsrc, st, geo, f);
        relax_single<P, COLL>(f, fdst, offset_at<0, 0, 0>(st, dgeo), dgeo, cp);
    }
}

// ---------------------------------------------------------------------------
// Single-pass binary step: fused pull-stream + collision that computes phi
// itself.  A block owns a TX x TY column tile and marches through one chunk
// of at most geo.bz consecutive z planes (geo.gz chunks).  phi(s) = phi0 + sum_i e_i(s - c_i) needs the pulled
// g of s, which the collision of s needs anyway: each lane gathers g for
// plane z+1, sums it into the plane's phi tile in LDS and keeps the 19 values
// for the next plane's collision, in registers or (GLDS) in LDS.  On small
// lattices the host picks the two-pass step instead, because a few blocks
// walking their planes in sequence cannot hide the per-plane latency.
// The x/y halo ring of the
// tile (2 TX + 2 TY sites per plane) is summed by one lane each from its own
// gather; the chunk's first and last plane need one extra plane of phi each.
// Three phi planes (z-1, z, z+1) rotate in LDS.  Lanes outside the lattice
// (ragged tiles) compute phi at the periodic image of their coordinates so
// that every LDS slot holds the value its neighbours read.  The summation
// order of phi is the same as in k_phi, so results equal the two-pass path.
// ---------------------------------------------------------------------------

// Site at wrapped coordinates (x, y in range), plane z.
__device__ __forceinline__ Site site_wrapped(int x, int y, int z, const Geo& g) {
    Site s;
    s.x = x; s.y = y; s.z = z;
    s.xm = x == 0 ? g.nx - 1 : x - 1;
    s.xp = x + 1 >= g.nx ? 0 : x + 1;
    s.ym = y == 0 ? g.ny - 1 : y - 1;
    s.yp = y + 1 >= g.ny ? 0 : y + 1;
    s.zm = z == 0 ? g.nz - 1 : z - 1;
    s.zp = z + 1 >= g.nz ? 0 : z + 1;
    s.active = true;
    return s;
}

__device__ __forceinline__ int wrap_plane(int z, int nz) {
    return z < 0 ? z + nz : (z >= nz ? z - nz : z);
}

// phi of the pulled g at st: the 19 values are loaded into registers first
// and then summed (in k_phi's order), so the loads go out as one batch
// rather than one at a time behind the running sum.
template <class P, class S, class T>
__device__ __forceinline__ T phi_of_gathered(const S* g, const Site& st, const Geo& geo, T phi0) {
    T v[Q];
    load_site<P, true>(g, st, geo, v);
    return phi_sum<typename Accum<S>::T>(v, phi0);
}

// With GLDS the 19 pulled g of the next plane wait in LDS (each lane only
// touches its own slots, so no barrier is involved) instead of registers,
// which lowers register pressure and raises occupancy.  RING is the number of
// phi planes kept in LDS: with 3 a second barrier per plane keeps the write of
// plane z+2 from overtaking the reads of plane z-1; with 4 the slot written
// next is never one still being read, so one barrier per plane suffices.
// With PHI_OUT the kernel also stores the phi it computes for its own sites
// (phi_out[s], canonical), i.e. phi of the state this step collides.
// BLK: the arrays are in the blocked layout, whose direction stride (64
// elements) is then a compile-time constant: every direction of a site is
// one address plus an immediate offset, and a site's loads need one 64-bit
// address instead of one per direction.
template <class P, class S, bool GLDS, int RING = 3, bool PHI_OUT = false, int COLL = COLL_BGK, bool BLK = false>
__global__ __launch_bounds__(P::TPB) void k_binary_march(const S* __restrict__ fsrc, const S* __restrict__ gsrc,
                                                         S* __restrict__ fdst, S* __restrict__ gdst, Geo geo_in,
                                                         CollParams<typename Compute<S>::T> cp,
                                                         typename Compute<S>::T* __restrict__ phi_out = nullptr) {
    using T = typename Compute<S>::T;
    Geo geo = geo_in;
    if constexpr (BLK) geo.dstride = 64;
    constexpr int TX = P::TX, TY = P::TY, LX = TX + 2, LY = TY + 2;
    constexpr int NHALO = 2 * TX + 2 * TY;
    static_assert(NHALO <= P::TPB, "one halo site per lane");
    static_assert(RING == 3 || RING == 4, "3 or 4 phi planes");
    __shared__ T ring[RING][LY][LX];
    __shared__ T gkeep[GLDS ? Q : 1][GLDS ? P::TPB : 1];

    const int b = tile_index<P>(geo);
    const int bx = b % geo.gx;
    const int t = b / geo.gx;
    const int by = t % geo.gy;
    // Under the XCD remap each XCD takes a contiguous run of tiles, so a short
    // last chunk would land on the last XCDs and leave them idle while the
    // others finish: the gz chunks then split nz evenly (8-14% faster at 208^3
    // with 64-plane chunks).  Without the remap blocks reach the XCDs in launch
    // order and the short last chunk, launched last, fills the tail (even
    // chunks measured 5-6% slower at 272^3).
    const int zc = t / geo.gy;
    int z0, z1;
    if (xcd_remapped<P>(geo)) {
        z0 = (int)((int64_t)zc * geo.nz / geo.gz);
        z1 = (int)((int64_t)(zc + 1) * geo.nz / geo.gz);
    } else {
        z0 = zc * geo.bz;
        z1 = min(z0 + geo.bz, geo.nz);
    }
    const int x0 = bx * TX, y0 = by * TY;
    const int tx = (int)(threadIdx.x % TX), ty = (int)(threadIdx.x / TX);
    const bool active = (x0 + tx < geo.nx) && (y0 + ty < geo.ny);
    const int xw = (x0 + tx) % geo.nx, yw = (y0 + ty) % geo.ny;

    // This lane's halo site (if any): LDS slot (hlx, hly) of the ring, taken
    // in order (the y-halo rows land on whole wavefronts, so their gathers are
    // contiguous; measured faster than spreading the ring over all
    // wavefronts).
    const int k = threadIdx.x;
    int hlx = 0, hly = 0;
    if (k < TX) { hlx = k + 1; hly = 0; }
    else if (k < 2 * TX) { hlx = k - TX + 1; hly = TY + 1; }
    else if (k < 2 * TX + TY) { hlx = 0; hly = k - 2 * TX + 1; }
    else if (k < NHALO) { hlx = TX + 1; hly = k - 2 * TX - TY + 1; }
    const bool has_halo = k < NHALO;
    int hx = (x0 - 1 + hlx) % geo.nx, hy = (y0 - 1 + hly) % geo.ny;
    hx += hx < 0 ? geo.nx : 0;
    hy += hy < 0 ? geo.ny : 0;

    const int lx = tx + 1, ly = ty + 1;
    auto slot = [&](int z) { return (z - z0 + RING) % RING; };

    // Prologue: phi of planes z0-1 and z0; g of plane z0 kept for its collision.
    T gc[Q];
    {
        const int zm = wrap_plane(z0 - 1, geo.nz);
        ring[slot(z0 - 1)][ly][lx] = phi_of_gathered<P>(gsrc, site_wrapped(xw, yw, zm, geo), geo, cp.phi0);
        if (has_halo)
            ring[slot(z0 - 1)][hly][hlx] = phi_of_gathered<P>(gsrc, site_wrapped(hx, hy, zm, geo), geo, cp.phi0);
        const Site s0 = site_wrapped(xw, yw, z0, geo);
        load_site<P, true>(gsrc, s0, geo, gc);
        ring[slot(z0)][ly][lx] = phi_sum<typename Accum<S>::T>(gc, cp.phi0);
        if constexpr (PHI_OUT)
            if (active) phi_out[canon_at<0, 0, 0>(s0, geo)] = ring[slot(z0)][ly][lx];
        if constexpr (GLDS) {
#pragma unroll
            for (int i = 0; i < Q; ++i) gkeep[i][threadIdx.x] = gc[i];
        }
        if (has_halo)
            ring[slot(z0)][hly][hlx] = phi_of_gathered<P>(gsrc, site_wrapped(hx, hy, z0, geo), geo, cp.phi0);
    }

    for (int z = z0; z < z1; ++z) {
        const int zn = wrap_plane(z + 1, geo.nz);
        const Site sc = site_wrapped(xw, yw, z, geo);
        // every lane loads (a lane outside a ragged tile reads the periodic
        // image of its coordinates, valid memory it never stores), so these
        // loads share one basic block, and one wait, with the g loads below
        T fc[Q];
        load_site<P, true>(fsrc, sc, geo, fc);
        T gn[Q];
        load_site<P, true>(gsrc, site_wrapped(xw, yw, zn, geo), geo, gn);
        ring[slot(z + 1)][ly][lx] = phi_sum<typename Accum<S>::T>(gn, cp.phi0);
        if constexpr (PHI_OUT)
            if (active && z + 1 < z1) phi_out[canon_at<0, 0, 0>(site_wrapped(xw, yw, zn, geo), geo)] =
                ring[slot(z + 1)][ly][lx];
        if (has_halo)
            ring[slot(z + 1)][hly][hlx] = phi_of_gathered<P>(gsrc, site_wrapped(hx, hy, zn, geo), geo, cp.phi0);
        if constexpr (GLDS) {
            // swap this plane's g out of LDS and park the next plane's
#pragma unroll
            for (int i = 0; i < Q; ++i) {
                gc[i] = gkeep[i][threadIdx.x];
                gkeep[i][threadIdx.x] = gn[i];
            }
        }
        __syncthreads();
        if (active) {
            const int r = slot(z);
            const T phic = ring[r][ly][lx];
            const T pxm = ring[r][ly][lx - 1], pxp = ring[r][ly][lx + 1];
            const T pym = ring[r][ly - 1][lx], pyp = ring[r][ly + 1][lx];
            const T pzm = ring[slot(z - 1)][ly][lx], pzp = ring[slot(z + 1)][ly][lx];
            const T gx = T(0.5) * (pxp - pxm);
            const T gy = T(0.5) * (pyp - pym);
            const T gz = T(0.5) * (pzp - pzm);
            const T lap = (pxp + pxm) + (pyp + pym) + (pzp + pzm) - T(6) * phic;
            relax_binary<P, COLL>(fc, gc, fdst, gdst, offset_at<0, 0, 0>(sc, geo), geo, cp, phic, gx, gy, gz, lap);
        }
        if constexpr (!GLDS) {
#pragma unroll
            for (int i = 0; i < Q; ++i) gc[i] = gn[i];
        }
        if constexpr (RING == 3) __syncthreads();
    }
}

// ---------------------------------------------------------------------------
// Stand-alone propagation (pull, GATHER): dst_i(s) = src_i(s - c_i), or a
// plain copy (no GATHER): dst_i(s) = src_i(s).  The source is addressed with
// geo's layout and the destination with dgeo's, so the same kernels move a
// state between the context's layout and canonical caller memory.
// ---------------------------------------------------------------------------

template <class P, class S, bool GATHER = true>
__global__ __launch_bounds__(P::TPB) void k_stream(const S* __restrict__ src, S* __restrict__ dst, Geo geo,
                                                   Geo dgeo) {
    const Column col = column_of_thread<P>(geo);
#pragma unroll
    for (int v = 0; v < P::TZ; ++v) {
        const Site st = site_at(col, v, geo);
        if (!st.active) continue;
        const uint32_t off = offset_at<0, 0, 0>(st, dgeo);
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            stg<P::nt_store>(dst + i * dgeo.dstride, off,
                             ldg<P::nt_load>(src + i * geo.dstride, src_offset<i, GATHER>(st, geo)));
        });
    }
}

// Both distributions of the binary fluid in one launch: 38 pulls and 38
// stores per site, the memory traffic of the binary step without its
// arithmetic (what the step's access pattern can reach on this memory
// system), and one launch instead of two for lb_propagate.
template <class P, class S, bool GATHER = true>
__global__ __launch_bounds__(P::TPB) void k_stream2(const S* __restrict__ fsrc, const S* __restrict__ gsrc,
                                                    S* __restrict__ fdst, S* __restrict__ gdst, Geo geo,
                                                    Geo dgeo) {
    const Column col = column_of_thread<P>(geo);
#pragma unroll
    for (int v = 0; v < P::TZ; ++v) {
        const Site st = site_at(col, v, geo);
        if (!st.active) continue;
        const uint32_t off = offset_at<0, 0, 0>(st, dgeo);
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const uint32_t up = src_offset<i, GATHER>(st, geo);
            const S fv = ldg<P::nt_load>(fsrc + i * geo.dstride, up);
            const S gv = ldg<P::nt_load>(gsrc + i * geo.dstride, up);
            stg<P::nt_store>(fdst + i * dgeo.dstride, off, fv);
            stg<P::nt_store>(gdst + i * dgeo.dstride, off, gv);
        });
    }
}

// ---------------------------------------------------------------------------
// Equilibrium initialisation (FP64 arithmetic, stored in S as deviations).
// ---------------------------------------------------------------------------

template <class P, int MODEL, class S>
__global__ __launch_bounds__(P::TPB) void k_init(const double* __restrict__ rho_in, const double* __restrict__ u_in,
                                                 const double* __restrict__ phi_in, S* __restrict__ f,
                                                 S* __restrict__ g, Geo geo, CollParams<double> cp) {
    const Column col = column_of_thread<P>(geo);
    for (int v = 0; v < P::TZ; ++v) {
        const Site st = site_at(col, v, geo);
        if (!st.active) continue;
        const uint32_t off = offset_at<0, 0, 0>(st, geo);
        const uint32_t sc = canon_at<0, 0, 0>(st, geo);
        const double rho = rho_in[sc];
        const double ux = u_in[sc], uy = u_in[geo.nsite + sc], uz = u_in[2 * (size_t)geo.nsite + sc];
        const double usq = ux * ux + uy * uy + uz * uz;
        const double drho = rho - cp.rho0;
        if constexpr (MODEL == MODEL_BINARY) {
            const double p = phi_in[sc];
            const double pxm = phi_in[canon_at<-1, 0, 0>(st, geo)], pxp = phi_in[canon_at<1, 0, 0>(st, geo)];
            const double pym = phi_in[canon_at<0, -1, 0>(st, geo)], pyp = phi_in[canon_at<0, 1, 0>(st, geo)];
            const double pzm = phi_in[canon_at<0, 0, -1>(st, geo)], pzp = phi_in[canon_at<0, 0, 1>(st, geo)];
            const double lap = (pxp + pxm) + (pyp + pym) + (pzp + pzm) - 6.0 * p;
            const FreeEnergy<double> fe(p, 0.5 * (pxp - pxm), 0.5 * (pyp - pym), 0.5 * (pzp - pzm), lap, cp);
            const double dphi = p - cp.phi0;
            static_for<0, Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                const double cu = cdot<i>(ux, uy, uz);
                const double base = 3.0 * cu + 4.5 * cu * cu - 1.5 * usq;
                *at(f + i * geo.dstride, off) =
                    static_cast<S>(weight<double>(i) * (drho + rho * base + fe.template stress_term<i>(cp)));
                *at(g + i * geo.dstride, off) =
                    static_cast<S>(weight<double>(i) * (dphi + p * base + fe.template mobility_term<i>(cp)));
            });
        } else {
            static_for<0, Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                const double cu = cdot<i>(ux, uy, uz);
                const double base = 3.0 * cu + 4.5 * cu * cu - 1.5 * usq;
                *at(f + i * geo.dstride, off) = static_cast<S>(weight<double>(i) * (drho + rho * base));
            });
        }
    }
}

// ---------------------------------------------------------------------------
// Moments of the current state in FP64 (pending buffers are read by pull).
// ---------------------------------------------------------------------------

template <class P, int MODEL, class S, bool GATHER>
__global__ __launch_bounds__(P::TPB) void k_moments(const S* __restrict__ f, const S* __restrict__ g,
                                                    double* __restrict__ rho_out, double* __restrict__ u_out,
                                                    double* __restrict__ phi_out, Geo geo, double rho0,
                                                    double phi0) {
    const Column col = column_of_thread<P>(geo);
    for (int v = 0; v < P::TZ; ++v) {
        const Site st = site_at(col, v, geo);
        if (!st.active) continue;
        const uint32_t off = canon_at<0, 0, 0>(st, geo);
        double fv[Q];
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            fv[i] = static_cast<double>(*at(f + i * geo.dstride, src_offset<i, GATHER>(st, geo)));
        });
        double drho, jx, jy, jz;
        moments_of(fv, drho, jx, jy, jz);
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
                    acc = acc + static_cast<double>(*at(g + i * geo.dstride, src_offset<i, GATHER>(st, geo)));
                });
                phi_out[off] = phi0 + acc;
            }
        }
    }
}

// ---------------------------------------------------------------------------
// Deterministic reductions: per-block tree in LDS, then one block summing the
// block partials in index order.
// ---------------------------------------------------------------------------

// Tree sum over the block of K values per thread, in a fixed order; on return
// sh[k][0] holds the block total of value k (visible to every thread).
template <int TPB, int K>
__device__ __forceinline__ void block_tree_sum(const double (&v)[K], double (*sh)[TPB]) {
    const int t = threadIdx.x;
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
template <class P, int MODEL, class S>
__global__ __launch_bounds__(P::TPB) void k_sums_partial(const S* __restrict__ f, const S* __restrict__ g, Geo geo,
                                                         double* __restrict__ partial) {
    __shared__ double sh[5][P::TPB];
    const Column col = column_of_thread<P>(geo);
    double v5[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
    for (int v = 0; v < P::TZ; ++v) {
        const Site st = site_at(col, v, geo);
        if (!st.active) continue;
        const uint32_t off = offset_at<0, 0, 0>(st, geo);
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double a = static_cast<double>(*at(f + i * geo.dstride, off));
            v5[0] = v5[0] + a;
            if constexpr (cx(i) != 0) v5[1] = v5[1] + cx(i) * a;
            if constexpr (cy(i) != 0) v5[2] = v5[2] + cy(i) * a;
            if constexpr (cz(i) != 0) v5[3] = v5[3] + cz(i) * a;
            if constexpr (MODEL == MODEL_BINARY) v5[4] = v5[4] + static_cast<double>(*at(g + i * geo.dstride, off));
        });
    }
    block_tree_sum<P::TPB, 5>(v5, sh);
    const int t = threadIdx.x;
    if (t < 5) partial[8 * (size_t)blockIdx.x + t] = sh[t][0];
}

// out[k] = base[k] + sum_b partial[8 b + k], k < K; one block of P::TPB threads.
template <int TPB, int K>
__device__ __forceinline__ void final_sums(const double* __restrict__ partial, int nblocks, double* out,
                                           double base0, double base4, int accumulate) {
    __shared__ double sh[K][TPB];
    const int t = threadIdx.x;
    double v[K];
#pragma unroll
    for (int k = 0; k < K; ++k) v[k] = 0.0;
    for (int b = t; b < nblocks; b += TPB) {
#pragma unroll
        for (int k = 0; k < K; ++k) v[k] = v[k] + partial[8 * (size_t)b + k];
    }
    block_tree_sum<TPB, K>(v, sh);
    if (t == 0) {
        for (int k = 0; k < K; ++k) {
            double r = sh[k][0];
            if (k == 0) r = base0 + r;
            if (k == 4) r = base4 + r;
            out[k] = accumulate ? out[k] + r : r;
        }
    }
}

template <class P, int K>
__global__ __launch_bounds__(P::TPB) void k_sums_final(const double* __restrict__ partial, int nblocks, double* out,
                                                       double base0, double base4, int accumulate) {
    final_sums<P::TPB, K>(partial, nblocks, out, base0, base4, accumulate);
}

// ---------------------------------------------------------------------------
// Field statistics of the current state (device reductions, fixed order):
// 0 sum rho, 1-3 sum j, 4 sum phi, 5 sum rho u.u, 6 min phi, 7 max phi,
// 8 sum phi^2, 9 max u.u.  Sums per block by an LDS tree, then one block over
// the block partials in index order; min and max likewise.
// ---------------------------------------------------------------------------

constexpr int NSTAT = 10;

template <int TPB>
__device__ __forceinline__ void block_tree_stats(double (&v)[NSTAT], double (*sh)[TPB]) {
    const int t = threadIdx.x;
#pragma unroll
    for (int k = 0; k < NSTAT; ++k) sh[k][t] = v[k];
    __syncthreads();
    for (int half = TPB / 2; half > 0; half >>= 1) {
        if (t < half) {
#pragma unroll
            for (int k = 0; k < NSTAT; ++k) {
                const double a = sh[k][t], b = sh[k][t + half];
                sh[k][t] = k == 6 ? fmin(a, b) : (k == 7 || k == 9 ? fmax(a, b) : a + b);
            }
        }
        __syncthreads();
    }
}

template <class P, int MODEL, class S, bool GATHER>
__global__ __launch_bounds__(P::TPB) void k_stats_partial(const S* __restrict__ f, const S* __restrict__ g, Geo geo,
                                                          double rho0, double phi0, double* __restrict__ partial) {
    __shared__ double sh[NSTAT][P::TPB];
    const Column col = column_of_thread<P>(geo);
    double v[NSTAT] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, INFINITY, -INFINITY, 0.0, 0.0};
    for (int z = 0; z < P::TZ; ++z) {
        const Site st = site_at(col, z, geo);
        if (!st.active) continue;
        double fv[Q];
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            fv[i] = static_cast<double>(*at(f + i * geo.dstride, src_offset<i, GATHER>(st, geo)));
        });
        double drho, jx, jy, jz;
        moments_of(fv, drho, jx, jy, jz);
        const double rho = rho0 + drho;
        const double uu = (jx * jx + jy * jy + jz * jz) / (rho * rho);
        v[0] += rho; v[1] += jx; v[2] += jy; v[3] += jz;
        v[5] += rho * uu;
        v[9] = fmax(v[9], uu);
        if constexpr (MODEL == MODEL_BINARY) {
            double acc = 0.0;
            static_for<0, Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                acc = acc + static_cast<double>(*at(g + i * geo.dstride, src_offset<i, GATHER>(st, geo)));
            });
            const double phi = phi0 + acc;
            v[4] += phi;
            v[6] = fmin(v[6], phi);
            v[7] = fmax(v[7], phi);
            v[8] += phi * phi;
        }
    }
    block_tree_stats<P::TPB>(v, sh);
    if ((int)threadIdx.x < NSTAT) partial[16 * (size_t)blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

template <class P>
__global__ __launch_bounds__(P::TPB) void k_stats_final(const double* __restrict__ partial, int nblocks,
                                                        double* __restrict__ out, int binary) {
    __shared__ double sh[NSTAT][P::TPB];
    const int t = threadIdx.x;
    double v[NSTAT] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, INFINITY, -INFINITY, 0.0, 0.0};
    for (int b = t; b < nblocks; b += P::TPB) {
        const double* q = partial + 16 * (size_t)b;
#pragma unroll
        for (int k = 0; k < NSTAT; ++k)
            v[k] = k == 6 ? fmin(v[k], q[k]) : (k == 7 || k == 9 ? fmax(v[k], q[k]) : v[k] + q[k]);
    }
    block_tree_stats<P::TPB>(v, sh);
    if (t == 0) {
        for (int k = 0; k < NSTAT; ++k) out[k] = sh[k][0];
        if (!binary) { out[4] = 0.0; out[6] = 0.0; out[7] = 0.0; out[8] = 0.0; }
    }
}

// ---------------------------------------------------------------------------
// Adjoint of one single-fluid FP64 step (canonical layout, stride N).
// lambda*_i(s) = lambda^{n+1}_i(s + c_i) is the transpose of the pull.
// ---------------------------------------------------------------------------

// F_PENDING: fn holds the post-collision field of step n-1 and f^n is pulled
// from it (f^n_i(s) = fn_i(s - c_i)); otherwise fn is f^n itself.
//
// Every collision is f* = f - Omega (f - f^eq(f)) with a constant symmetric
// Omega: omega I (BGK), omega_f P+ + omega_m P- (TRT, P+- the projections on
// the parts even and odd under c -> -c), and for MRT that plus
// (omega_k - its TRT rate) times the projection on each of the seven moments
// with their own rates (M^-1 = M^T D^-1 for the orthogonal basis, so every
// such projection is symmetric).  The transpose of the collision Jacobian
// I - Omega (I - J), J = d f^eq / d f, then gives, with mu = Omega lambda*,
//   lambda^n_j = lambda*_j - mu_j + S + sum_a T_a (c_ja - u_a),
//   S = sum_i mu_i w_i E_i,  T_a = sum_i mu_i w_i (3 c_ia + 9 (c_i.u) c_ia - 3 u_a),
// and dL/domega_k = sum_s (P_k lambda*).(f^eq - f) for each rate group k.
// K (the number of rate sums) is 1 for BGK, 2 for TRT (omega_f, omega_m)
// and 5 for MRT (shear, energy flux, energy, even ghosts, odd ghosts); they
// go to partial[8 b + k].  With prev_partial given, block 0 also adds the
// previous step's block partials (prev_nblocks of them, in block order) into
// sums[0..K): a sweep over several steps alternates two partial arrays and
// saves one reduction launch per step.
template <int COLL> struct AdjointRates { static constexpr int K = COLL == COLL_MRT ? 5 : (COLL == COLL_TRT ? 2 : 1); };

template <class P, bool F_PENDING, int COLL = COLL_BGK>
__global__ __launch_bounds__(P::TPB) void k_adjoint(const double* __restrict__ fn, const double* __restrict__ lam_next,
                                                    double* __restrict__ lam_n, double* __restrict__ partial, Geo geo,
                                                    CollParams<double> cp,
                                                    const double* __restrict__ prev_partial = nullptr,
                                                    int prev_nblocks = 0, double* sums = nullptr) {
    constexpr int K = AdjointRates<COLL>::K;
    __shared__ double sh[K][P::TPB];
    const Column col = column_of_thread<P>(geo);
    double dw[K];
    for (int k = 0; k < K; ++k) dw[k] = 0.0;
    for (int v = 0; v < P::TZ; ++v) {
        const Site st = site_at(col, v, geo);
        if (!st.active) continue;
        const uint32_t off = offset_at<0, 0, 0>(st, geo);
        double f[Q], ls[Q];
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            f[i] = *at(fn + i * geo.dstride, src_offset<i, F_PENDING>(st, geo));
            ls[i] = *at(lam_next + i * geo.dstride, offset_at<cx(i), cy(i), cz(i)>(st, geo));
        });
        double rho, jx, jy, jz;
        moments_of(f, rho, jx, jy, jz);
        const double ux = jx / rho, uy = jy / rho, uz = jz / rho;
        const double usq = ux * ux + uy * uy + uz * uz;
        if constexpr (COLL == COLL_BGK) {
            const double omega = cp.omega_f;
            // S = sum_i lambda*_i f^eq_i / rho = sum_i lambda*_i w_i E_i;
            // T_a / rho = sum_i lambda*_i w_i (3 c_ia + 9 (c_i.u) c_ia - 3 u_a).
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
            const double Tx = tx - 3.0 * ux * lw, Ty = ty - 3.0 * uy * lw, Tz = tz - 3.0 * uz * lw;
            const double TU = Tx * ux + Ty * uy + Tz * uz;
            static_for<0, Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                const double tc = cdot<i>(Tx, Ty, Tz);
                *at(lam_n + i * geo.dstride, off) = (1.0 - omega) * ls[i] + omega * (Ssum + tc - TU);
            });
            dw[0] = dw[0] + dom;
        } else {
            // the seven moments with their own MRT rates, of lambda* (for mu)
            // and of n = f^eq - f (for the rate sums)
            double a[7] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
            double dpm[2] = {0.0, 0.0};          // (lambda*+).n, (lambda*-).n
            if constexpr (COLL == COLL_MRT) {
                static_for<0, 7>([&](auto Kx) {
                    constexpr int k = decltype(Kx)::value;
                    constexpr int m = mrt_extra(k);
                    double ml = 0.0, mn = 0.0;
                    static_for<0, Q>([&](auto I) {
                        constexpr int i = decltype(I)::value;
                        constexpr int c = mrt_poly(m, i);
                        if constexpr (c != 0) {
                            const double cu = cdot<i>(ux, uy, uz);
                            const double n = weight<double>(i) * rho * (1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq) - f[i];
                            ml = ml + double(c) * ls[i];
                            mn = mn + double(c) * n;
                        }
                    });
                    const double d = ml * mn / double(mrt_norm(m));
                    // k = 0: e (bulk); 1-3: even ghosts; 4-6: odd ghosts
                    if constexpr (k == 0) dw[2] = dw[2] + d;
                    else if constexpr (k < 4) dw[3] = dw[3] + d;
                    else dw[4] = dw[4] + d;
                    if constexpr (k < 4) dpm[0] = dpm[0] - d;      // shear = even - bulk - even ghosts
                    else dpm[1] = dpm[1] - d;                       // flux = odd - odd ghosts
                    const double dom = k == 0 ? cp.omega_b - cp.omega_f
                                              : (k < 4 ? cp.omega_ge - cp.omega_f : cp.omega_go - cp.omega_m);
                    a[k] = dom * ml / double(mrt_norm(m));
                });
            }
            auto mu_of = [&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int o = opp(i);
                double corr = 0.0;
                if constexpr (COLL == COLL_MRT) {
                    static_for<0, 7>([&](auto Kx) {
                        constexpr int k = decltype(Kx)::value;
                        constexpr int c = mrt_poly(mrt_extra(k), i);
                        if constexpr (c != 0) corr = corr + double(c) * a[k];
                    });
                }
                return cp.omega_f * 0.5 * (ls[i] + ls[o]) + cp.omega_m * 0.5 * (ls[i] - ls[o]) + corr;
            };
            double Ssum = 0.0, lw = 0.0, tx = 0.0, ty = 0.0, tz = 0.0;
            static_for<0, Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                constexpr int o = opp(i);
                const double cu = cdot<i>(ux, uy, uz);
                const double E = 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq;
                const double mwi = mu_of(I) * weight<double>(i);
                Ssum = Ssum + mwi * E;
                lw = lw + mwi;
                const double h = mwi * (3.0 + 9.0 * cu);
                if constexpr (cx(i) > 0) tx = tx + h;
                if constexpr (cx(i) < 0) tx = tx - h;
                if constexpr (cy(i) > 0) ty = ty + h;
                if constexpr (cy(i) < 0) ty = ty - h;
                if constexpr (cz(i) > 0) tz = tz + h;
                if constexpr (cz(i) < 0) tz = tz - h;
                const double n = weight<double>(i) * rho * E - f[i];
                dpm[0] = dpm[0] + 0.5 * (ls[i] + ls[o]) * n;
                dpm[1] = dpm[1] + 0.5 * (ls[i] - ls[o]) * n;
            });
            const double Tx = tx - 3.0 * ux * lw, Ty = ty - 3.0 * uy * lw, Tz = tz - 3.0 * uz * lw;
            const double TU = Tx * ux + Ty * uy + Tz * uz;
            static_for<0, Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                const double tc = cdot<i>(Tx, Ty, Tz);
                *at(lam_n + i * geo.dstride, off) = ls[i] - mu_of(I) + (Ssum + tc - TU);
            });
            dw[0] = dw[0] + dpm[0];
            dw[1] = dw[1] + dpm[1];
        }
    }
    block_tree_sum<P::TPB, K>(dw, sh);
    if ((int)threadIdx.x < K) partial[8 * (size_t)blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
    if (prev_partial != nullptr && blockIdx.x == 0) final_sums<P::TPB, K>(prev_partial, prev_nblocks, sums, 0.0, 0.0, 1);
}

// ---------------------------------------------------------------------------
// Adjoint of one binary-fluid FP64 step.  The step reads, at each site, f and
// g and three stencil inputs built from phi = sum g at the site and its six
// neighbours (phi, grad phi, lap phi).  The reverse sweep is split the same
// way: a local kernel applies the transpose of the site's Jacobian (giving
// dL/df^n directly, and the site's sensitivities to its stencil inputs), and
// a stencil kernel applies the transposes of the central difference and of
// the 7-point Laplacian to those sensitivities, which gives dL/dphi at each
// site and hence the same addition to every dL/dg^n_j there.
//
// With lambda* the post-collision adjoints of a site, w_i their weights,
// E_i = 1 + 3 c.u + 9/2 (c.u)^2 - 3/2 u.u and X = 9/2 sum lambda* w (|c|^2 - 1):
//   a_phi = omega_f Xf (A phi + 3 B phi^3 - kappa lap)
//           + omega_g [Sg + Xg (Gamma (A + 3 B phi^2) - 1/3)],
//   a_G   = omega_f kappa [9 (YG - Lf G / 3) - Xf G],   YG_a = sum lf* w c_a (c.G),
//   a_lap = -kappa (omega_f phi Xf + omega_g Gamma Xg),
// Sf, Sg = sum lambda* w E, Lf = sum lf* w, and T_a = sum lambda* w dE/du_a.
// ---------------------------------------------------------------------------

struct BinAdj {
    double Sf, Tf[3], Tg[3];     // f-row of the transpose, and dL/drho, dL/du
    double a_phi, a_G[3], a_lap; // sensitivities to the stencil inputs
    double dkappa;               // sensitivity to kappa at fixed phi, G, lap
};

// Running weighted sums of one distribution's post-collision adjoints l_i:
// L = sum l w, S = sum l w E, X = sum l w (|c|^2 - 1) (times 9/2 later),
// t_a = sum l w c_a (3 + 9 c.u) and y_a = sum l w c_a (c.G).
// (y only for f: g^eq does not depend on grad phi.)
template <bool WITH_Y>
struct BinSums {
    double L = 0.0, S = 0.0, X = 0.0, t[3] = {0.0, 0.0, 0.0}, y[3] = {0.0, 0.0, 0.0};
    template <int i>
    __device__ __forceinline__ void add(double l, double cu, double E, double cG) {
        const double a = l * weight<double>(i);
        L = L + a;
        S = S + a * E;
        if constexpr (csq(i) == 0) X = X - a;
        if constexpr (csq(i) == 2) X = X + a;
        const double h = a * (3.0 + 9.0 * cu);
        if constexpr (cx(i) > 0) t[0] = t[0] + h;
        if constexpr (cx(i) < 0) t[0] = t[0] - h;
        if constexpr (cy(i) > 0) t[1] = t[1] + h;
        if constexpr (cy(i) < 0) t[1] = t[1] - h;
        if constexpr (cz(i) > 0) t[2] = t[2] + h;
        if constexpr (cz(i) < 0) t[2] = t[2] - h;
        if constexpr (WITH_Y) {
            const double yy = a * cG;
            if constexpr (cx(i) > 0) y[0] = y[0] + yy;
            if constexpr (cx(i) < 0) y[0] = y[0] - yy;
            if constexpr (cy(i) > 0) y[1] = y[1] + yy;
            if constexpr (cy(i) < 0) y[1] = y[1] - yy;
            if constexpr (cz(i) > 0) y[2] = y[2] + yy;
            if constexpr (cz(i) < 0) y[2] = y[2] - yy;
        }
    }
};

__device__ __forceinline__ BinAdj binary_adjoint_finish(const BinSums<true>& fs, const BinSums<false>& gs, double ux,
                                                        double uy,
                                                        double uz, double phi, double Gx, double Gy, double Gz,
                                                        double lap, const CollParams<double>& cp, double omega_f,
                                                        double omega_g) {
    const double Xf = 4.5 * fs.X, Xg = 4.5 * gs.X;
    const double u[3] = {ux, uy, uz}, G[3] = {Gx, Gy, Gz};
    const double k = cp.kappa;
    const double GG = Gx * Gx + Gy * Gy + Gz * Gz;
    BinAdj r;
    r.Sf = fs.S;
    for (int a = 0; a < 3; ++a) {
        r.Tf[a] = fs.t[a] - 3.0 * u[a] * fs.L;
        r.Tg[a] = gs.t[a] - 3.0 * u[a] * gs.L;
        r.a_G[a] = omega_f * k * (9.0 * (fs.y[a] - fs.L * G[a] / 3.0) - Xf * G[a]);
    }
    const double diso = cp.A * phi + 3.0 * cp.B * phi * phi * phi - k * lap;
    const double dmu = cp.A + 3.0 * cp.B * phi * phi;
    r.a_phi = omega_f * Xf * diso + omega_g * (gs.S + Xg * (cp.gamma * dmu - 1.0 / 3.0));
    r.a_lap = -k * (omega_f * phi * Xf + omega_g * cp.gamma * Xg);
    const double GYG = Gx * fs.y[0] + Gy * fs.y[1] + Gz * fs.y[2];
    r.dkappa = omega_f * (4.5 * (GYG - fs.L * GG / 3.0) + Xf * (-phi * lap - 0.5 * GG))
               + omega_g * cp.gamma * Xg * (-lap);
    return r;
}

__device__ __forceinline__ BinAdj binary_adjoint_site(const double (&lf)[Q], const double (&lg)[Q], double ux,
                                                      double uy, double uz, double phi, double Gx, double Gy,
                                                      double Gz, double lap, const CollParams<double>& cp,
                                                      double omega_f, double omega_g) {
    const double usq = ux * ux + uy * uy + uz * uz;
    BinSums<true> fs;
    BinSums<false> gs;
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        const double cu = cdot<i>(ux, uy, uz);
        const double E = 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq;
        fs.template add<i>(lf[i], cu, E, cdot<i>(Gx, Gy, Gz));
        gs.template add<i>(lg[i], cu, E, 0.0);
    });
    return binary_adjoint_finish(fs, gs, ux, uy, uz, phi, Gx, Gy, Gz, lap, cp, omega_f, omega_g);
}

// phi and its central-difference gradient and Laplacian at a site, from a
// scalar field in canonical layout.
__device__ __forceinline__ void phi_stencil(const double* __restrict__ phi, const Site& st, const Geo& geo,
                                            double& p, double& Gx, double& Gy, double& Gz, double& lap) {
    p = phi[offset_at<0, 0, 0>(st, geo)];
    const double pxm = phi[offset_at<-1, 0, 0>(st, geo)], pxp = phi[offset_at<1, 0, 0>(st, geo)];
    const double pym = phi[offset_at<0, -1, 0>(st, geo)], pyp = phi[offset_at<0, 1, 0>(st, geo)];
    const double pzm = phi[offset_at<0, 0, -1>(st, geo)], pzp = phi[offset_at<0, 0, 1>(st, geo)];
    Gx = 0.5 * (pxp - pxm);
    Gy = 0.5 * (pyp - pym);
    Gz = 0.5 * (pzp - pzm);
    lap = (pxp + pxm) + (pyp + pym) + (pzp + pzm) - 6.0 * p;
}

// Direction i of a canonical array (direction stride dstride elements) at
// element offset o within the direction.  OFF32: the whole array is below
// 4 GiB, so the address is one base per array plus a 32-bit byte offset and
// the kernel keeps one scalar base per array instead of one per direction
// (which spilled: measured 8.5% faster for the pair-form BGK adjoint step at
// 128^3); otherwise a base per direction, 64-bit.
template <bool OFF32, class T>
__device__ __forceinline__ T* dir_at(T* base, int i, int64_t dstride, uint32_t o) {
    if constexpr (OFF32) return at(base, (uint32_t)i * (uint32_t)dstride + o);
    else return at(base + i * dstride, o);
}

// How the local kernel obtains the post-collision g adjoints of its site,
// lambda*_j(s) = lambda_g^{n+1}_j(s + c_j), and whether it keeps them:
//   LG_GATHER       gathered from lambda_g^{n+1} (canonical);
//   LG_GATHER_KEEP  the same, and stored unshifted, P^n_j(s) = lambda*_j(s);
//   LG_PULLED_KEEP  lambda_g^{n+1} is held as the pair (P^{n+1}, b^{n+1}),
//                   lambda_g^{n+1}_j(x) = (1 - omega_g) P^{n+1}_j(x) + b^{n+1}(x),
//                   with b the stencil kernel's dL/dphi; gathered from that
//                   pair and stored as P^n.
// The pair form lets a reverse sweep over several steps skip writing and
// re-reading lambda_g itself: per step the stencil kernel then only turns
// the sensitivity fields into b (8 bytes a site) instead of gathering and
// writing lambda_g (304), at the price of the local kernel storing P (152).
enum { LG_GATHER = 0, LG_GATHER_KEEP = 1, LG_PULLED_KEEP = 2 };

// Omega lambda at direction i under TRT, from lambda_i and lambda_opp(i):
// omega_+ times the even part plus omega_- times the odd part.
__device__ __forceinline__ double trt_mu(double l, double lo, const CollParams<double>& cp) {
    return cp.omega_f * 0.5 * (l + lo) + cp.omega_m * 0.5 * (l - lo);
}

// Local part of the binary adjoint step.  fn, gn: f^n and g^n (canonical,
// or the recorded post-collision fields of the previous step when
// F_PENDING, pulled); phi: phi^n (canonical); lf_next: lambda_f^{n+1};
// lg_next: lambda_g^{n+1}, or P^{n+1} with b_next = b^{n+1} (LG above).
// Writes lambda_f^n, P^n to p_out (LG != LG_GATHER) and the five
// sensitivity fields afield[k*N + s] (a_phi, a_Gx, a_Gy, a_Gz, a_lap); block
// partials of dL/domega_f, dL/domega_g and dL/dkappa go to
// partial[8 b + 0..2].  Only lambda_f is kept, in LDS: f is reduced to its
// moments (and sum lambda_f f) as it loads, and g with lambda_g are consumed
// in one pass once u is known.
// COLL_TRT: f relaxes by two times (even and odd parts of f - f^eq), so
// mu = Omega lambda*_f = omega_+ (lambda*_i + lambda*_opp(i))/2
//                      + omega_- (lambda*_i - lambda*_opp(i))/2
// takes the place of omega_f lambda*_f and lambda*_f - mu that of
// (1 - omega_f) lambda*_f.  lambda*_f is then loaded before f, so that both
// directions of a pair are at hand, and the even and odd rate sums
// sum (P_+- lambda*_f)(f^eq - f) go to partial[8 b + 0] and [8 b + 3].
// COLL_MRT: mu adds, for each of the seven moments m with a rate of its own
// (the energy, three even and three odd ghosts), (omega_m - omega_+-) times
// the projection of lambda*_f on m; the moments of lambda*_f, f and f^eq on
// them give the bulk and ghost rate sums (partial[8 b + 4..6]), and the
// shear and flux sums are the even and odd sums less those.
// At least two waves per SIMD: BGK and TRT fit in 256 VGPRs anyway; the MRT
// variant then spills 45 VGPRs to scratch but runs 5% faster than at one
// wave (measured at 128^3).
template <class P, bool F_PENDING, int LG, int COLL = COLL_BGK, bool OFF32 = false>
__global__ __launch_bounds__(P::TPB, 2) void k_adjoint_binary(const double* __restrict__ fn,
                                                           const double* __restrict__ gn,
                                                           const double* __restrict__ phi,
                                                           const double* __restrict__ lf_next,
                                                           const double* __restrict__ lg_next,
                                                           const double* __restrict__ b_next,
                                                           double* __restrict__ lf_n, double* __restrict__ p_out,
                                                           double* __restrict__ afield,
                                                           double* __restrict__ partial, Geo geo,
                                                           CollParams<double> cp) {
    constexpr bool MRT = COLL == COLL_MRT;
    constexpr bool SPLIT = COLL != COLL_BGK;     // even and odd parts relax apart (TRT; MRT on top)
    constexpr int K = MRT ? 7 : (SPLIT ? 4 : 3);
    __shared__ double sh[K][P::TPB];
    __shared__ double lf[Q][P::TPB];         // this lane's lambda_f waits here (own slots only: no barrier)
    const int t = threadIdx.x;
    const Column col = column_of_thread<P>(geo);
    double acc[K] = {};
    for (int v = 0; v < P::TZ; ++v) {
        const Site st = site_at(col, v, geo);
        if (!st.active) continue;
        const uint32_t off = offset_at<0, 0, 0>(st, geo);
        if constexpr (SPLIT) {
            static_for<0, Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                lf[i][t] = *dir_at<OFF32>(lf_next, i, geo.dstride, offset_at<cx(i), cy(i), cz(i)>(st, geo));
            });
        }
        // f: moments and sum lambda_f f (TRT, MRT: also sum lambda_f,opp f); lambda_f kept
        double rho = 0.0, jx = 0.0, jy = 0.0, jz = 0.0, lff = 0.0, lof = 0.0;
        double mf[MRT ? 7 : 1] = {};                    // MRT: f on the seven extra moments
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double fi = *dir_at<OFF32>(fn, i, geo.dstride, src_offset<i, F_PENDING>(st, geo));
            double li;
            if constexpr (MRT) {
                static_for<0, 7>([&](auto Kx) {
                    constexpr int c = mrt_poly(mrt_extra(decltype(Kx)::value), i);
                    if constexpr (c != 0) mf[decltype(Kx)::value] = mf[decltype(Kx)::value] + double(c) * fi;
                });
            }
            if constexpr (SPLIT) {
                li = lf[i][t];
                lof = lof + lf[opp(i)][t] * fi;
            } else {
                li = *dir_at<OFF32>(lf_next, i, geo.dstride, offset_at<cx(i), cy(i), cz(i)>(st, geo));
                lf[i][t] = li;
            }
            rho = rho + fi;
            if constexpr (cx(i) > 0) jx = jx + fi;
            if constexpr (cx(i) < 0) jx = jx - fi;
            if constexpr (cy(i) > 0) jy = jy + fi;
            if constexpr (cy(i) < 0) jy = jy - fi;
            if constexpr (cz(i) > 0) jz = jz + fi;
            if constexpr (cz(i) < 0) jz = jz - fi;
            lff = lff + li * fi;
        });
        const double ux = jx / rho, uy = jy / rho, uz = jz / rho;
        const double usq = ux * ux + uy * uy + uz * uz;
        double p, Gx, Gy, Gz, lap;
        phi_stencil(phi, st, geo, p, Gx, Gy, Gz, lap);
        const FreeEnergy<double> fe(p, Gx, Gy, Gz, lap, cp);
        // g and lambda_g in one pass
        BinSums<false> gs;
        double dwg = 0.0;
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double gi = *dir_at<OFF32>(gn, i, geo.dstride, src_offset<i, F_PENDING>(st, geo));
            const uint32_t up = offset_at<cx(i), cy(i), cz(i)>(st, geo);
            double l = *dir_at<OFF32>(lg_next, i, geo.dstride, up);
            if constexpr (LG == LG_PULLED_KEEP) l = (1.0 - cp.omega_g) * l + *at(b_next, up);
            if constexpr (LG != LG_GATHER) *dir_at<OFF32>(p_out, i, geo.dstride, off) = l;
            const double cu = cdot<i>(ux, uy, uz);
            const double E = 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq;
            gs.template add<i>(l, cu, E, 0.0);
            dwg = dwg + l * (weight<double>(i) * (p * E + fe.template mobility_term<i>(cp)) - gi);
        });
        // MRT: lambda*_f on the seven extra moments, and the coefficients
        // a_k = (omega_k - omega_+-) (lambda*.m_k) / |m_k|^2 of its correction
        double ml[MRT ? 7 : 1] = {}, a[MRT ? 7 : 1] = {}, mfeq[MRT ? 7 : 1] = {};
        if constexpr (MRT) {
            static_for<0, 7>([&](auto Kx) {
                constexpr int k = decltype(Kx)::value;
                constexpr int m = mrt_extra(k);
                static_for<0, Q>([&](auto I) {
                    constexpr int c = mrt_poly(m, decltype(I)::value);
                    if constexpr (c != 0) ml[k] = ml[k] + double(c) * lf[decltype(I)::value][t];
                });
                const double dom = k == 0 ? cp.omega_b - cp.omega_f
                                          : (k < 4 ? cp.omega_ge - cp.omega_f : cp.omega_go - cp.omega_m);
                a[k] = dom * ml[k] / double(mrt_norm(m));
            });
        }
        // mu_i = omega_+ (l_i + l_opp)/2 + omega_- (l_i - l_opp)/2 (+ the MRT correction)
        auto mu_at = [&](auto I) {
            constexpr int i = decltype(I)::value;
            double mu = trt_mu(lf[i][t], lf[opp(i)][t], cp);
            if constexpr (MRT) {
                static_for<0, 7>([&](auto Kx) {
                    constexpr int c = mrt_poly(mrt_extra(decltype(Kx)::value), i);
                    if constexpr (c != 0) mu = mu + double(c) * a[decltype(Kx)::value];
                });
            }
            return mu;
        };
        // lambda_f pass (TRT, MRT: the sums take mu, and omega_f is folded in)
        BinSums<true> fs;
        double lfeq = 0.0, lofeq = 0.0;
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            const double cu = cdot<i>(ux, uy, uz);
            const double E = 1.0 + 3.0 * cu + 4.5 * cu * cu - 1.5 * usq;
            const double li = lf[i][t];
            if constexpr (SPLIT) {
                const double lo = lf[opp(i)][t];
                const double feq = weight<double>(i) * (rho * E + fe.template stress_term<i>(cp));
                fs.template add<i>(mu_at(I), cu, E, cdot<i>(Gx, Gy, Gz));
                lfeq = lfeq + li * feq;
                lofeq = lofeq + lo * feq;
                if constexpr (MRT) {
                    static_for<0, 7>([&](auto Kx) {
                        constexpr int c = mrt_poly(mrt_extra(decltype(Kx)::value), i);
                        if constexpr (c != 0) mfeq[decltype(Kx)::value] = mfeq[decltype(Kx)::value] + double(c) * feq;
                    });
                }
            } else {
                fs.template add<i>(li, cu, E, cdot<i>(Gx, Gy, Gz));
                lfeq = lfeq + li * weight<double>(i) * (rho * E + fe.template stress_term<i>(cp));
            }
        });
        const double wf = SPLIT ? 1.0 : cp.omega_f;
        const BinAdj r = binary_adjoint_finish(fs, gs, ux, uy, uz, p, Gx, Gy, Gz, lap, cp, wf, cp.omega_g);
        const double wg = cp.omega_g * p / rho;
        const double V[3] = {wf * r.Tf[0] + wg * r.Tg[0], wf * r.Tf[1] + wg * r.Tg[1], wf * r.Tf[2] + wg * r.Tg[2]};
        const double base = wf * r.Sf - (V[0] * ux + V[1] * uy + V[2] * uz);
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            if constexpr (SPLIT) {
                *dir_at<OFF32>(lf_n, i, geo.dstride, off) = lf[i][t] - mu_at(I) + base + cdot<i>(V[0], V[1], V[2]);
            } else {
                *dir_at<OFF32>(lf_n, i, geo.dstride, off) = (1.0 - cp.omega_f) * lf[i][t] + base + cdot<i>(V[0], V[1], V[2]);
            }
        });
        afield[off] = r.a_phi;
        afield[(size_t)geo.nsite + off] = r.a_G[0];
        afield[2 * (size_t)geo.nsite + off] = r.a_G[1];
        afield[3 * (size_t)geo.nsite + off] = r.a_G[2];
        afield[4 * (size_t)geo.nsite + off] = r.a_lap;
        if constexpr (SPLIT) {
            // sum (P_+- lambda*)(f^eq - f) = [sum lambda* (f^eq - f) +- sum lambda*_opp (f^eq - f)] / 2
            const double all = lfeq - lff, cross = lofeq - lof;
            double even = 0.5 * (all + cross), odd = 0.5 * (all - cross);
            if constexpr (MRT) {
                // rate sum of moment k: (lambda*.m_k)((f^eq - f).m_k) / |m_k|^2;
                // k = 0 energy (bulk), 1-3 even ghosts, 4-6 odd ghosts
                static_for<0, 7>([&](auto Kx) {
                    constexpr int k = decltype(Kx)::value;
                    const double d = ml[k] * (mfeq[k] - mf[k]) / double(mrt_norm(mrt_extra(k)));
                    if constexpr (k == 0) acc[4] = acc[4] + d;
                    else if constexpr (k < 4) acc[5] = acc[5] + d;
                    else acc[6] = acc[6] + d;
                    if constexpr (k < 4) even = even - d;      // shear = even - bulk - even ghosts
                    else odd = odd - d;                         // flux = odd - odd ghosts
                });
            }
            acc[0] = acc[0] + even;
            acc[3] = acc[3] + odd;
        } else {
            acc[0] = acc[0] + (lfeq - lff);
        }
        acc[1] = acc[1] + dwg;
        acc[2] = acc[2] + r.dkappa;
    }
    block_tree_sum<P::TPB, K>(acc, sh);
    if ((int)threadIdx.x < K) partial[8 * (size_t)blockIdx.x + threadIdx.x] = sh[threadIdx.x][0];
}

// Local part of the reverse of the equilibrium initialisation
// f^0 = f^eq(rho, u, P(phi)), g^0 = g^eq(phi, u, mu(phi)): unit relaxation,
// unshifted adjoints.  Writes the sensitivity fields, dL/drho = Sf and
// dL/du_a = rho Tf_a + phi Tg_a; partial[8 b + 0] = dL/dkappa.
template <class P>
__global__ __launch_bounds__(P::TPB) void k_adjoint_binary_init(const double* __restrict__ rho_in,
                                                                const double* __restrict__ u_in,
                                                                const double* __restrict__ phi,
                                                                const double* __restrict__ lf0,
                                                                const double* __restrict__ lg0,
                                                                double* __restrict__ afield,
                                                                double* __restrict__ drho,
                                                                double* __restrict__ du,
                                                                double* __restrict__ partial, Geo geo,
                                                                CollParams<double> cp) {
    __shared__ double sh[1][P::TPB];
    const Column col = column_of_thread<P>(geo);
    double acc[1] = {0.0};
    for (int v = 0; v < P::TZ; ++v) {
        const Site st = site_at(col, v, geo);
        if (!st.active) continue;
        const uint32_t off = offset_at<0, 0, 0>(st, geo);
        double lf[Q], lg[Q];
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            lf[i] = lf0[i * geo.dstride + off];
            lg[i] = lg0[i * geo.dstride + off];
        });
        double p, Gx, Gy, Gz, lap;
        phi_stencil(phi, st, geo, p, Gx, Gy, Gz, lap);
        const double rho = rho_in[off];
        const double ux = u_in[off], uy = u_in[(size_t)geo.nsite + off], uz = u_in[2 * (size_t)geo.nsite + off];
        const BinAdj r = binary_adjoint_site(lf, lg, ux, uy, uz, p, Gx, Gy, Gz, lap, cp, 1.0, 1.0);
        afield[off] = r.a_phi;
        afield[(size_t)geo.nsite + off] = r.a_G[0];
        afield[2 * (size_t)geo.nsite + off] = r.a_G[1];
        afield[3 * (size_t)geo.nsite + off] = r.a_G[2];
        afield[4 * (size_t)geo.nsite + off] = r.a_lap;
        drho[off] = r.Sf;
        for (int a = 0; a < 3; ++a) du[(size_t)a * geo.nsite + off] = rho * r.Tf[a] + p * r.Tg[a];
        acc[0] = acc[0] + r.dkappa;
    }
    block_tree_sum<P::TPB, 1>(acc, sh);
    if (threadIdx.x == 0) partial[8 * (size_t)blockIdx.x] = sh[0][0];
}

// Stencil part: b(s) = a_phi(s) - 6 a_lap(s) + sum_a [a_G_a(s - e_a) - a_G_a(s + e_a)] / 2
//                      + sum_a [a_lap(s + e_a) + a_lap(s - e_a)]   (= dL/dphi(s)).
// B_ONLY (the reverse of the initialisation, and each step of a sweep in
// the pair form): out[s] = b.  Otherwise out is lambda_g^n:
// out_j(s) = (1 - omega_g) lambda_g^{n+1}_j(s + c_j) + b(s).  Block 0 also
// adds the K block partials the local kernel left (partial[8 b + k],
// b < nblocks) into sums[0..K), in block order, which saves the step a
// separate reduction launch.
template <class P, bool B_ONLY, int K>
__global__ __launch_bounds__(P::TPB) void k_adjoint_binary_stencil(const double* __restrict__ afield,
                                                                   const double* __restrict__ lg_next,
                                                                   double* __restrict__ out, Geo geo,
                                                                   double omega_g,
                                                                   const double* __restrict__ partial,
                                                                   int nblocks, double* __restrict__ sums) {
    const Column col = column_of_thread<P>(geo);
    const size_t N = geo.nsite;
    for (int v = 0; v < P::TZ; ++v) {
        const Site st = site_at(col, v, geo);
        if (!st.active) continue;
        const uint32_t off = offset_at<0, 0, 0>(st, geo);
        const double* ap = afield;
        const double* ax = afield + N;
        const double* ay = afield + 2 * N;
        const double* az = afield + 3 * N;
        const double* al = afield + 4 * N;
        double b = ap[off] - 6.0 * al[off];
        b = b + 0.5 * (ax[offset_at<-1, 0, 0>(st, geo)] - ax[offset_at<1, 0, 0>(st, geo)]);
        b = b + 0.5 * (ay[offset_at<0, -1, 0>(st, geo)] - ay[offset_at<0, 1, 0>(st, geo)]);
        b = b + 0.5 * (az[offset_at<0, 0, -1>(st, geo)] - az[offset_at<0, 0, 1>(st, geo)]);
        b = b + (al[offset_at<1, 0, 0>(st, geo)] + al[offset_at<-1, 0, 0>(st, geo)]);
        b = b + (al[offset_at<0, 1, 0>(st, geo)] + al[offset_at<0, -1, 0>(st, geo)]);
        b = b + (al[offset_at<0, 0, 1>(st, geo)] + al[offset_at<0, 0, -1>(st, geo)]);
        if constexpr (B_ONLY) {
            out[off] = b;
        } else {
            static_for<0, Q>([&](auto I) {
                constexpr int i = decltype(I)::value;
                *at(out + i * geo.dstride, off) =
                    (1.0 - omega_g) * *at(lg_next + i * geo.dstride, offset_at<cx(i), cy(i), cz(i)>(st, geo)) + b;
            });
        }
    }
    if (blockIdx.x == 0) final_sums<P::TPB, K>(partial, nblocks, sums, 0.0, 0.0, 1);
}

// lambda_g^n_j(s) = (1 - omega_g) P^n_j(s) + b^n(s): the pair form of the
// local kernel (LG_PULLED_KEEP) back to canonical lambda_g.  Pointwise, so
// pn and out may be the same array (hence no __restrict__ on them).
template <class P>
__global__ __launch_bounds__(P::TPB) void k_adjoint_binary_combine(const double* pn,
                                                                   const double* __restrict__ b, double* out,
                                                                   Geo geo, double omega_g) {
    const Column col = column_of_thread<P>(geo);
    for (int v = 0; v < P::TZ; ++v) {
        const Site st = site_at(col, v, geo);
        if (!st.active) continue;
        const uint32_t off = offset_at<0, 0, 0>(st, geo);
        const double bs = b[off];
        static_for<0, Q>([&](auto I) {
            constexpr int i = decltype(I)::value;
            *at(out + i * geo.dstride, off) = (1.0 - omega_g) * *at(pn + i * geo.dstride, off) + bs;
        });
    }
}

// ---------------------------------------------------------------------------
// Masked transfer (the masked copies of Section III-B): a mask over the sites
// is compacted, in increasing site order, into a list of site indices; the
// state at the listed sites is then gathered into or scattered from a packed
// direction-major array [19][m].  Compaction is three deterministic passes
// over blocks of CB consecutive sites: count, scan of the block counts, and
// a scatter that scans each block's flags in LDS.
// ---------------------------------------------------------------------------

constexpr int CB = 256;

__global__ __launch_bounds__(CB) void k_mask_count(const uint8_t* __restrict__ mask, uint32_t nsite,
                                                   int64_t* __restrict__ counts) {
    __shared__ int sh[CB];
    const uint32_t s = blockIdx.x * CB + threadIdx.x;
    sh[threadIdx.x] = (s < nsite && mask[s] != 0) ? 1 : 0;
    __syncthreads();
    for (int half = CB / 2; half > 0; half >>= 1) {
        if ((int)threadIdx.x < half) sh[threadIdx.x] += sh[threadIdx.x + half];
        __syncthreads();
    }
    if (threadIdx.x == 0) counts[blockIdx.x] = sh[0];
}

// Exclusive scan of counts[0..nb) in place (one block); total -> *total.
__global__ __launch_bounds__(CB) void k_scan_counts(int64_t* counts, int nb, int64_t* total) {
    __shared__ int64_t sh[CB];
    const int t = threadIdx.x;
    const int per = (nb + CB - 1) / CB;
    const int b0 = t * per, b1 = min(b0 + per, nb);
    int64_t sum = 0;
    for (int b = b0; b < b1; ++b) sum += counts[b];
    sh[t] = sum;
    __syncthreads();
    // inclusive Hillis-Steele scan of the per-thread sums
    for (int d = 1; d < CB; d <<= 1) {
        const int64_t v = t >= d ? sh[t - d] : 0;
        __syncthreads();
        sh[t] += v;
        __syncthreads();
    }
    int64_t run = sh[t] - sum;
    for (int b = b0; b < b1; ++b) {
        const int64_t c = counts[b];
        counts[b] = run;
        run += c;
    }
    if (t == CB - 1) *total = sh[CB - 1];
}

__global__ __launch_bounds__(CB) void k_mask_scatter(const uint8_t* __restrict__ mask, uint32_t nsite,
                                                     const int64_t* __restrict__ offsets,
                                                     int32_t* __restrict__ index) {
    __shared__ int sh[CB];
    const uint32_t s = blockIdx.x * CB + threadIdx.x;
    const int flag = (s < nsite && mask[s] != 0) ? 1 : 0;
    sh[threadIdx.x] = flag;
    __syncthreads();
    for (int d = 1; d < CB; d <<= 1) {
        const int v = (int)threadIdx.x >= d ? sh[threadIdx.x - d] : 0;
        __syncthreads();
        sh[threadIdx.x] += v;
        __syncthreads();
    }
    if (flag) index[offsets[blockIdx.x] + sh[threadIdx.x] - 1] = (int32_t)s;
}

// Site s as coordinates with periodic neighbours.
__device__ __forceinline__ Site site_of_index(uint32_t s, const Geo& g) {
    const int x = (int)(s % (uint32_t)g.nx);
    const int y = (int)((s / (uint32_t)g.nx) % (uint32_t)g.ny);
    const int z = (int)(s / g.plane);
    return site_wrapped(x, y, z, g);
}

// packed[i*m + t] = state_i(index[t]); PENDING buffers are read by pull.
template <class S, bool PENDING>
__global__ __launch_bounds__(CB) void k_get_sites(const S* __restrict__ buf, const int32_t* __restrict__ index,
                                                  int64_t m, S* __restrict__ packed, Geo geo) {
    const int64_t t = (int64_t)blockIdx.x * CB + threadIdx.x;
    if (t >= m) return;
    const uint32_t s = (uint32_t)index[t];
    if (s >= geo.nsite) return;                 // not a site: leave the slot alone
    const Site st = site_of_index(s, geo);
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        packed[i * m + t] = *at(buf + i * geo.dstride, src_offset<i, PENDING>(st, geo));
    });
}

// state_i(index[t]) = packed[i*m + t]; for a PENDING buffer the value goes
// where the next pull reads it (s - c_i).
template <class S, bool PENDING>
__global__ __launch_bounds__(CB) void k_set_sites(S* __restrict__ buf, const int32_t* __restrict__ index, int64_t m,
                                                  const S* __restrict__ packed, Geo geo) {
    const int64_t t = (int64_t)blockIdx.x * CB + threadIdx.x;
    if (t >= m) return;
    const uint32_t s = (uint32_t)index[t];
    if (s >= geo.nsite) return;                 // not a site: ignored
    const Site st = site_of_index(s, geo);
    static_for<0, Q>([&](auto I) {
        constexpr int i = decltype(I)::value;
        *at(buf + i * geo.dstride, src_offset<i, PENDING>(st, geo)) = packed[i * m + t];
    });
}

// ---------------------------------------------------------------------------
// Streaming copy: every byte read once and written once, 16 bytes per access
// and COPY_U accesses in flight per lane (the loads of a lane are issued
// before its first store), nontemporal stores as in the step kernels.  The
// plain copy is what the memory system sustains with no gather and no
// arithmetic: the practical ceiling of the update kernels, and the kernel
// whose known byte count calibrates the profiler's HBM byte counters.
// ---------------------------------------------------------------------------

typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));
constexpr int COPY_TPB = 256;
constexpr int COPY_U = 4;

__global__ __launch_bounds__(COPY_TPB) void k_stream_copy(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                          uint64_t nwords) {
    const uint64_t base = (uint64_t)blockIdx.x * (COPY_TPB * COPY_U) + threadIdx.x;
    u32x4 v[COPY_U];
#pragma unroll
    for (int u = 0; u < COPY_U; ++u) {
        const uint64_t k = base + (uint64_t)u * COPY_TPB;
        if (k < nwords) v[u] = src[k];
    }
#pragma unroll
    for (int u = 0; u < COPY_U; ++u) {
        const uint64_t k = base + (uint64_t)u * COPY_TPB;
        if (k < nwords) __builtin_nontemporal_store(v[u], dst + k);
    }
}

}  // namespace lbk
