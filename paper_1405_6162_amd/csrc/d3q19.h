// D3Q19 lattice, site geometry and storage codecs for the gfx950 kernels.
//
// Velocity ordering: rest first, then the 18 velocities with |c|^2 in {1,2}
// in lexicographic order of (c_x, c_y, c_z); weights 1/3, 1/18, 1/36 and
// c_s^2 = 1/3.  Everything here is compile-time: with the direction loops
// fully unrolled every c_i and w_i becomes an immediate.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

namespace lbk {

constexpr int Q = 19;

__host__ __device__ constexpr int cx(int i) {
    constexpr int t[Q] = {0, -1, -1, -1, -1, -1, 0, 0, 0, 0, 0, 0, 0, 0, 1, 1, 1, 1, 1};
    return t[i];
}
__host__ __device__ constexpr int cy(int i) {
    constexpr int t[Q] = {0, -1, 0, 0, 0, 1, -1, -1, -1, 0, 0, 1, 1, 1, -1, 0, 0, 0, 1};
    return t[i];
}
__host__ __device__ constexpr int cz(int i) {
    constexpr int t[Q] = {0, 0, -1, 0, 1, 0, -1, 0, 1, -1, 1, -1, 0, 1, 0, -1, 0, 1, 0};
    return t[i];
}
__host__ __device__ constexpr int csq(int i) { return cx(i) * cx(i) + cy(i) * cy(i) + cz(i) * cz(i); }

// Index of the opposite velocity, c_opp(i) = -c_i.
__host__ __device__ constexpr int opp(int i) {
    for (int j = 0; j < Q; ++j)
        if (cx(j) == -cx(i) && cy(j) == -cy(i) && cz(j) == -cz(i)) return j;
    return -1;
}
static_assert(opp(0) == 0 && opp(1) == 18 && opp(9) == 10, "D3Q19 opposites");

template <class T>
__host__ __device__ constexpr T weight(int i) {
    return csq(i) == 0 ? T(1) / T(3) : (csq(i) == 1 ? T(1) / T(18) : T(1) / T(36));
}

// Moments of the orthogonal D3Q19 basis of d'Humieres et al. (2002) that the
// multiple-relaxation-time collision relaxes at rates of their own (the
// others relax as in the two-relaxation-time collision): polynomial m at
// velocity i, for m = 1 (e), 2 (eps), 10 (3 pi_xx), 12 (pi_ww), 16, 17, 18
// (m_x, m_y, m_z).
__host__ __device__ constexpr int mrt_poly(int m, int i) {
    const int x = cx(i), y = cy(i), z = cz(i), c2 = csq(i);
    switch (m) {
        case 1: return 19 * c2 - 30;
        case 2: return (21 * c2 * c2 - 53 * c2 + 24) / 2;
        case 10: return (3 * c2 - 5) * (3 * x * x - c2);
        case 12: return (3 * c2 - 5) * (y * y - z * z);
        case 16: return (y * y - z * z) * x;
        case 17: return (z * z - x * x) * y;
        case 18: return (x * x - y * y) * z;
    }
    return 0;
}
__host__ __device__ constexpr int mrt_extra(int k) {
    constexpr int t[7] = {1, 2, 10, 12, 16, 17, 18};
    return t[k];
}
__host__ __device__ constexpr int mrt_norm(int m) {
    int s = 0;
    for (int i = 0; i < Q; ++i) s += mrt_poly(m, i) * mrt_poly(m, i);
    return s;
}
static_assert(mrt_norm(1) == 2394 && mrt_norm(2) == 252 && mrt_norm(10) == 72 && mrt_norm(12) == 24 &&
              mrt_norm(16) == 8, "MRT basis norms");

// Compute type for each storage type: FP64 storage computes in FP64, the
// reduced-precision storages compute in FP32.
template <class S> struct Compute;
template <> struct Compute<double>   { using T = double; };
template <> struct Compute<float>    { using T = float; };
template <> struct Compute<_Float16> { using T = float; };

// Type of the moment sums rho - rho0 = sum d_i, j = sum c_i d_i and
// phi - phi0 = sum e_i inside the collision.  FP64 sums in the FP32 binary
// step were measured against FP32 ones: the first steps' phi and u errors
// fall about 3x, the error after 500 steps of spinodal growth is unchanged,
// the drift of sum phi grows from ~1e-11 to ~1e-7 per site over 500 steps
// and the step slows by 9%; the reduced-precision collision therefore sums
// in its compute type.  Reported sums (lb_conserved_sums, lb_field_stats,
// lb_moments) are FP64 for every storage.
template <class S> struct Accum { using T = typename Compute<S>::T; };


// Lattice geometry and the layout of the distribution arrays it addresses.
// Element (i, x, y, z) of a distribution is at
//     i * dstride + z * zs + y * ys + (x / 64) * xbs + x % 64.
// Canonical (structure of arrays, x fastest): zs = nx * ny, ys = nx,
// xbs = 64, dstride >= N, i.e. i * dstride + x + nx (y + ny z).  Blocked:
// each run of 64 x-consecutive sites holds its 19 directions together,
// dstride = 64, xbs = 19 * 64, ys = ceil(nx / 64) * xbs, zs = ny * ys, so the
// 19 pulls of a wavefront land in one 19 * 64-element block per source row
// instead of 19 arrays N elements apart.  Offsets fit in 32 bits (checked on
// the host); i * dstride is formed in 64 bits.  Scalar fields (phi, moments,
// inputs) are always canonical: site index x + nx (y + ny z) (canon_at).
// gx, gy, gz and nblocks describe the tiling of the launch that receives
// this Geo.
struct Geo {
    int nx, ny, nz;
    uint32_t plane;     // nx * ny
    uint32_t nsite;     // nx * ny * nz
    int64_t dstride;    // elements between consecutive directions
    int gx, gy, gz;     // tiles along x, y and z
    int nblocks;        // gx * gy * gz: the 1-D grid size
    uint32_t zs, ys, xbs;   // site-offset strides of the distribution layout
    int bz;             // z planes per block of the single-pass march (its chunk depth)
};

// Launch policy.  A block covers TX x TY x TZ sites; each lane owns one
// (x, y) column of the tile and TZ consecutive z planes of it (TZ sites per
// lane: the strip-mined "virtual vector" of the targetDP execution model,
// Section III-C, mapped onto a GPU lane).  A wavefront spans 64 consecutive
// x, so every direction array is read and written in contiguous runs.
// Blocks form a 1-D grid; with XCD ordering, block b is given tile
// (b mod 8) * nblocks/8 + b/8, so each of the eight XCDs (which receive
// blocks round-robin) sweeps a contiguous slab of tiles and the neighbouring
// rows a pull or a stencil touches are in its own L2.  NTL / NTS select
// nontemporal loads / stores of the distributions.
template <int TX_, int TY_, int TZ_, bool NTL_, bool NTS_, bool XCD_>
struct Tiling {
    static constexpr int TX = TX_, TY = TY_, TZ = TZ_, TPB = TX_ * TY_;
    static constexpr bool nt_load = NTL_, nt_store = NTS_, xcd = XCD_;
    static_assert(TPB % 64 == 0, "whole wavefronts");
};

__host__ __device__ constexpr int tiles(int n, int t) { return (n + t - 1) / t; }

// The lane's (x, y) column, its +-1 neighbours (periodic), and the tile origin.
struct Column {
    int x, y, xm, xp, ym, yp;
    int x0, y0, z0;
    bool active;        // (x, y) inside the lattice
};

// One site of the column: z, its +-1 neighbours, and whether z < nz.
struct Site {
    int x, y, z, xm, xp, ym, yp, zm, zp;
    bool active;
};

template <class P>
__device__ __forceinline__ bool xcd_remapped(const Geo& g) {
    return P::xcd && (g.nblocks & 7) == 0;
}

template <class P>
__device__ __forceinline__ int tile_index(const Geo& g) {
    int b = blockIdx.x;
    if (xcd_remapped<P>(g)) b = (b & 7) * (g.nblocks >> 3) + (b >> 3);
    return b;
}

template <class P>
__device__ __forceinline__ Column column_of_thread(const Geo& g) {
    const int b = tile_index<P>(g);
    const int bx = b % g.gx;
    const int t = b / g.gx;
    const int by = t % g.gy;
    Column c;
    c.z0 = (t / g.gy) * P::TZ;
    c.x0 = bx * P::TX;
    c.y0 = by * P::TY;
    c.x = c.x0 + (int)(threadIdx.x % P::TX);
    c.y = c.y0 + (int)(threadIdx.x / P::TX);
    c.active = (c.x < g.nx) && (c.y < g.ny);
    c.xm = c.x == 0 ? g.nx - 1 : c.x - 1;
    c.xp = c.x + 1 >= g.nx ? 0 : c.x + 1;
    c.ym = c.y == 0 ? g.ny - 1 : c.y - 1;
    c.yp = c.y + 1 >= g.ny ? 0 : c.y + 1;
    return c;
}

__device__ __forceinline__ Site site_at(const Column& c, int v, const Geo& g) {
    Site s;
    s.x = c.x; s.y = c.y; s.xm = c.xm; s.xp = c.xp; s.ym = c.ym; s.yp = c.yp;
    s.z = c.z0 + v;
    s.active = c.active && s.z < g.nz;
    s.zm = s.z == 0 ? g.nz - 1 : s.z - 1;
    s.zp = s.z + 1 >= g.nz ? 0 : s.z + 1;
    return s;
}

// Global loads and stores of element `off` of an array whose base is the
// same for the whole launch, nontemporal when the policy says so.  For 2-
// and 8-byte elements the byte offset is formed in 32 bits (such arrays are
// below 4 GiB here, checked on the host), so the address is a scalar base
// plus a 32-bit vector offset and no 64-bit address arithmetic is spent per
// lane.  4-byte elements take the element offset, scaled in 64 bits, so
// that an FP32 state of up to 2^32 values keeps the blocked layout (384^3:
// 4.3 GB, 7% faster than the structure of arrays it needed in bytes; no
// difference at 256^3).  For 8-byte elements the 64-bit form was 0.6%
// slower at 256^3 and 14% slower in the binary adjoint kernel.  (2-byte
// elements once ran 20-30% slower in the 32-bit form, because a running sum
// over 19 gathered values then sent its loads out one at a time; with the
// values gathered into an array before the sum it is 1% faster for them.)
template <class S>
__device__ __forceinline__ const S* at(const S* base, uint32_t off) {
    if constexpr (sizeof(S) == 4) return base + off;
    else return reinterpret_cast<const S*>(reinterpret_cast<const char*>(base) + (uint32_t)(off * (uint32_t)sizeof(S)));
}
template <class S>
__device__ __forceinline__ S* at(S* base, uint32_t off) {
    if constexpr (sizeof(S) == 4) return base + off;
    else return reinterpret_cast<S*>(reinterpret_cast<char*>(base) + (uint32_t)(off * (uint32_t)sizeof(S)));
}
template <bool NT, class S>
__device__ __forceinline__ S ldg(const S* base, uint32_t off) {
    const S* p = at(base, off);
    if constexpr (NT) return __builtin_nontemporal_load(p);
    else return *p;
}
template <bool NT, class S>
__device__ __forceinline__ void stg(S* base, uint32_t off, S v) {
    S* p = at(base, off);
    if constexpr (NT) __builtin_nontemporal_store(v, p);
    else *p = v;
}

// Offset, within one direction of a distribution in g's layout, of the site
// s + (dx, dy, dz), each of dx, dy, dz in {-1, 0, 1}.  Everything is formed
// from the coordinates and g's own strides, so one Site can address arrays
// of different layouts (a source and a destination).
template <int DX, int DY, int DZ>
__device__ __forceinline__ uint32_t offset_at(const Site& s, const Geo& g) {
    const uint32_t xx = (uint32_t)(DX == 0 ? s.x : (DX > 0 ? s.xp : s.xm));
    const int yy = DY == 0 ? s.y : (DY > 0 ? s.yp : s.ym);
    const int zz = DZ == 0 ? s.z : (DZ > 0 ? s.zp : s.zm);
    return (uint32_t)zz * g.zs + (uint32_t)yy * g.ys + (xx >> 6) * g.xbs + (xx & 63u);
}

// Canonical site index x + nx (y + ny z) of s + (dx, dy, dz): the index of
// scalar fields and of caller arrays.
template <int DX, int DY, int DZ>
__device__ __forceinline__ uint32_t canon_at(const Site& s, const Geo& g) {
    const int xx = DX == 0 ? s.x : (DX > 0 ? s.xp : s.xm);
    const int yy = DY == 0 ? s.y : (DY > 0 ? s.yp : s.ym);
    const int zz = DZ == 0 ? s.z : (DZ > 0 ? s.zp : s.zm);
    return (uint32_t)zz * g.plane + (uint32_t)yy * (uint32_t)g.nx + (uint32_t)xx;
}

// Offset of the upstream site s - c_i (pull) or of s itself (local).
template <int I, bool GATHER>
__device__ __forceinline__ uint32_t src_offset(const Site& s, const Geo& g) {
    if constexpr (GATHER) return offset_at<-cx(I), -cy(I), -cz(I)>(s, g);
    else return offset_at<0, 0, 0>(s, g);
}

// Compile-time loop over the 19 directions.
template <int I, int N, class F>
__device__ __forceinline__ void static_for(F&& f) {
    if constexpr (I < N) {
        f(std::integral_constant<int, I>{});
        static_for<I + 1, N>(f);
    }
}

}  // namespace lbk
