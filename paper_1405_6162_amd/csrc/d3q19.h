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

template <class T>
__host__ __device__ constexpr T weight(int i) {
    return csq(i) == 0 ? T(1) / T(3) : (csq(i) == 1 ? T(1) / T(18) : T(1) / T(36));
}

// Compute type for each storage type: FP64 storage computes in FP64, the
// reduced-precision storages compute in FP32.
template <class S> struct Compute;
template <> struct Compute<double>   { using T = double; };
template <> struct Compute<float>    { using T = float; };
template <> struct Compute<_Float16> { using T = float; };

template <class T, class S> __device__ __forceinline__ T load_as(const S* p) { return static_cast<T>(*p); }
template <class S, class T> __device__ __forceinline__ void store_as(S* p, T v) { *p = static_cast<S>(v); }

// Lattice geometry.  Site offsets fit in 32 bits (N < 2^31 is checked on
// the host); direction offsets (i * dstride) are 64-bit.
struct Geo {
    int nx, ny, nz;
    uint32_t plane;     // nx * ny
    uint32_t nsite;     // nx * ny * nz
    int64_t dstride;    // elements between consecutive direction arrays
};

// Launch tile: one site per lane, 64 x 4 sites of one z plane per block, so a
// wavefront covers 64 consecutive x and every direction array is read and
// written in 512-byte (FP64) contiguous runs.
constexpr int TX = 64;
constexpr int TY = 4;
constexpr int TPB = TX * TY;

// Coordinates of this lane's site and of its +-1 neighbours (periodic).
struct Site {
    int x, y, z, xm, xp, ym, yp, zm, zp;
    bool active;
};

__device__ __forceinline__ Site site_of_thread(const Geo& g) {
    Site s;
    s.x = blockIdx.x * TX + threadIdx.x;
    s.y = blockIdx.y * TY + threadIdx.y;
    s.z = blockIdx.z;
    s.active = (s.x < g.nx) && (s.y < g.ny);
    s.xm = s.x == 0 ? g.nx - 1 : s.x - 1;
    s.xp = s.x + 1 >= g.nx ? 0 : s.x + 1;
    s.ym = s.y == 0 ? g.ny - 1 : s.y - 1;
    s.yp = s.y + 1 >= g.ny ? 0 : s.y + 1;
    s.zm = s.z == 0 ? g.nz - 1 : s.z - 1;
    s.zp = s.z + 1 >= g.nz ? 0 : s.z + 1;
    return s;
}

// Offset of the site s + (dx, dy, dz), each of dx, dy, dz in {-1, 0, 1}.
template <int DX, int DY, int DZ>
__device__ __forceinline__ uint32_t offset_at(const Site& s, const Geo& g) {
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
