// C ABI of the gfx950 D3Q19 lattice-Boltzmann library: argument checks,
// workspace carving, the direct/pending state machine and kernel launches on
// the caller's stream.  See include/lb.h for the contract of every call.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdlib>
#include <cstring>
#include <mutex>
#include <new>
#include <type_traits>
#include <vector>

#include "../../include/lb.h"
#include "kernels.h"

using namespace lbk;

namespace {

// Launch policy of every kernel in the library but the single-pass binary
// step (below): 64 x 4 sites per block, one site per lane, nontemporal
// stores (the next step reads the values from HBM anyway), XCD-ordered
// tiles.  Chosen by a sweep over tile shapes, sites per lane (1, 2, 4),
// nontemporal loads/stores and direction padding on 128^3 and 256^3
// lattices; the differences were within 5%.
using Pol = Tiling<64, 4, 1, false, true, true>;
// The same with 2 and 4 sites per lane along z (lb_params.vvl).
using Pol2 = Tiling<64, 4, 2, false, true, true>;
using Pol4 = Tiling<64, 4, 4, false, true, true>;
// Single-pass binary step (k_binary_march), per storage type: the tile and
// whether the next plane's g waits in LDS or in registers.  A 64 x 8 tile
// has 144 halo sites per 512 against 136 per 256 for 64 x 4, so the halo's
// phi gathers (mostly re-reads of neighbouring tiles' g) fall from 53% to
// 28% of the sites gathered: measured A/B on one box, 64 x 8 is 6.5% faster
// than 64 x 4 in FP64 at 256^3, 2% at 128^3, 3% in FP32 and 1% in FP16;
// 64 x 16 and 32 x 16 were slower in every storage.  In FP32 and FP16 a
// 128 x 4 tile (W), which has half the x-halo sites (whose gathers each hit
// a cache line of their own, 2 or 4 bytes used), is faster again: 3% in
// FP16 at 256^3 and 384^3, 0.8-1.5% in FP32 (FP64: 0.4% slower; 128 x 8
// slower in FP16); it is used where its 128-site rows leave no more lanes
// idle than 64-site rows (nx mod 128 is 0 or above 64).  g waits in
// registers in FP64 (1% faster than LDS at 256^3) and FP32, in LDS in FP16
// (30% faster than registers at 384^3; as FP16 values no faster than as
// FP32).
template <class S> struct March;
template <> struct March<double> {
    using P = Tiling<64, 8, 1, false, true, true>;
    using W = P;
    static constexpr bool glds = false;
};
template <> struct March<float> {
    using P = Tiling<64, 8, 1, false, true, true>;
    using W = Tiling<128, 4, 1, false, true, true>;
    static constexpr bool glds = false;
};
template <> struct March<_Float16> {
    using P = Tiling<64, 8, 1, false, true, true>;
    using W = Tiling<128, 4, 1, false, true, true>;
    static constexpr bool glds = true;
};
// Chunks of the march: each chunk's first and last plane cost one extra
// plane of phi (2/depth more g reads), while deeper chunks leave fewer blocks.
// Two 512-lane march blocks fit a CU, so kMarchSlots blocks run at once.
// Where 64-plane chunks give more blocks than that, the depth is 64 (64
// against 32 planes 0.8% faster in FP64 at 256^3, 1.5% in FP32, 1% at 320^3,
// equal at 384^3).  Otherwise nz is cut into as many chunks as fill one round
// of slots, at least nz/64 and at most nz/16 of them (rounded up).  Measured
// A/B against the fixed depths of 64, 32 or 16 planes it replaced: 8-12%
// faster at 160^3 (480 blocks of 20 planes instead of 600 of 16) and 4-9% at
// 192^3 (504 of 28 instead of 432 of 32) in FP64, FP32 and FP16, 1% slower at
// 176^3.  The kernel cuts nz evenly where the blocks are remapped to XCDs
// (block count a multiple of 8), else into chunks of the depth and a shorter
// last one.
constexpr int kMarchSlots = 512;

constexpr size_t kAlign = 4096;
// Extra bytes between consecutive direction arrays, so the 19 (38) streams of
// a power-of-two lattice do not start on the same HBM channel (measured:
// 0 B padding is 5-10% slower than the best offsets; 9472 B = 37 x 256 B was
// among the best on 128^3 and 256^3).
constexpr size_t kDirPadBytes = 9472;

size_t round_up(size_t v, size_t a) { return (v + a - 1) / a * a; }

size_t storage_size(int storage) { return storage == LB_F64 ? 8 : (storage == LB_F32 ? 4 : 2); }
size_t compute_size(int storage) { return storage == LB_F64 ? 8 : 4; }

struct Layout {
    int64_t nsite;
    int64_t dstride;        // elements between consecutive directions
    bool blocked;           // 64-site blocks holding their 19 directions together
    uint32_t zs, ys, xbs;   // site-offset strides (Geo)
    size_t dist_bytes;      // one 19-direction buffer
    size_t phi_bytes;
    int nblocks;
    size_t partial_bytes;
    size_t off_f[2], off_g[2], off_phi, off_partial, total;
};

int check_params(const lb_params* p) {
    if (!p) return LB_EINVAL;
    if (p->nx < 1 || p->ny < 1 || p->nz < 1) return LB_EINVAL;
    const int64_t n = (int64_t)p->nx * p->ny * p->nz;
    // Kernels form byte offsets of FP64 arrays in 32 bits: N * 8 < 2^32.
    if (n >= ((int64_t)1 << 29)) return LB_EINVAL;
    if (p->model != LB_SINGLE && p->model != LB_BINARY) return LB_EINVAL;
    if (p->storage != LB_F64 && p->storage != LB_F32 && p->storage != LB_F16) return LB_EINVAL;
    if (p->vvl != 0 && p->vvl != 1 && p->vvl != 2 && p->vvl != 4) return LB_EINVAL;
    if (p->binary_step < LB_STEP_AUTO || p->binary_step > LB_STEP_TWO_PASS) return LB_EINVAL;
    if (p->collision != LB_BGK && p->collision != LB_TRT && p->collision != LB_MRT) return LB_EINVAL;
    auto valid_tau = [](double t) { return std::isfinite(t) && t > 0.5; };
    if (p->collision != LB_BGK && !valid_tau(p->tau_minus)) return LB_EINVAL;
    if (p->collision == LB_MRT &&
        (!valid_tau(p->tau_bulk) || !valid_tau(p->tau_ghost_even) || !valid_tau(p->tau_ghost_odd)))
        return LB_EINVAL;
    if (!std::isfinite(p->tau_f) || !(p->tau_f > 0.5)) return LB_EINVAL;
    if (p->model == LB_BINARY) {
        if (!std::isfinite(p->A) || !std::isfinite(p->B) || !std::isfinite(p->kappa)) return LB_EINVAL;
        if (!(p->kappa >= 0.0)) return LB_EINVAL;
        if (!std::isfinite(p->mobility) || !(p->mobility > 0.0)) return LB_EINVAL;
        if (!std::isfinite(p->gamma) || !(p->gamma > 0.0)) return LB_EINVAL;
    }
    if (!std::isfinite(p->rho0) || !std::isfinite(p->phi0)) return LB_EINVAL;
    return LB_OK;
}

Layout layout_of(const lb_params* p) {
    Layout L{};
    L.nsite = (int64_t)p->nx * p->ny * p->nz;
    const size_t es = storage_size(p->storage);
    // Blocked layout (see Geo) whenever a buffer's offsets fit in 32 bits
    // (in bytes; for 4-byte elements, which are addressed by element, in
    // elements);
    // the last x block of a row is padded to 64 sites.  Measured A/B on one
    // box against the structure-of-arrays layout: the single-fluid step
    // +4.6% (FP64) and +5.6% (FP32) at 256^3, the binary march +4.3% (FP64,
    // 256^3), +3.0% (FP64, 128^3), +3.6% (FP16, 384^3) and +2.5 to +5.6%
    // (FP32, 128^3 to 256^3); padding between the buffers changed none of
    // these.
    const uint64_t xblocks = (uint64_t)tiles(p->nx, 64);
    const uint64_t blocked_elems = (uint64_t)p->nz * (uint64_t)p->ny * xblocks * Q * 64;
    L.blocked = (es == 4 ? blocked_elems : blocked_elems * es) < ((uint64_t)1 << 32);
    if (L.blocked) {
        L.dstride = 64;
        L.xbs = Q * 64;
        L.ys = (uint32_t)(xblocks * L.xbs);
        L.zs = (uint32_t)((uint64_t)p->ny * L.ys);
        L.dist_bytes = round_up((size_t)blocked_elems * es, kAlign);
    } else {
        const size_t stride_bytes = round_up((size_t)L.nsite * es, kAlign) + kDirPadBytes;
        L.dstride = (int64_t)(stride_bytes / es);
        L.xbs = 64;
        L.ys = (uint32_t)p->nx;
        L.zs = (uint32_t)p->nx * (uint32_t)p->ny;
        L.dist_bytes = round_up(stride_bytes * Q, kAlign);
    }
    L.phi_bytes = round_up((size_t)L.nsite * compute_size(p->storage), kAlign);
    L.nblocks = tiles(p->nx, Pol::TX) * tiles(p->ny, Pol::TY) * tiles(p->nz, Pol::TZ);
    L.partial_bytes = round_up((size_t)L.nblocks * 16 * sizeof(double), kAlign);
    size_t o = 0;
    for (int b = 0; b < 2; ++b) { L.off_f[b] = o; o += L.dist_bytes; }
    if (p->model == LB_BINARY) {
        for (int b = 0; b < 2; ++b) { L.off_g[b] = o; o += L.dist_bytes; }
        L.off_phi = o; o += L.phi_bytes;
    } else {
        L.off_g[0] = L.off_g[1] = L.off_phi = 0;
    }
    L.off_partial = o; o += L.partial_bytes;
    L.total = o;
    return L;
}

struct Rec { int kind; hipEvent_t start, stop; };

}  // namespace

// Partial sums of lb_conserved_sums_noalloc (8 doubles per block).  In host
// code this name is only a stand-in for the symbol: kernels get the device
// address that hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) double scratch[8 * (size_t)LB_NOALLOC_MAX_BLOCKS];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mutex;
double* scratch_ptr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (each device holds its own copy of the array).
int scratch_on_current_device(double** out) {
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= kMaxDevices) return LB_EDEVICE;
    std::lock_guard<std::mutex> lock(scratch_mutex);
    if (!scratch_ptr[dev]) {
        double* ptr = nullptr;
        if (hipGetSymbolAddress((void**)&ptr, HIP_SYMBOL(scratch)) != hipSuccess || !ptr) return LB_EDEVICE;
        scratch_ptr[dev] = ptr;
    }
    *out = scratch_ptr[dev];
    return LB_OK;
}

}  // namespace

struct lb_ctx {
    lb_params p;
    Layout L;
    hipStream_t stream;
    char* ws;
    int cur;          // buffer index holding the state
    bool pending;     // true: the state is propagate(buffer[cur])
    bool profiling;
    unsigned profile_kinds;   // bit k: time launches of kernel class k
    bool launched;    // any device work queued (lb_destroy waits for it)
    std::vector<Rec> recs;
    std::vector<hipEvent_t> pool;

    Geo geo() const {
        Geo g;
        g.nx = p.nx; g.ny = p.ny; g.nz = p.nz;
        g.plane = (uint32_t)p.nx * (uint32_t)p.ny;
        g.nsite = (uint32_t)L.nsite;
        g.dstride = L.dstride;
        g.gx = tiles(p.nx, Pol::TX);
        g.gy = tiles(p.ny, Pol::TY);
        g.gz = tiles(p.nz, Pol::TZ);
        g.nblocks = g.gx * g.gy * g.gz;
        g.zs = L.zs; g.ys = L.ys; g.xbs = L.xbs;
        g.bz = Pol::TZ;
        return g;
    }
    // g with the layout of canonical caller arrays: direction stride N, x fastest
    Geo canonical(Geo g) const {
        g.dstride = L.nsite;
        g.zs = g.plane; g.ys = (uint32_t)p.nx; g.xbs = 64;
        return g;
    }
    Geo canonical_geo() const { return canonical(geo()); }
    template <class P>
    Geo geo_for() const {
        Geo g = geo();
        g.gz = tiles(p.nz, P::TZ);
        g.nblocks = g.gx * g.gy * g.gz;
        return g;
    }
    template <class MP>
    Geo march_geo() const {
        Geo g = geo();
        g.gx = tiles(p.nx, MP::TX);
        g.gy = tiles(p.ny, MP::TY);
        const int col = g.gx * g.gy;
        if (col * tiles(p.nz, 64) > kMarchSlots) {
            g.bz = 64;
        } else {
            const int chunks = std::min(tiles(p.nz, 16), std::max(tiles(p.nz, 64), kMarchSlots / col));
            g.bz = tiles(p.nz, chunks);
        }
        g.gz = tiles(p.nz, g.bz);
        g.nblocks = g.gx * g.gy * g.gz;
        return g;
    }
    dim3 grid() const { return dim3(L.nblocks); }
    static dim3 block() { return dim3(Pol::TPB); }
    void* fbuf(int b) const { return ws + L.off_f[b]; }
    void* gbuf(int b) const { return p.model == LB_BINARY ? ws + L.off_g[b] : nullptr; }
    void* phi() const { return ws + L.off_phi; }
    double* partial() const { return reinterpret_cast<double*>(ws + L.off_partial); }

    // Timing-only events.  An ordinary event record ends with a system-scope
    // fence (cache write-back and invalidation); between two dependent
    // launches of the 128^3 binary step with profiling on, the rocprofv3
    // kernel trace shows 11 us gaps with it and 8.5 us without.  Without it
    // the profiled 64^3 adjoint rollout runs 12% faster and the 128^3 binary
    // step 1%.  The events are only
    // ever read by lb_kernel_times.
    hipEvent_t take_event() {
        if (!pool.empty()) { hipEvent_t e = pool.back(); pool.pop_back(); return e; }
        hipEvent_t e = nullptr;
        if (hipEventCreateWithFlags(&e, hipEventDisableSystemFence) != hipSuccess) return nullptr;
        return e;
    }
    void release_records() {
        for (auto& r : recs) { pool.push_back(r.start); pool.push_back(r.stop); }
        recs.clear();
    }
};

namespace {

// Brackets one launch with an event pair when profiling is on.
struct Timed {
    lb_ctx* c; int kind; hipEvent_t a = nullptr, b = nullptr;
    Timed(lb_ctx* c_, int kind_) : c(c_), kind(kind_) {
        if (c->profiling && ((c->profile_kinds >> kind) & 1u)) {
            a = c->take_event(); b = c->take_event();
            if (a && b) (void)hipEventRecord(a, c->stream);
        }
    }
    ~Timed() {
        if (a && b) {
            (void)hipEventRecord(b, c->stream);
            c->recs.push_back({kind, a, b});
        } else {
            if (a) c->pool.push_back(a);
            if (b) c->pool.push_back(b);
        }
    }
};

int launch_status() { return hipGetLastError() == hipSuccess ? LB_OK : LB_EDEVICE; }



template <class S>
CollParams<typename Compute<S>::T> coll_params(const lb_ctx* c) {
    using T = typename Compute<S>::T;
    CollParams<T> cp;
    cp.omega_f = (T)(1.0 / c->p.tau_f);
    const double tau_g = c->p.model == LB_BINARY ? c->p.mobility / c->p.gamma + 0.5 : 1.0;
    cp.omega_g = (T)(1.0 / tau_g);
    cp.A = (T)c->p.A; cp.B = (T)c->p.B; cp.kappa = (T)c->p.kappa; cp.gamma = (T)c->p.gamma;
    const bool dev = c->p.storage != LB_F64;
    cp.rho0 = dev ? (T)c->p.rho0 : T(0);
    cp.phi0 = dev ? (T)c->p.phi0 : T(0);
    cp.omega_m = c->p.collision != LB_BGK ? (T)(1.0 / c->p.tau_minus) : cp.omega_f;
    const bool mrt = c->p.collision == LB_MRT;
    cp.omega_b = mrt ? (T)(1.0 / c->p.tau_bulk) : cp.omega_f;
    cp.omega_ge = mrt ? (T)(1.0 / c->p.tau_ghost_even) : cp.omega_f;
    cp.omega_go = mrt ? (T)(1.0 / c->p.tau_ghost_odd) : cp.omega_m;
    return cp;
}

// ----- typed launchers ------------------------------------------------------

// Calls fn with the launch policy of the context's sites per lane.
template <class F>
int by_vvl(const lb_ctx* c, F&& fn) {
    switch (c->p.vvl) {
        case 0: case 1: return fn(Pol{});
        case 2: return fn(Pol2{});
        case 4: return fn(Pol4{});
    }
    return LB_EINVAL;
}

template <class S>
int run_phi(lb_ctx* c) {
    using T = typename Compute<S>::T;
    Timed t(c, LB_K_PHI);
    const S* g = (const S*)c->gbuf(c->cur);
    const T phi0 = coll_params<S>(c).phi0;
    by_vvl(c, [&](auto pol) {
        using P = decltype(pol);
        const Geo geo = c->template geo_for<P>();
        if (c->pending) k_phi<P, S, true><<<geo.nblocks, P::TPB, 0, c->stream>>>(g, (T*)c->phi(), geo, phi0);
        else k_phi<P, S, false><<<geo.nblocks, P::TPB, 0, c->stream>>>(g, (T*)c->phi(), geo, phi0);
        return 0;
    });
    return launch_status();
}

// One collision of the logical state; on return the state is direct.
// Single-pass binary step from a pending buffer; on return the state is direct.
template <class S>
int run_binary_march(lb_ctx* c) {
    using MP = typename March<S>::P;
    using MW = typename March<S>::W;
    const auto cp = coll_params<S>(c);
    const int src = c->cur, dst = 1 - c->cur;
    const bool wide = tiles(c->p.nx, MW::TX) * MW::TX == tiles(c->p.nx, MP::TX) * MP::TX;
    auto launch = [&](auto tiling) {
        using TP = decltype(tiling);
        const Geo g = c->template march_geo<TP>();
        Timed t(c, LB_K_COLLIDE);
        const dim3 grid(g.nblocks), block(TP::TPB);
        const S* fs = (const S*)c->fbuf(src);
        const S* gs = (const S*)c->gbuf(src);
        S* fd = (S*)c->fbuf(dst);
        S* gd = (S*)c->gbuf(dst);
        auto go = [&](auto coll, auto blk) {
            constexpr int COLL = decltype(coll)::value;
            constexpr bool BLK = decltype(blk)::value;
            k_binary_march<TP, S, March<S>::glds, 3, false, COLL, BLK><<<grid, block, 0, c->stream>>>(fs, gs, fd, gd, g, cp);
        };
        auto by_coll = [&](auto blk) {
            if (c->p.collision == LB_TRT) go(std::integral_constant<int, COLL_TRT>{}, blk);
            else if (c->p.collision == LB_MRT) go(std::integral_constant<int, COLL_MRT>{}, blk);
            else go(std::integral_constant<int, COLL_BGK>{}, blk);
        };
        if (c->L.blocked) by_coll(std::true_type{});
        else by_coll(std::false_type{});
    };
    if (wide) launch(MW{});
    else launch(MP{});
    int rc = launch_status();
    if (rc) return rc;
    c->cur = dst;
    c->pending = false;
    return LB_OK;
}

// The single-pass march runs one block per tile column and chunk, each
// marching its planes in sequence, so on small lattices it has too few blocks
// to hide its per-plane latency: 64^3 FP64 (32 blocks) took 122 us a step
// against 39 us for the two-pass step (phi pass + fused collide, every site in
// parallel), 96^3 (144 blocks) 142 against 136 us, 112^3 (196 blocks) 198
// against 204 us and 128^3 (256 blocks) 248 against 301 us; FP32 and FP16
// cross over between 112^3 and 128^3.  With LB_STEP_AUTO the march runs from
// kMarchMinBlocks blocks (one per CU) up.  The two paths give the same bits.
constexpr int kMarchMinBlocks = 256;

template <class S>
bool march_pays(const lb_ctx* c) {
    if (c->p.binary_step == LB_STEP_MARCH) return true;
    if (c->p.binary_step == LB_STEP_TWO_PASS) return false;
    return c->template march_geo<typename March<S>::P>().nblocks >= kMarchMinBlocks;
}

template <class S>
int run_collide(lb_ctx* c) {
    using T = typename Compute<S>::T;
    const bool bin = c->p.model == LB_BINARY;
    if (bin && c->pending && march_pays<S>(c)) return run_binary_march<S>(c);
    if (bin) { int rc = run_phi<S>(c); if (rc) return rc; }
    const auto cp = coll_params<S>(c);
    const int src = c->cur, dst = c->pending ? 1 - c->cur : c->cur;
    const S* fs = (const S*)c->fbuf(src); S* fd = (S*)c->fbuf(dst);
    const S* gs = (const S*)c->gbuf(src); S* gd = (S*)c->gbuf(dst);
    const T* phi = (const T*)c->phi();
    {
        Timed t(c, LB_K_COLLIDE);
        by_vvl(c, [&](auto pol) {
            using P = decltype(pol);
            const Geo geo = c->template geo_for<P>();
            const dim3 grid(geo.nblocks), block(P::TPB);
            if (bin && c->p.collision == LB_TRT) {
                if (c->pending) k_collide<P, MODEL_BINARY, S, true, COLL_TRT><<<grid, block, 0, c->stream>>>(fs, gs, fd, gd, phi, geo, cp);
                else k_collide<P, MODEL_BINARY, S, false, COLL_TRT><<<grid, block, 0, c->stream>>>(fs, gs, fd, gd, phi, geo, cp);
            } else if (bin && c->p.collision == LB_MRT) {
                if (c->pending) k_collide<P, MODEL_BINARY, S, true, COLL_MRT><<<grid, block, 0, c->stream>>>(fs, gs, fd, gd, phi, geo, cp);
                else k_collide<P, MODEL_BINARY, S, false, COLL_MRT><<<grid, block, 0, c->stream>>>(fs, gs, fd, gd, phi, geo, cp);
            } else if (bin) {
                if (c->pending) k_collide<P, MODEL_BINARY, S, true><<<grid, block, 0, c->stream>>>(fs, gs, fd, gd, phi, geo, cp);
                else k_collide<P, MODEL_BINARY, S, false><<<grid, block, 0, c->stream>>>(fs, gs, fd, gd, phi, geo, cp);
            } else if (c->p.collision == LB_TRT) {
                if (c->pending) k_collide<P, MODEL_SINGLE, S, true, COLL_TRT><<<grid, block, 0, c->stream>>>(fs, gs, fd, gd, phi, geo, cp);
                else k_collide<P, MODEL_SINGLE, S, false, COLL_TRT><<<grid, block, 0, c->stream>>>(fs, gs, fd, gd, phi, geo, cp);
            } else if (c->p.collision == LB_MRT) {
                if (c->pending) k_collide<P, MODEL_SINGLE, S, true, COLL_MRT><<<grid, block, 0, c->stream>>>(fs, gs, fd, gd, phi, geo, cp);
                else k_collide<P, MODEL_SINGLE, S, false, COLL_MRT><<<grid, block, 0, c->stream>>>(fs, gs, fd, gd, phi, geo, cp);
            } else {
                if (c->pending) k_collide<P, MODEL_SINGLE, S, true><<<grid, block, 0, c->stream>>>(fs, gs, fd, gd, phi, geo, cp);
                else k_collide<P, MODEL_SINGLE, S, false><<<grid, block, 0, c->stream>>>(fs, gs, fd, gd, phi, geo, cp);
            }
            return 0;
        });
    }
    int rc = launch_status();
    if (rc) return rc;
    c->cur = dst;
    c->pending = false;
    return LB_OK;
}

// Materialise propagate(buffer[src]) into (f, g) of layout dgeo.
template <class S>
int run_stream_into(lb_ctx* c, int src, S* f, S* g, const Geo& dgeo) {
    Timed t(c, LB_K_STREAM);
    if (c->p.model == LB_BINARY)
        k_stream2<Pol, S><<<c->grid(), c->block(), 0, c->stream>>>((const S*)c->fbuf(src), (const S*)c->gbuf(src), f,
                                                                   g, c->geo(), dgeo);
    else
        k_stream<Pol, S><<<c->grid(), c->block(), 0, c->stream>>>((const S*)c->fbuf(src), f, c->geo(), dgeo);
    return launch_status();
}

// Copy a state (f, and g for the binary model) from layout sgeo to layout
// dgeo, site by site (the context's layout <-> canonical caller memory).
template <class S>
int run_convert(lb_ctx* c, const S* fs, const S* gs, S* fd, S* gd, const Geo& sgeo, const Geo& dgeo) {
    if (c->p.model == LB_BINARY)
        k_stream2<Pol, S, false><<<c->grid(), c->block(), 0, c->stream>>>(fs, gs, fd, gd, sgeo, dgeo);
    else
        k_stream<Pol, S, false><<<c->grid(), c->block(), 0, c->stream>>>(fs, fd, sgeo, dgeo);
    return launch_status();
}

template <class S>
int run_propagate(lb_ctx* c) {
    if (!c->pending) { c->pending = true; return LB_OK; }   // propagation of a direct buffer is deferred
    const int dst = 1 - c->cur;
    int rc = run_stream_into<S>(c, c->cur, (S*)c->fbuf(dst), (S*)c->gbuf(dst), c->geo());
    if (rc) return rc;
    c->cur = dst;
    return LB_OK;
}

template <class S>
int run_step(lb_ctx* c, int32_t n) {
    for (int32_t k = 0; k < n; ++k) {
        int rc = run_collide<S>(c);
        if (rc) return rc;
        c->pending = true;
    }
    return LB_OK;
}

template <class S>
int run_init(lb_ctx* c, const double* rho, const double* u, const double* phi) {
    Timed t(c, LB_K_OTHER);
    CollParams<double> cp;
    const auto ct = coll_params<S>(c);
    cp.omega_f = ct.omega_f; cp.omega_g = ct.omega_g;
    cp.A = c->p.A; cp.B = c->p.B; cp.kappa = c->p.kappa; cp.gamma = c->p.gamma;
    cp.rho0 = c->p.storage == LB_F64 ? 0.0 : c->p.rho0;
    cp.phi0 = c->p.storage == LB_F64 ? 0.0 : c->p.phi0;
    S* f = (S*)c->fbuf(c->cur);
    S* g = (S*)c->gbuf(c->cur);
    if (c->p.model == LB_BINARY) k_init<Pol, MODEL_BINARY, S><<<c->grid(), c->block(), 0, c->stream>>>(rho, u, phi, f, g, c->geo(), cp);
    else k_init<Pol, MODEL_SINGLE, S><<<c->grid(), c->block(), 0, c->stream>>>(rho, u, phi, f, g, c->geo(), cp);
    int rc = launch_status();
    if (rc == LB_OK) c->pending = false;
    return rc;
}

template <class S>
int run_moments(lb_ctx* c, double* rho, double* u, double* phi) {
    Timed t(c, LB_K_OTHER);
    const double r0 = c->p.storage == LB_F64 ? 0.0 : c->p.rho0;
    const double p0 = c->p.storage == LB_F64 ? 0.0 : c->p.phi0;
    const S* f = (const S*)c->fbuf(c->cur);
    const S* g = (const S*)c->gbuf(c->cur);
    const dim3 grid = c->grid(), block = c->block();
    if (c->p.model == LB_BINARY) {
        if (c->pending) k_moments<Pol, MODEL_BINARY, S, true><<<grid, block, 0, c->stream>>>(f, g, rho, u, phi, c->geo(), r0, p0);
        else k_moments<Pol, MODEL_BINARY, S, false><<<grid, block, 0, c->stream>>>(f, g, rho, u, phi, c->geo(), r0, p0);
    } else {
        if (c->pending) k_moments<Pol, MODEL_SINGLE, S, true><<<grid, block, 0, c->stream>>>(f, g, rho, u, nullptr, c->geo(), r0, p0);
        else k_moments<Pol, MODEL_SINGLE, S, false><<<grid, block, 0, c->stream>>>(f, g, rho, u, nullptr, c->geo(), r0, p0);
    }
    return launch_status();
}

template <class S>
int run_sums(lb_ctx* c, double* out) {
    Timed t(c, LB_K_OTHER);
    const S* f = (const S*)c->fbuf(c->cur);
    const S* g = (const S*)c->gbuf(c->cur);
    if (c->p.model == LB_BINARY) k_sums_partial<Pol, MODEL_BINARY, S><<<c->grid(), c->block(), 0, c->stream>>>(f, g, c->geo(), c->partial());
    else k_sums_partial<Pol, MODEL_SINGLE, S><<<c->grid(), c->block(), 0, c->stream>>>(f, g, c->geo(), c->partial());
    const bool dev = c->p.storage != LB_F64;
    const double n = (double)c->L.nsite;
    const double b0 = dev ? n * c->p.rho0 : 0.0;
    const double b4 = (dev && c->p.model == LB_BINARY) ? n * c->p.phi0 : 0.0;
    k_sums_final<Pol, 5><<<1, c->block(), 0, c->stream>>>(c->partial(), c->L.nblocks, out, b0, b4, 0);
    return launch_status();
}

template <class S>
int run_get_state(lb_ctx* c, S* f, S* g) {
    if (c->pending) return run_stream_into<S>(c, c->cur, f, g, c->canonical_geo());
    Timed t(c, LB_K_OTHER);
    return run_convert<S>(c, (const S*)c->fbuf(c->cur), (const S*)c->gbuf(c->cur), f, g, c->geo(),
                          c->canonical_geo());
}

template <class S>
int run_set_state(lb_ctx* c, const S* f, const S* g) {
    Timed t(c, LB_K_OTHER);
    const int rc = run_convert<S>(c, f, g, (S*)c->fbuf(c->cur), (S*)c->gbuf(c->cur), c->canonical_geo(), c->geo());
    if (rc) return rc;
    c->pending = false;
    return LB_OK;
}

// nsteps single-fluid steps whose post-collision fields go to post[k] (canonical
// stride N); afterwards the state is pending on a copy of the last of them.
// Binary: step k writes post-collision f then g at post + k*38*N.  Step 0
// collides the context's state in its own buffers and copies the result out;
// later steps march from post[k-1] to post[k] (both of direction stride N).
template <class S>
int run_step_record_binary(lb_ctx* c, int32_t n, S* post, typename Compute<S>::T* phi) {
    using T = typename Compute<S>::T;
    const int64_t N = c->L.nsite;
    const auto cp = coll_params<S>(c);
    if (phi) {                                        // phi of the state step 0 collides
        Timed t(c, LB_K_PHI);
        const S* g = (const S*)c->gbuf(c->cur);
        if (c->pending) k_phi<Pol, S, true><<<c->grid(), c->block(), 0, c->stream>>>(g, phi, c->geo(), cp.phi0);
        else k_phi<Pol, S, false><<<c->grid(), c->block(), 0, c->stream>>>(g, phi, c->geo(), cp.phi0);
    }
    int rc = run_collide<S>(c);                       // state now direct: the post-collision field
    if (rc) return rc;
    {
        Timed t(c, LB_K_OTHER);
        rc = run_convert<S>(c, (const S*)c->fbuf(c->cur), (const S*)c->gbuf(c->cur), post, post + Q * N, c->geo(),
                            c->canonical_geo());
        if (rc) return rc;
    }
    c->pending = true;
    using MP = typename March<S>::P;
    const Geo g = c->canonical(c->template march_geo<MP>());
    const bool march = march_pays<S>(c);
    Geo cg = c->canonical_geo();
    for (int32_t k = 1; k < n; ++k) {
        const S* src = post + (size_t)(k - 1) * 2 * Q * N;
        S* dst = post + (size_t)k * 2 * Q * N;
        if (!march) {
            // two-pass: phi of the recorded state, then the fused collide, both on stride N
            T* ph = phi ? phi + (size_t)k * N : (T*)c->phi();
            {
                Timed t(c, LB_K_PHI);
                k_phi<Pol, S, true><<<c->grid(), c->block(), 0, c->stream>>>(src + Q * N, ph, cg, cp.phi0);
            }
            {
                Timed t(c, LB_K_COLLIDE);
                if (c->p.collision == LB_TRT)
                    k_collide<Pol, MODEL_BINARY, S, true, COLL_TRT><<<c->grid(), c->block(), 0, c->stream>>>(
                        src, src + Q * N, dst, dst + Q * N, ph, cg, cp);
                else if (c->p.collision == LB_MRT)
                    k_collide<Pol, MODEL_BINARY, S, true, COLL_MRT><<<c->grid(), c->block(), 0, c->stream>>>(
                        src, src + Q * N, dst, dst + Q * N, ph, cg, cp);
                else
                    k_collide<Pol, MODEL_BINARY, S, true><<<c->grid(), c->block(), 0, c->stream>>>(
                        src, src + Q * N, dst, dst + Q * N, ph, cg, cp);
            }
            rc = launch_status();
            if (rc) return rc;
            continue;
        }
        {
            Timed t(c, LB_K_COLLIDE);
            const dim3 grid(g.nblocks), block(MP::TPB);
            auto go = [&](auto coll) {
                constexpr int COLL = decltype(coll)::value;
                if (phi)
                    k_binary_march<MP, S, March<S>::glds, 3, true, COLL><<<grid, block, 0, c->stream>>>(
                        src, src + Q * N, dst, dst + Q * N, g, cp, phi + (size_t)k * N);
                else
                    k_binary_march<MP, S, March<S>::glds, 3, false, COLL><<<grid, block, 0, c->stream>>>(
                        src, src + Q * N, dst, dst + Q * N, g, cp);
            };
            if (c->p.collision == LB_TRT) go(std::integral_constant<int, COLL_TRT>{});
            else if (c->p.collision == LB_MRT) go(std::integral_constant<int, COLL_MRT>{});
            else go(std::integral_constant<int, COLL_BGK>{});
        }
        rc = launch_status();
        if (rc) return rc;
    }
    if (n > 1) {
        Timed t(c, LB_K_OTHER);
        const S* last = post + (size_t)(n - 1) * 2 * Q * N;
        rc = run_convert<S>(c, last, last + Q * N, (S*)c->fbuf(c->cur), (S*)c->gbuf(c->cur), c->canonical_geo(),
                            c->geo());
        if (rc) return rc;
    }
    return LB_OK;
}

template <class S>
int run_step_record(lb_ctx* c, int32_t n, S* post, typename Compute<S>::T* phi) {
    if (c->p.model == LB_BINARY) return run_step_record_binary<S>(c, n, post, phi);
    const int64_t N = c->L.nsite;
    const auto cp = coll_params<S>(c);
    const dim3 grid = c->grid(), block = c->block();
    // one collision from src (layout sg; pull from a pending src when GATHER)
    // into canonical dst, for the context's collision
    const Geo cg = c->canonical_geo();
    auto collide = [&](auto gather, const S* src, const Geo& sg, S* dst) {
        constexpr bool G = decltype(gather)::value;
        if (c->p.collision == LB_TRT)
            k_collide_single_strided<Pol, S, G, COLL_TRT><<<grid, block, 0, c->stream>>>(src, dst, sg, cg, cp);
        else if (c->p.collision == LB_MRT)
            k_collide_single_strided<Pol, S, G, COLL_MRT><<<grid, block, 0, c->stream>>>(src, dst, sg, cg, cp);
        else
            k_collide_single_strided<Pol, S, G><<<grid, block, 0, c->stream>>>(src, dst, sg, cg, cp);
    };
    for (int32_t k = 0; k < n; ++k) {
        S* dst = post + (size_t)k * Q * N;
        {
            Timed t(c, LB_K_COLLIDE);
            if (k == 0) {
                const S* src = (const S*)c->fbuf(c->cur);
                if (c->pending) collide(std::true_type{}, src, c->geo(), dst);
                else collide(std::false_type{}, src, c->geo(), dst);
            } else {
                collide(std::true_type{}, post + (size_t)(k - 1) * Q * N, cg, dst);
            }
        }
        int rc = launch_status();
        if (rc) return rc;
    }
    Timed t(c, LB_K_OTHER);
    const int rc = run_convert<S>(c, post + (size_t)(n - 1) * Q * N, nullptr, (S*)c->fbuf(c->cur), nullptr, cg,
                                  c->geo());
    if (rc) return rc;
    c->pending = true;
    return LB_OK;
}

template <class S>
int run_sites(lb_ctx* c, const int32_t* index, int64_t m, S* f, S* g, bool set) {
    Timed t(c, LB_K_OTHER);
    const int nb = (int)((m + CB - 1) / CB);
    const Geo geo = c->geo();
    S* bufs[2] = {(S*)c->fbuf(c->cur), (S*)c->gbuf(c->cur)};
    S* packs[2] = {f, g};
    for (int d = 0; d < (c->p.model == LB_BINARY ? 2 : 1); ++d) {
        if (set) {
            if (c->pending) k_set_sites<S, true><<<nb, CB, 0, c->stream>>>(bufs[d], index, m, packs[d], geo);
            else k_set_sites<S, false><<<nb, CB, 0, c->stream>>>(bufs[d], index, m, packs[d], geo);
        } else {
            if (c->pending) k_get_sites<S, true><<<nb, CB, 0, c->stream>>>(bufs[d], index, m, packs[d], geo);
            else k_get_sites<S, false><<<nb, CB, 0, c->stream>>>(bufs[d], index, m, packs[d], geo);
        }
    }
    return launch_status();
}

// Dispatch on the storage type.
template <class F>
int by_storage(lb_ctx* c, F&& fn) {
    c->launched = true;
    switch (c->p.storage) {
        case LB_F64: return fn((double*)nullptr);
        case LB_F32: return fn((float*)nullptr);
        case LB_F16: return fn((_Float16*)nullptr);
    }
    return LB_EINVAL;
}

}  // namespace

namespace {

// True when two device ranges [a, a + na) and [b, b + nb) (in doubles) overlap.
bool overlaps(const double* a, size_t na, const double* b, size_t nb) {
    if (!a || !b) return false;
    return a < b + nb && b < a + na;
}

template <int LG>
void launch_adjoint_binary_local(lb_ctx* c, bool pending, const double* f, const double* g, const double* phi,
                                 const double* lf_next, const double* lg_next, const double* b_next, double* lf_n,
                                 double* p_out, double* afield, const Geo& geo, const CollParams<double>& cp) {
    // 32-bit byte offsets from one base per array when every array of 19
    // directions fits below 4 GiB (lattices up to about 300^3)
    const bool off32 = (uint64_t)Q * (uint64_t)geo.dstride * sizeof(double) <= ((uint64_t)1 << 32);
    auto go = [&](auto coll, auto o32) {
        constexpr int COLL = decltype(coll)::value;
        constexpr bool OFF32 = decltype(o32)::value;
        if (pending)
            k_adjoint_binary<Pol, true, LG, COLL, OFF32><<<c->grid(), c->block(), 0, c->stream>>>(
                f, g, phi, lf_next, lg_next, b_next, lf_n, p_out, afield, c->partial(), geo, cp);
        else
            k_adjoint_binary<Pol, false, LG, COLL, OFF32><<<c->grid(), c->block(), 0, c->stream>>>(
                f, g, phi, lf_next, lg_next, b_next, lf_n, p_out, afield, c->partial(), geo, cp);
    };
    auto by_coll = [&](auto o32) {
        if (c->p.collision == LB_TRT) go(std::integral_constant<int, COLL_TRT>{}, o32);
        else if (c->p.collision == LB_MRT) go(std::integral_constant<int, COLL_MRT>{}, o32);
        else go(std::integral_constant<int, COLL_BGK>{}, o32);
    };
    if (off32) by_coll(std::true_type{});
    else by_coll(std::false_type{});
}

// Gradient sums of a binary adjoint step: dL/domega_f, dL/domega_g,
// dL/dkappa; for TRT and MRT then dL/domega_minus (omega_f being the even,
// or shear, rate and omega_minus the odd, or flux, one); for MRT then the
// bulk, even-ghost and odd-ghost rates.
int binary_adjoint_grad_count(const lb_ctx* c) {
    return c->p.collision == LB_MRT ? 7 : (c->p.collision == LB_TRT ? 4 : 3);
}

// The stencil kernel of a binary adjoint step, with block 0 adding the
// local kernel's partials (one per gradient sum) into grads.
template <bool B_ONLY>
void launch_adjoint_binary_stencil(lb_ctx* c, const double* afield, const double* lg_next, double* out,
                                   const Geo& geo, double omega_g, double* grads) {
    const int ng = binary_adjoint_grad_count(c);
    if (ng == 7)
        k_adjoint_binary_stencil<Pol, B_ONLY, 7><<<c->grid(), c->block(), 0, c->stream>>>(
            afield, lg_next, out, geo, omega_g, c->partial(), c->L.nblocks, grads);
    else if (ng == 4)
        k_adjoint_binary_stencil<Pol, B_ONLY, 4><<<c->grid(), c->block(), 0, c->stream>>>(
            afield, lg_next, out, geo, omega_g, c->partial(), c->L.nblocks, grads);
    else
        k_adjoint_binary_stencil<Pol, B_ONLY, 3><<<c->grid(), c->block(), 0, c->stream>>>(
            afield, lg_next, out, geo, omega_g, c->partial(), c->L.nblocks, grads);
}

// Rate sums an adjoint step of the single fluid accumulates: 1 (BGK), 2
// (TRT) or 5 (MRT), in the order of lb_params' relaxation times.
int adjoint_rate_count(const lb_ctx* c) {
    return c->p.collision == LB_MRT ? 5 : (c->p.collision == LB_TRT ? 2 : 1);
}

// One single-fluid adjoint kernel launch writing its block partials to
// `partial`; with prev given, its block 0 also accumulates the previous
// step's partials into domega.
template <bool PEND, int COLL>
void adjoint_single_launch(lb_ctx* c, const double* f, const double* lam_next, double* lam_n, const Geo& geo,
                           const CollParams<double>& cp, double* partial, const double* prev, double* domega) {
    Timed t(c, LB_K_ADJOINT);
    k_adjoint<Pol, PEND, COLL><<<c->grid(), c->block(), 0, c->stream>>>(f, lam_next, lam_n, partial, geo, cp, prev,
                                                                        c->L.nblocks, domega);
}

template <int COLL>
void adjoint_single_sums(lb_ctx* c, const double* partial, double* domega) {
    k_sums_final<Pol, AdjointRates<COLL>::K><<<1, c->block(), 0, c->stream>>>(partial, c->L.nblocks, domega, 0.0,
                                                                               0.0, 1);
}

// One single-fluid adjoint step for the context's collision.  sums_now: the
// step's rate sums are reduced into domega by a separate launch right away;
// otherwise they stay in `partial` for the next step (prev) or the caller.
void adjoint_single_step(lb_ctx* c, const double* f, bool pending, const double* lam_next, double* lam_n,
                         const Geo& geo, const CollParams<double>& cp, double* partial, const double* prev,
                         double* domega, bool sums_now) {
    auto go = [&](auto coll) {
        constexpr int COLL = decltype(coll)::value;
        if (pending) adjoint_single_launch<true, COLL>(c, f, lam_next, lam_n, geo, cp, partial, prev, domega);
        else adjoint_single_launch<false, COLL>(c, f, lam_next, lam_n, geo, cp, partial, prev, domega);
        if (sums_now) adjoint_single_sums<COLL>(c, partial, domega);
    };
    if (c->p.collision == LB_TRT) go(std::integral_constant<int, COLL_TRT>{});
    else if (c->p.collision == LB_MRT) go(std::integral_constant<int, COLL_MRT>{});
    else go(std::integral_constant<int, COLL_BGK>{});
}

// The rate sums left in `partial` by the last step of a sweep.
void adjoint_single_flush(lb_ctx* c, const double* partial, double* domega) {
    if (c->p.collision == LB_TRT) adjoint_single_sums<COLL_TRT>(c, partial, domega);
    else if (c->p.collision == LB_MRT) adjoint_single_sums<COLL_MRT>(c, partial, domega);
    else adjoint_single_sums<COLL_BGK>(c, partial, domega);
}

}  // namespace

extern "C" {

int lb_workspace_bytes(const lb_params* p, size_t* bytes) {
    if (!bytes) return LB_EINVAL;
    int rc = check_params(p);
    if (rc) return rc;
    *bytes = layout_of(p).total;
    return LB_OK;
}

int lb_create(const lb_params* p, void* workspace, size_t workspace_bytes, void* stream, lb_ctx** out) {
    if (!out) return LB_EINVAL;
    *out = nullptr;
    int rc = check_params(p);
    if (rc) return rc;
    if (!workspace || ((uintptr_t)workspace % 256) != 0) return LB_EINVAL;
    const Layout L = layout_of(p);
    if (workspace_bytes < L.total) return LB_ENOMEM;
    lb_ctx* c = new (std::nothrow) lb_ctx();
    if (!c) return LB_ENOMEM;
    c->p = *p;
    c->L = L;
    c->stream = (hipStream_t)stream;
    c->ws = (char*)workspace;
    c->cur = 0;
    c->pending = false;
    c->profiling = false;
    c->profile_kinds = 0;
    c->launched = false;
    *out = c;
    return LB_OK;
}

int lb_set_stream(lb_ctx* c, void* stream) {
    if (!c) return LB_EINVAL;
    c->stream = (hipStream_t)stream;
    return LB_OK;
}

int lb_init_equilibrium(lb_ctx* c, const double* rho, const double* u, const double* phi) {
    if (!c || !rho || !u) return LB_EINVAL;
    if (c->p.model == LB_BINARY && !phi) return LB_EINVAL;
    return by_storage(c, [&](auto tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        return run_init<S>(c, rho, u, phi);
    });
}

int lb_collide(lb_ctx* c) {
    if (!c) return LB_EINVAL;
    return by_storage(c, [&](auto tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        return run_collide<S>(c);
    });
}

int lb_propagate(lb_ctx* c) {
    if (!c) return LB_EINVAL;
    return by_storage(c, [&](auto tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        return run_propagate<S>(c);
    });
}

int lb_step(lb_ctx* c, int32_t nsteps) {
    if (!c || nsteps < 0) return LB_EINVAL;
    if (nsteps == 0) return LB_OK;
    return by_storage(c, [&](auto tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        return run_step<S>(c, nsteps);
    });
}

int lb_moments(lb_ctx* c, double* rho, double* u, double* phi) {
    if (!c) return LB_EINVAL;
    if (phi && c->p.model != LB_BINARY) return LB_EINVAL;
    if (!rho && !u && !phi) return LB_OK;
    return by_storage(c, [&](auto tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        return run_moments<S>(c, rho, u, phi);
    });
}

int lb_conserved_sums(lb_ctx* c, double* out) {
    if (!c || !out) return LB_EINVAL;
    return by_storage(c, [&](auto tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        return run_sums<S>(c, out);
    });
}

int lb_conserved_sums_noalloc(const lb_params* p, const void* f, const void* g, double* out, void* stream) {
    if (!p || !f || !out) return LB_EINVAL;
    int rc = check_params(p);
    if (rc) return rc;
    if ((p->model == LB_BINARY) != (g != nullptr)) return LB_EINVAL;
    // the launch of lb_conserved_sums, on the canonical layout
    Geo geo;
    geo.nx = p->nx; geo.ny = p->ny; geo.nz = p->nz;
    geo.plane = (uint32_t)p->nx * (uint32_t)p->ny;
    geo.nsite = geo.plane * (uint32_t)p->nz;
    geo.dstride = geo.nsite;
    geo.zs = geo.plane; geo.ys = (uint32_t)p->nx; geo.xbs = 64;
    geo.gx = tiles(p->nx, Pol::TX);
    geo.gy = tiles(p->ny, Pol::TY);
    geo.gz = tiles(p->nz, Pol::TZ);
    geo.bz = Pol::TZ;
    const int64_t nblocks = (int64_t)geo.gx * geo.gy * geo.gz;
    if (nblocks > LB_NOALLOC_MAX_BLOCKS) return LB_ERANGE;
    geo.nblocks = (int)nblocks;
    double* partial = nullptr;
    rc = scratch_on_current_device(&partial);
    if (rc) return rc;
    const hipStream_t s = (hipStream_t)stream;
    const bool dev = p->storage != LB_F64;
    const double n = (double)geo.nsite;
    const double b0 = dev ? n * p->rho0 : 0.0;
    const double b4 = (dev && p->model == LB_BINARY) ? n * p->phi0 : 0.0;
    auto launch = [&](auto tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        if (p->model == LB_BINARY)
            k_sums_partial<Pol, MODEL_BINARY, S><<<geo.nblocks, Pol::TPB, 0, s>>>((const S*)f, (const S*)g, geo, partial);
        else
            k_sums_partial<Pol, MODEL_SINGLE, S><<<geo.nblocks, Pol::TPB, 0, s>>>((const S*)f, nullptr, geo, partial);
        k_sums_final<Pol, 5><<<1, Pol::TPB, 0, s>>>(partial, geo.nblocks, out, b0, b4, 0);
        return launch_status();
    };
    if (p->storage == LB_F64) return launch((double*)nullptr);
    if (p->storage == LB_F32) return launch((float*)nullptr);
    return launch((_Float16*)nullptr);
}

int lb_field_stats(lb_ctx* c, double* out) {
    if (!c || !out) return LB_EINVAL;
    return by_storage(c, [&](auto tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        Timed t(c, LB_K_OTHER);
        const S* f = (const S*)c->fbuf(c->cur);
        const S* g = (const S*)c->gbuf(c->cur);
        const bool dev = c->p.storage != LB_F64;
        const double r0 = dev ? c->p.rho0 : 0.0, p0 = dev ? c->p.phi0 : 0.0;
        const Geo geo = c->geo();
        const bool bin = c->p.model == LB_BINARY;
        if (bin && c->pending)
            k_stats_partial<Pol, MODEL_BINARY, S, true><<<c->grid(), c->block(), 0, c->stream>>>(f, g, geo, r0, p0, c->partial());
        else if (bin)
            k_stats_partial<Pol, MODEL_BINARY, S, false><<<c->grid(), c->block(), 0, c->stream>>>(f, g, geo, r0, p0, c->partial());
        else if (c->pending)
            k_stats_partial<Pol, MODEL_SINGLE, S, true><<<c->grid(), c->block(), 0, c->stream>>>(f, g, geo, r0, p0, c->partial());
        else
            k_stats_partial<Pol, MODEL_SINGLE, S, false><<<c->grid(), c->block(), 0, c->stream>>>(f, g, geo, r0, p0, c->partial());
        k_stats_final<Pol><<<1, c->block(), 0, c->stream>>>(c->partial(), c->L.nblocks, out, bin ? 1 : 0);
        return launch_status();
    });
}

int lb_get_state(lb_ctx* c, void* f, void* g) {
    if (!c || !f) return LB_EINVAL;
    if ((c->p.model == LB_BINARY) != (g != nullptr)) return LB_EINVAL;
    return by_storage(c, [&](auto tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        return run_get_state<S>(c, (S*)f, (S*)g);
    });
}

int lb_set_state(lb_ctx* c, const void* f, const void* g) {
    if (!c || !f) return LB_EINVAL;
    if ((c->p.model == LB_BINARY) != (g != nullptr)) return LB_EINVAL;
    return by_storage(c, [&](auto tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        return run_set_state<S>(c, (const S*)f, (const S*)g);
    });
}

int lb_set_tau(lb_ctx* c, double tau_f) {
    if (!c || !std::isfinite(tau_f) || !(tau_f > 0.5)) return LB_EINVAL;
    c->p.tau_f = tau_f;
    return LB_OK;
}

int lb_step_record(lb_ctx* c, int32_t nsteps, void* post, void* phi) {
    if (!c || nsteps < 0) return LB_EINVAL;
    if (phi && c->p.model != LB_BINARY) return LB_EINVAL;
    if (nsteps == 0) return LB_OK;
    if (!post) return LB_EINVAL;
    return by_storage(c, [&](auto tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        return run_step_record<S>(c, nsteps, (S*)post, (typename Compute<S>::T*)phi);
    });
}

int lb_set_params(lb_ctx* c, const lb_params* p) {
    if (!c || !p) return LB_EINVAL;
    int rc = check_params(p);
    if (rc) return rc;
    const lb_params& q = c->p;
    if (p->nx != q.nx || p->ny != q.ny || p->nz != q.nz || p->model != q.model || p->storage != q.storage ||
        p->vvl != q.vvl || p->collision != q.collision || p->binary_step != q.binary_step || p->rho0 != q.rho0 ||
        p->phi0 != q.phi0)
        return LB_EINVAL;
    c->p = *p;
    return LB_OK;
}

int lb_adjoint_step_binary(lb_ctx* c, const double* f, const double* g, const double* phi_n, int pending,
                           const double* lf_next, const double* lg_next, double* lf_n, double* lg_n,
                           double* grads) {
    if (!c || !f || !g || !lf_next || !lg_next || !lf_n || !lg_n || !grads) return LB_EINVAL;
    if (c->p.model != LB_BINARY || c->p.storage != LB_F64) return LB_ENOTSUP;
    const double* outs[2] = {lf_n, lg_n};
    const double* ins[5] = {f, g, lf_next, lg_next, phi_n};
    for (const double* o : outs)
        for (const double* i : ins)
            if (o == i) return LB_EINVAL;
    if (lf_n == lg_n) return LB_EINVAL;
    c->launched = true;
    const Geo geo = c->canonical_geo();
    const auto cp = coll_params<double>(c);
    const double* phi = phi_n;
    double* afield = (double*)c->fbuf(1 - c->cur);       // spare state buffer: >= 19 N doubles, 5 N used
    if (!phi) {
        Timed t(c, LB_K_ADJOINT);
        double* p = (double*)c->phi();
        if (pending) k_phi<Pol, double, true><<<c->grid(), c->block(), 0, c->stream>>>(g, p, geo, 0.0);
        else k_phi<Pol, double, false><<<c->grid(), c->block(), 0, c->stream>>>(g, p, geo, 0.0);
        phi = p;
    }
    {
        Timed t(c, LB_K_ADJOINT);
        launch_adjoint_binary_local<LG_GATHER>(c, pending != 0, f, g, phi, lf_next, lg_next, nullptr, lf_n, nullptr,
                                               afield, geo, cp);
    }
    {
        Timed t(c, LB_K_ADJOINT);
        launch_adjoint_binary_stencil<false>(c, afield, lg_next, lg_n, geo, cp.omega_g, grads);
    }
    return launch_status();
}

int lb_adjoint_init_binary(lb_ctx* c, const double* rho, const double* u, const double* phi, const double* lf0,
                           const double* lg0, double* dphi, double* drho, double* du, double* dkappa) {
    if (!c || !rho || !u || !phi || !lf0 || !lg0 || !dphi || !drho || !du || !dkappa) return LB_EINVAL;
    if (c->p.model != LB_BINARY || c->p.storage != LB_F64) return LB_ENOTSUP;
    c->launched = true;
    const Geo geo = c->canonical_geo();
    const auto cp = coll_params<double>(c);
    double* afield = (double*)c->fbuf(1 - c->cur);
    {
        Timed t(c, LB_K_ADJOINT);
        k_adjoint_binary_init<Pol><<<c->grid(), c->block(), 0, c->stream>>>(rho, u, phi, lf0, lg0, afield, drho, du,
                                                                           c->partial(), geo, cp);
        k_adjoint_binary_stencil<Pol, true, 1><<<c->grid(), c->block(), 0, c->stream>>>(
            afield, nullptr, dphi, geo, 1.0, c->partial(), c->L.nblocks, dkappa);
    }
    return launch_status();
}

int lb_adjoint_step(lb_ctx* c, const double* f, int f_pending, const double* lam_next, double* lam_n,
                    double* domega) {
    if (!c || !f || !lam_next || !lam_n || !domega) return LB_EINVAL;
    if (c->p.model != LB_SINGLE || c->p.storage != LB_F64) return LB_ENOTSUP;
    if (lam_n == lam_next || lam_n == f) return LB_EINVAL;
    c->launched = true;
    adjoint_single_step(c, f, f_pending != 0, lam_next, lam_n, c->canonical_geo(), coll_params<double>(c),
                        c->partial(), nullptr, domega, true);
    return launch_status();
}

int lb_adjoint_segment(lb_ctx* c, const double* f0, const double* post, int32_t length, double* lam, double* work,
                       double* domega) {
    if (!c || !f0 || !lam || !work || !domega || length < 1) return LB_EINVAL;
    if (length > 1 && !post) return LB_EINVAL;
    if (c->p.model != LB_SINGLE || c->p.storage != LB_F64) return LB_ENOTSUP;
    const size_t n19 = (size_t)Q * c->L.nsite;
    const size_t npost = length > 1 ? (size_t)(length - 1) * n19 : 0;
    const size_t nw = (size_t)adjoint_rate_count(c);
    if (overlaps(lam, n19, work, n19) || overlaps(lam, n19, f0, n19) || overlaps(work, n19, f0, n19) ||
        overlaps(lam, n19, post, npost) || overlaps(work, n19, post, npost) || overlaps(domega, nw, lam, n19) ||
        overlaps(domega, nw, work, n19) || overlaps(domega, nw, f0, n19) || overlaps(domega, nw, post, npost))
        return LB_EINVAL;
    c->launched = true;
    const Geo geo = c->canonical_geo();
    const auto cp = coll_params<double>(c);
    double* cur = lam;            // lambda^{n+1}
    double* nxt = work;
    // two partial arrays in the context's partial buffer (16 doubles per
    // block, each step using slots 8 b + k of one half): step k's block 0
    // reduces step k-1's half while the other blocks fill its own
    double* halves[2] = {c->partial(), c->partial() + 8 * (size_t)c->L.nblocks};
    const double* prev = nullptr;
    for (int32_t n = length - 1, k = 0; n >= 0; --n, ++k) {
        double* part = halves[k & 1];
        const double* fn = n > 0 ? post + (size_t)(n - 1) * n19 : f0;
        adjoint_single_step(c, fn, n > 0, cur, nxt, geo, cp, part, prev, domega, false);
        prev = part;
        std::swap(cur, nxt);
    }
    adjoint_single_flush(c, prev, domega);
    if (cur != lam) {
        Timed t(c, LB_K_OTHER);
        if (hipMemcpyAsync(lam, cur, n19 * sizeof(double), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
            return LB_EDEVICE;
    }
    return launch_status();
}

int lb_adjoint_segment_binary(lb_ctx* c, const double* f0, const double* g0, const double* post, const double* phi,
                              int32_t length, double* lf, double* lg, double* work, double* grads) {
    if (!c || !f0 || !g0 || !lf || !lg || !work || !grads || length < 1) return LB_EINVAL;
    if (length > 1 && !post) return LB_EINVAL;
    if (c->p.model != LB_BINARY || c->p.storage != LB_F64) return LB_ENOTSUP;
    const size_t N = c->L.nsite, n19 = (size_t)Q * N;
    const size_t ng = (size_t)binary_adjoint_grad_count(c);
    const size_t npost = length > 1 ? (size_t)(length - 1) * 2 * n19 : 0;
    const size_t nphi = phi && length > 1 ? (size_t)(length - 1) * N : 0;
    struct R { const double* p; size_t n; };
    const R outs[3] = {{lf, n19}, {lg, n19}, {work, 2 * n19}};
    const R all[8] = {{lf, n19}, {lg, n19}, {work, 2 * n19}, {f0, n19}, {g0, n19}, {post, npost}, {phi, nphi},
                      {grads, ng}};
    for (int o = 0; o < 3; ++o)                      // all[o] is outs[o]
        for (int a = 0; a < 8; ++a)
            if (a != o && overlaps(outs[o].p, outs[o].n, all[a].p, all[a].n)) return LB_EINVAL;
    if (overlaps(grads, ng, f0, n19) || overlaps(grads, ng, g0, n19) || overlaps(grads, ng, post, npost))
        return LB_EINVAL;
    c->launched = true;
    const Geo geo = c->canonical_geo();
    const auto cp = coll_params<double>(c);
    double* afield = (double*)c->fbuf(1 - c->cur);   // spare state buffer: >= 19 N doubles, 6 N used
    double* bfield = afield + 5 * N;
    double* lf_cur = lf;                              // lambda_f^{n+1}
    double* lf_nxt = work;
    double* p_cur = lg;                               // lambda_g^{n+1} (first step) or P^{n+1}
    double* p_nxt = work + n19;
    for (int32_t n = length - 1; n >= 0; --n) {
        Timed t(c, LB_K_ADJOINT);
        const bool pending = n > 0;
        const double* fn = pending ? post + (size_t)(n - 1) * 2 * n19 : f0;
        const double* gn = pending ? fn + n19 : g0;
        const double* ph = (phi && n < length - 1) ? phi + (size_t)n * N : nullptr;
        if (!ph) {
            double* p = (double*)c->phi();
            if (pending) k_phi<Pol, double, true><<<c->grid(), c->block(), 0, c->stream>>>(gn, p, geo, 0.0);
            else k_phi<Pol, double, false><<<c->grid(), c->block(), 0, c->stream>>>(gn, p, geo, 0.0);
            ph = p;
        }
        if (n == length - 1)
            launch_adjoint_binary_local<LG_GATHER_KEEP>(c, pending, fn, gn, ph, lf_cur, p_cur, nullptr, lf_nxt,
                                                        p_nxt, afield, geo, cp);
        else
            launch_adjoint_binary_local<LG_PULLED_KEEP>(c, pending, fn, gn, ph, lf_cur, p_cur, bfield, lf_nxt,
                                                        p_nxt, afield, geo, cp);
        launch_adjoint_binary_stencil<true>(c, afield, nullptr, bfield, geo, 1.0, grads);
        std::swap(lf_cur, lf_nxt);
        std::swap(p_cur, p_nxt);
    }
    {
        // lambda_g^{s0} = (1 - omega_g) P^{s0} + b^{s0}, into lg (in place when P^{s0} is there)
        Timed t(c, LB_K_ADJOINT);
        k_adjoint_binary_combine<Pol><<<c->grid(), c->block(), 0, c->stream>>>(p_cur, bfield, lg, geo, cp.omega_g);
    }
    if (lf_cur != lf) {
        Timed t(c, LB_K_OTHER);
        if (hipMemcpyAsync(lf, lf_cur, n19 * sizeof(double), hipMemcpyDeviceToDevice, c->stream) != hipSuccess)
            return LB_EDEVICE;
    }
    return launch_status();
}

int lb_mask_index(lb_ctx* c, const uint8_t* mask, int32_t* index, int64_t* count) {
    if (!c || !mask || !index || !count) return LB_EINVAL;
    c->launched = true;
    const uint32_t n = (uint32_t)c->L.nsite;
    const int nb = (int)((n + CB - 1) / CB);
    int64_t* counts = reinterpret_cast<int64_t*>(c->partial());   // nb <= tiles of the launch grid
    Timed t(c, LB_K_OTHER);
    k_mask_count<<<nb, CB, 0, c->stream>>>(mask, n, counts);
    k_scan_counts<<<1, CB, 0, c->stream>>>(counts, nb, count);
    k_mask_scatter<<<nb, CB, 0, c->stream>>>(mask, n, counts, index);
    return launch_status();
}


int lb_get_sites(lb_ctx* c, const int32_t* index, int64_t m, void* f, void* g) {
    if (!c || m < 0 || m > c->L.nsite) return LB_EINVAL;
    if (m == 0) return LB_OK;
    if (!index || !f || ((c->p.model == LB_BINARY) != (g != nullptr))) return LB_EINVAL;
    return by_storage(c, [&](auto tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        return run_sites<S>(c, index, m, (S*)f, (S*)g, false);
    });
}

int lb_set_sites(lb_ctx* c, const int32_t* index, int64_t m, const void* f, const void* g) {
    if (!c || m < 0 || m > c->L.nsite) return LB_EINVAL;
    if (m == 0) return LB_OK;
    if (!index || !f || ((c->p.model == LB_BINARY) != (g != nullptr))) return LB_EINVAL;
    return by_storage(c, [&](auto tag) {
        using S = std::remove_pointer_t<decltype(tag)>;
        return run_sites<S>(c, index, m, (S*)f, (S*)g, true);
    });
}

int lb_profile_mask(lb_ctx* c, unsigned kinds) {
    if (!c || (kinds >> (LB_K_OTHER + 1)) != 0) return LB_EINVAL;
    if (kinds) {
        if (hipStreamSynchronize(c->stream) != hipSuccess) return LB_EDEVICE;
        c->release_records();
    }
    c->profiling = kinds != 0;
    c->profile_kinds = kinds;
    return LB_OK;
}

int lb_profile(lb_ctx* c, int enable) {
    return lb_profile_mask(c, enable ? (1u << (LB_K_OTHER + 1)) - 1u : 0u);
}

int lb_kernel_times(lb_ctx* c, int kind, double* total_ms, int64_t* launches) {
    if (!c || !total_ms || !launches || kind < 0 || kind > LB_K_OTHER) return LB_EINVAL;
    double ms = 0.0;
    int64_t n = 0;
    for (auto& r : c->recs) {
        if (r.kind != kind) continue;
        if (hipEventSynchronize(r.stop) != hipSuccess) return LB_EDEVICE;
        float e = 0.0f;
        if (hipEventElapsedTime(&e, r.start, r.stop) != hipSuccess) return LB_EDEVICE;
        ms += e;
        ++n;
    }
    *total_ms = ms;
    *launches = n;
    return LB_OK;
}

int lb_destroy(lb_ctx* c) {
    if (!c) return LB_OK;
    int rc = LB_OK;
    if (c->launched && hipStreamSynchronize(c->stream) != hipSuccess) rc = LB_EDEVICE;
    c->release_records();
    for (hipEvent_t e : c->pool) (void)hipEventDestroy(e);
    delete c;
    return rc;
}

int lb_stream_copy(void* dst, const void* src, size_t bytes, void* stream) {
    if (bytes == 0) return LB_OK;
    if (!dst || !src) return LB_EINVAL;
    const uintptr_t d = reinterpret_cast<uintptr_t>(dst), s = reinterpret_cast<uintptr_t>(src);
    if (d % 16 != 0 || s % 16 != 0 || bytes % 16 != 0) return LB_EINVAL;
    if (d < s + bytes && s < d + bytes) return LB_EINVAL;
    const uint64_t nwords = bytes / 16;
    const uint64_t per_block = (uint64_t)COPY_TPB * COPY_U;
    const uint64_t nblocks = (nwords + per_block - 1) / per_block;
    if (nblocks > 0x7fffffffull) return LB_EINVAL;
    k_stream_copy<<<(unsigned)nblocks, COPY_TPB, 0, (hipStream_t)stream>>>(
        static_cast<const u32x4*>(src), static_cast<u32x4*>(dst), nwords);
    return launch_status();
}

const char* lb_strerror(int status) {
    switch (status) {
        case LB_OK: return "ok";
        case LB_EINVAL: return "invalid argument";
        case LB_ENOMEM: return "workspace too small";
        case LB_EDEVICE: return "HIP runtime or kernel launch failure";
        case LB_ENOTSUP: return "not supported for this model or storage";
        case LB_ERANGE: return "lattice too large for the fixed scratch of an allocation-free call";
    }
    return "unknown status";
}

}  // extern "C"
