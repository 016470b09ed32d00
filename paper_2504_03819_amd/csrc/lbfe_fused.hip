// Fused collide + stream + next-step moments of one time step on gfx950
// (Eqs. (10), (11), (21)-(26), (28), (32); halfway bounce-back at the walls).
//
// The step's population traffic is one read and one write of the 27
// populations per node: besides colliding and streaming its nodes, each
// workgroup forms the density and momentum of the next step, rho(t+1) =
// sum_i f*_i(x - c_i) and j(t+1) = sum_i c_i f*_i(x - c_i), and mu0(rho(t+1))
// for the stencil chain of the next step, so no separate pass reads the
// streamed populations back.
//
// Tile: TX x TY owned columns plus a one-node ring, marching in z over a
// chunk of planes.  Per source plane s:
//   1. every ring-inclusive node (one per lane) collides the populations it
//      prefetched during the previous plane, issues the loads of plane s+1,
//      and writes its 27 post-collision values, in their storage encoding,
//      to one LDS plane [27][(TX+2)(TY+2)];
//   2. every owned column (x, y) reads from LDS the 27 values that arrive
//      from plane s at (x, y) in the destination planes s-1, s, s+1
//      (f*_i(x - c_i)), stores them to the output lattice as aligned rows,
//      and adds them to the destination planes' moment sums (three
//      destination planes in flight in registers; plane s-1 is complete
//      once source plane s has been added).
// The ring nodes are collided by the neighbouring tiles too (ring overhead
// (TX+2)(TY+2)/(TX TY) - 1); their populations mostly come from L2, since
// consecutive tiles run on one XCD.  The moments are summed in the order of
// moments() (lbfe_device.h), so rho, j and mu0 are bit for bit those of the
// separate moments pass over the stored lattice.
#include <type_traits>

#include "lbfe_device.h"

namespace lbfe {
namespace {

// Raw buffer access to one z-plane of a row-blocked lattice or of a [z][y][x]
// field: the plane's base goes into a buffer descriptor (scalar registers),
// every access takes a 32-bit per-lane byte offset plus a uniform slot
// offset, so the 27 population addresses of a node cost no vector
// registers.  A lane with offset kOOB (past the plane) reads 0 and stores
// nothing.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr unsigned kOOB = 0x80000000u;
constexpr int kPopStore = 2;  // population stores non-temporal (read only by the next step)
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void *base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}
__device__ inline double bld(double *, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
}
__device__ inline float bld(float *, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
}
__device__ inline __half bld(__half *, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    return __builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
}
template <int POL = 0> __device__ inline void bst(double x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, v, s, POL);
}
template <int POL = 0> __device__ inline void bst(float x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, v, s, POL);
}
template <int POL = 0> __device__ inline void bst(__half x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, v, s, POL);
}

// Storage encoding of one population value (a store then a load of the
// lattice returns dec(enc(v))) and the plane geometry of the row-blocked
// lattice: NS slots of nx values per x-row, S bytes each; with f0 in FP32 the
// rest population lives in a float [z][y][x] array after the half rows.
template <int P> struct Code {
    using st = float;
    static constexpr unsigned S = 4, NS = 27;
    __device__ static st enc(int, float v) { return v; }
    __device__ static float dec(int, st v) { return v; }
    __device__ static int slot(int i) { return i; }
};
template <> struct Code<LBFE_FP64> {
    using st = double;
    static constexpr unsigned S = 8, NS = 27;
    __device__ static st enc(int, double v) { return v; }
    __device__ static double dec(int, st v) { return v; }
    __device__ static int slot(int i) { return i; }
};
template <> struct Code<LBFE_FP16_DEV> {
    using st = __half;
    static constexpr unsigned S = 2, NS = 27;
    __device__ static st enc(int i, float v) { return enc16(i, v); }
    __device__ static float dec(int i, st v) { return dec16(i, v); }
    __device__ static int slot(int i) { return i; }
};
template <> struct Code<LBFE_FP16_DEV_F0FP32> {
    using st = __half;
    static constexpr unsigned S = 2, NS = 26;
    __device__ static st enc(int i, float v) { return enc16(i, v); }
    __device__ static float dec(int i, st v) { return dec16(i, v); }
    __device__ static int slot(int i) { return i < kRest ? i : i - 1; }
};

// One z-plane of a lattice: the half / real rows and, with f0 in FP32, the
// rest-population plane.
template <int P> struct LatPlane {
    using C = Code<P>;
    __amdgpu_buffer_rsrc_t r, r0;
    unsigned nxS;  // bytes per slot run
    __device__ LatPlane(const void *base, const KP &kp, int z) {
        const size_t rows = (size_t)C::NS * C::S * kp.plane;  // bytes of one plane's rows
        nxS = (unsigned)kp.nx * C::S;
        r = rsrc((const char *)base + (size_t)z * rows, (unsigned)rows);
        if constexpr (P == LBFE_FP16_DEV_F0FP32) {
            const size_t h = (26 * 2 * (size_t)kp.N + 255) & ~size_t(255);
            r0 = rsrc((const char *)base + h + (size_t)z * 4 * kp.plane, 4u * kp.plane);
        } else {
            r0 = r;
        }
    }
    // vo: byte offset of the node's row position, (y NS nx + x) S; vo0: of
    // the node in the rest-population plane, (y nx + x) 4
    __device__ typename Pol<P>::real ld(int i, unsigned vo, unsigned vo0) const {
        if constexpr (P == LBFE_FP16_DEV_F0FP32) {
            if (i == kRest) return bld((float *)nullptr, r0, vo0, 0);
        }
        return C::dec(i, bld((typename C::st *)nullptr, r, vo, (unsigned)C::slot(i) * nxS));
    }
};

// One LDS plane of post-collision values in their storage encoding.  With
// f0 in FP32 the rest population sits in a float array of its own.
template <int P, int NR> struct Plane {
    using C = Code<P>;
    using real = typename Pol<P>::real;
    typename C::st v[27][NR];
    __device__ void put(int i, int k, real x) { v[i][k] = C::enc(i, x); }
    __device__ real get(int i, int k) const { return C::dec(i, v[i][k]); }
    // raw encoded value i of LDS node k to slot `slot` of the lattice node
    // at byte offsets (vo, vo0) of plane L
    __device__ void store(const LatPlane<P> &L, int slot, int i, int k, unsigned vo, unsigned) const {
        bst<kPopStore>(v[i][k], L.r, vo, (unsigned)slot * L.nxS);
    }
};
template <int NR> struct Plane<LBFE_FP16_DEV_F0FP32, NR> {
    using C = Code<LBFE_FP16_DEV_F0FP32>;
    __half v[27][NR];  // slot kRest unused
    float r0[NR];
    __device__ void put(int i, int k, float x) {
        if (i == kRest)
            r0[k] = x;
        else
            v[i][k] = enc16(i, x);
    }
    __device__ float get(int i, int k) const { return i == kRest ? r0[k] : dec16(i, v[i][k]); }
    __device__ void store(const LatPlane<LBFE_FP16_DEV_F0FP32> &L, int slot, int i, int k, unsigned vo,
                          unsigned vo0) const {
        if (i == kRest)  // the rest population never changes slot
            bst<kPopStore>(r0[k], L.r0, vo0, 0);
        else
            bst<kPopStore>(v[i][k], L.r, vo, (unsigned)C::slot(slot) * L.nxS);
    }
};

__device__ inline int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

struct Acc {  // partial moments of one destination plane
    double r, jx, jy, lp;
};

template <int TX, int TY, int NT> struct Geo {
    static constexpr int WX = TX + 2, WY = TY + 2, NR = WX * WY;
    static_assert(NR <= NT, "one lane per ring-inclusive node");
    static_assert(TX * TY % 64 == 0, "owned columns fill whole waves");
};

template <int P, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_fused(KP kp, const void *fin_q, void *fout_q, const double *__restrict__ mu,
                                              const void *Fq, const void *Qq, double *__restrict__ rho, void *jq,
                                              double *__restrict__ mu0, int *flag, int cz) {
    using G = Geo<TX, TY, NT>;
    using C = Code<P>;
    using real = typename Pol<P>::real;
    __shared__ Plane<P, G::NR> pl;

    // tiles dealt to the XCDs in contiguous ranges (consecutive tiles, which
    // share ring columns, on one XCD), all tiles of a chunk together
    const int ntx = (kp.nx + TX - 1) / TX;
    const unsigned ntiles = gridDim.x, nb = gridDim.x * gridDim.y;
    const unsigned hw = blockIdx.y * gridDim.x + blockIdx.x;
    const unsigned qq = nb >> 3, rem = nb & 7u, xcd = hw & 7u;
    const unsigned lid = xcd * qq + (xcd < rem ? xcd : rem) + (hw >> 3);
    const int tile = (int)(lid % ntiles), chunk = (int)(lid / ntiles);
    const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY;
    const int zs = kp.z0 + chunk * cz;
    const int ze = min(zs + cz, kp.z1);

    const int k = threadIdx.x;
    const unsigned nx = (unsigned)kp.nx;
    // collision role: ring-inclusive node (a, b), a in [-1, TX], b in [-1, TY],
    // at LDS index k; byte offsets of the node in a lattice plane (vi, vi0)
    // and in a field plane (vf8, vfr); lanes past the ring read nothing
    const bool coll = k < G::NR;
    const unsigned cxg = (unsigned)wrapi(x0 + k % G::WX - 1, kp.nx), cyg = (unsigned)wrapi(y0 + k / G::WX - 1, kp.ny);
    const unsigned vi = coll ? (cyg * C::NS * nx + cxg) * C::S : kOOB;
    const unsigned vi0 = coll ? (cyg * nx + cxg) * 4u : kOOB;
    const unsigned vf8 = coll ? (cyg * nx + cxg) * 8u : kOOB;
    const unsigned vfr = coll ? (cyg * nx + cxg) * (unsigned)sizeof(real) : kOOB;
    // streaming role: owned column (oa, ob) at LDS index (ob + 1) WX + oa + 1
    const int oa = k % TX, ob = k / TX;
    const bool owner = k < TX * TY && x0 + oa < kp.nx && y0 + ob < kp.ny;
    const unsigned ox = (unsigned)(x0 + oa), oy = (unsigned)(y0 + ob);
    const int oc = owner ? (ob + 1) * G::WX + oa + 1 : G::WX + 1;
    const unsigned vo = owner ? (oy * C::NS * nx + ox) * C::S : kOOB;
    const unsigned vo0 = owner ? (oy * nx + ox) * 4u : kOOB;

    const size_t N = kp.N, plane = kp.plane;
    const real *F = (const real *)Fq, *Qa = (const real *)Qq;
    real *J = (real *)jq;

    auto fluid = [&](int s) { return kp.walls ? (s >= 1 && s <= kp.nz - 2) : true; };
    auto zw = [&](int s) { return s < 0 ? s + kp.nz : (s >= kp.nz ? s - kp.nz : s); };  // |s| within one period

    // prefetched inputs of the next source plane
    real fn[27];
    double mn = 0.0;
    real an[6];
#pragma unroll
    for (int i = 0; i < 27; ++i) fn[i] = 0;
#pragma unroll
    for (int i = 0; i < 6; ++i) an[i] = 0;
    // inputs of source plane s; with ok false (no such plane) and on lanes
    // past the ring the offsets are kOOB and the loads return zeros
    auto load = [&](int s, bool ok) {
        const int z = ok ? zw(s) : zs;
        const LatPlane<P> L(fin_q, kp, z);
        const unsigned a = ok ? vi : kOOB, a0 = ok ? vi0 : kOOB;
#pragma unroll
        for (int i = 0; i < 27; ++i) fn[i] = L.ld(i, a, a0);
        const unsigned a8 = ok ? vf8 : kOOB, ar = ok ? vfr : kOOB;
        const size_t pb = (size_t)z * plane;
        const unsigned b8 = 8u * kp.plane, br = (unsigned)sizeof(real) * kp.plane;
        mn = bld((double *)nullptr, rsrc(mu + pb, b8), a8, 0);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            an[c] = bld((real *)nullptr, rsrc(F + c * N + pb, br), ar, 0);
            an[3 + c] = bld((real *)nullptr, rsrc(Qa + c * N + pb, br), ar, 0);
        }
    };
    // moments of a completed destination plane z of the owned column; `ok`
    // false (not this chunk's plane, or no owned column) stores nothing
    const unsigned vn8 = (oy * nx + ox) * 8u, vnr = (oy * nx + ox) * (unsigned)sizeof(real);
    bool bad = false;  // some owned density left the EOS domain (flag set at the end)
    auto output = [&](bool ok, int z, const Acc &A, double Lm) {
        ok = ok && owner;
        const size_t pb = (size_t)z * plane;
        const unsigned b8 = 8u * kp.plane, br = (unsigned)sizeof(real) * kp.plane;
        const unsigned o8 = ok ? vn8 : kOOB, orr = ok ? vnr : kOOB;
        const double r = A.r + Lm;
        bst(r, rsrc(rho + pb, b8), o8, 0);
        bst(mu_bulk(kp, r), rsrc(mu0 + pb, b8), o8, 0);
        bst((real)A.jx, rsrc(J + pb, br), orr, 0);
        bst((real)A.jy, rsrc(J + N + pb, br), orr, 0);
        bst((real)(A.lp - Lm), rsrc(J + 2 * N + pb, br), orr, 0);
        bad = bad || (ok && !(r > 0.0 && kp.b * r < 1.0));
    };
    // One layer (cz = c) of the populations that arrive at the owned column
    // from the LDS plane, stored to plane L at lattice offsets (v, v0) (kOOB:
    // not stored), with its x- and y-partial sums in the order of moments().
    // refl (c = -1 at the bottom wall, c = +1 at the top wall): instead, the
    // node's own values of direction (-cx, -cy, c), which the wall reflects
    // into slots (cx, cy, -c) of the same node (halfway bounce-back); the
    // normal layer would enter the solid plane.  The choice is uniform, so
    // every plane issues the same stores.
    auto group = [&](auto cc, bool refl, unsigned v, unsigned v0, const LatPlane<P> &L) {
        constexpr int c = decltype(cc)::value;
        double R[3], X[3];
#pragma unroll
        for (int cy = -1; cy <= 1; ++cy) {
            real val[3];  // cx = 0, +1, -1
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const int cx = t == 0 ? 0 : (t == 1 ? 1 : -1);
                if constexpr (c == 0) {
                    const int i = dir(cx, cy, 0), kk = oc - cy * G::WX - cx;
                    val[t] = pl.get(i, kk);
                    pl.store(L, i, i, kk, v, v0);
                } else {
                    const int in = dir(cx, cy, c), ir = dir(-cx, -cy, c);
                    const int kk = refl ? oc : oc - cy * G::WX - cx;
                    val[t] = refl ? pl.get(ir, kk) : pl.get(in, kk);
                    pl.store(L, refl ? 26 - ir : in, refl ? ir : in, kk, v, v0);
                }
            }
            xpartial((double)val[0], (double)val[1], (double)val[2], R[cy + 1], X[cy + 1]);
        }
        return layer_of(R, X);
    };

    // Every global load and store below sits outside lane-divergent branches
    // (masked lanes carry kOOB offsets) and every plane issues the same
    // number of them, so the compiler can count the outstanding memory
    // operations: the next plane's loads stay in flight through the
    // collision, and the stores of one plane through the next collision.
    Acc prev{0, 0, 0, 0}, cur{0, 0, 0, 0};
    load(zs - 1, fluid(zs - 1));
    for (int s = zs - 1; s <= ze; ++s) {
        const bool sf = fluid(s);
        real f[27];
#pragma unroll
        for (int i = 0; i < 27; ++i) f[i] = fn[i];
        const double m = mn;
        const real Fx = an[0], Fy = an[1], Fz = an[2], q200 = an[3], q020 = an[4], q002 = an[5];
        load(s + 1, s + 1 <= ze && fluid(s + 1));
        if (sf && coll) {
            collide_node(kp, f, m, Fx, Fy, Fz, q200, q020, q002);
#pragma unroll
            for (int i = 0; i < 27; ++i) pl.put(i, k, f[i]);
        }
        __syncthreads();
        if (k < TX * TY) {  // the waves that hold owned columns (wave-uniform)
            const int zm = s - 1, zp = s + 1;
            const bool wall_lo = kp.walls && s == 1, wall_hi = kp.walls && s == kp.nz - 2;
            const bool own_m = sf && zm >= zs && zm < ze && fluid(zm);
            const bool own_0 = sf && s >= zs && s < ze;
            const bool own_p = sf && zp >= zs && zp < ze && fluid(zp);
            const LatPlane<P> D0(fout_q, kp, zw(s));
            const bool st_m = wall_lo ? own_0 : own_m, st_p = wall_hi ? own_0 : own_p;
            const Layer Lm = group(std::integral_constant<int, -1>{}, wall_lo, st_m ? vo : kOOB, kOOB,
                                   wall_lo ? D0 : LatPlane<P>(fout_q, kp, zw(zm)));
            const Layer L0 = group(std::integral_constant<int, 0>{}, false, own_0 ? vo : kOOB, own_0 ? vo0 : kOOB, D0);
            const Layer Lp = group(std::integral_constant<int, 1>{}, wall_hi, st_p ? vo : kOOB, kOOB,
                                   wall_hi ? D0 : LatPlane<P>(fout_q, kp, zw(zp)));
            // plane s-1 is complete with the layer cz = -1 of this plane; next
            // to the top wall (s = nz-1, solid) with the reflection that the
            // previous plane left in cur
            {
                const bool top = kp.walls && s == kp.nz - 1;
                const Layer Lc = top ? Layer{cur.r, cur.jx, cur.jy} : Lm;
                Acc A = prev;
                A.jx += Lc.JX;
                A.jy += Lc.JY;
                output(top ? zm >= zs && zm < ze : own_m, zw(zm), A, Lc.L);
            }
            // plane s: its cz = +1 layer came from plane s-1, or from the
            // reflection at the bottom wall
            if (wall_lo) cur = Acc{Lm.L, Lm.JX, Lm.JY, Lm.L};
            cur.r += L0.L;
            cur.jx += L0.JX;
            cur.jy += L0.JY;
            prev = cur;
            cur = Acc{Lp.L, Lp.JX, Lp.JY, Lp.L};
        }
        __syncthreads();
    }
    if (bad) *flag = 1;
}

// Planes per workgroup: long chunks amortise the two ring planes; enough
// workgroups to give every CU one.
int fused_chunk(const KP &kp, unsigned tiles) {
    const int nzf = kp.z1 - kp.z0;
    int cz = 64;
    while (cz > 8 && (size_t)tiles * ((nzf + cz - 1) / cz) < 256) cz /= 2;
    return cz;
}

template <int P, int TX, int TY, int NT> hipError_t launch(hipStream_t s, const KP &kp, const Bufs &b, int cur) {
    const unsigned ntx = (kp.nx + TX - 1) / TX, nty = (kp.ny + TY - 1) / TY;
    const int cz = fused_chunk(kp, ntx * nty);
    const int nzf = kp.z1 - kp.z0;
    const dim3 grid(ntx * nty, (nzf + cz - 1) / cz);
    k_fused<P, TX, TY, NT><<<grid, NT, 0, s>>>(kp, b.f[cur], b.f[1 - cur], b.mu, b.F, b.Q, b.rho, b.j, b.mu0,
                                                b.flag, cz);
    return hipGetLastError();
}

}  // namespace

bool fused_plane_ok(int prec, size_t plane) {
    // the rows of one plane and the kOOB offset of masked lanes below 2^31
    const size_t bytes = plane * 27 * real_bytes(prec == LBFE_FP64 ? LBFE_FP64 : LBFE_FP32);
    return bytes < kOOB;
}

hipError_t launch_fused(hipStream_t s, int prec, const KP &kp, const Bufs &b, int cur) {
    switch (prec) {
        case LBFE_FP64: return launch<LBFE_FP64, 32, 12, 512>(s, kp, b, cur);
        case LBFE_FP32: return launch<LBFE_FP32, 32, 12, 512>(s, kp, b, cur);
        case LBFE_FP16_DEV: return launch<LBFE_FP16_DEV, 32, 12, 512>(s, kp, b, cur);
        default: return launch<LBFE_FP16_DEV_F0FP32, 32, 12, 512>(s, kp, b, cur);
    }
}

}  // namespace lbfe
