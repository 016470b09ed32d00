// Moment-representation state of the D3Q27 free-energy LB step for the
// paper's rate setting, every relaxation rate but omega_1 at 1 (Sec. II B,
// stated after Eq. (26)).  Between steps the lattice holds, per node, the 16
// numbers of the post-collision state (collide_to_state, lbfe_device.h)
// instead of 27 populations: 16 S bytes per node and pass instead of 27 S.
//
// With the state m*(t-1) of every node and rho, j, mu0 of f(t) at hand, one
// step is
//   stencil chain   mu, F, Q of f(t)                     (lbfe_chain.hip)
//   k_mstate<kCollide>  every node of a tile and its one-node ring rebuilds
//       its 27 post-collision populations f*(t-1) from its state, once, into
//       an LDS plane; every owned column gathers the values that arrive at it,
//       f_i(x, t) = f*_i(x - c_i, t-1), across three source planes in
//       registers, collides them and writes its state m*(t)
//   k_mstate<kMoments>  the same rebuild and gather for m*(t); the owned
//       columns sum rho, j and mu0 of f(t+1) in the order of moments()
//       (lbfe_device.h) and store no populations.
// k_mstate_first enters the state form from stored populations (the
// collision alone), and k_mstate<kPops> leaves it: it writes f(t+1) to a
// population lattice as well as its moments.  The rebuilt populations equal
// those the collision of the population path produces (zero signs aside), so
// a run through the state form gives the populations of the two-pass path.
#include <type_traits>

#include "lbfe_plane.h"

namespace lbfe {
namespace {

using namespace plane;

constexpr int kMoments = kStateMoments, kPops = kStatePops, kCollide = kStateCollide;

// One z-plane of the state lattice: row-blocked like the populations, the
// kMState values of an x-row as kMState contiguous runs of nx.  Plane z
// starts where plane z of the population lattice starts (stride 27 S nx ny
// bytes), so a state in a population buffer never touches the bytes of the
// solid planes, which stay zero as on the population paths.
template <int P> struct StatePlane {
    using real = typename Pol<P>::real;
    __amdgpu_buffer_rsrc_t r;
    unsigned nxS;  // bytes per slot run
    __device__ StatePlane(const void *base, const KP &kp, int z) {
        const size_t rows = (size_t)kMState * sizeof(real) * kp.plane;
        nxS = (unsigned)kp.nx * (unsigned)sizeof(real);
        r = rsrc((const char *)base + (size_t)z * 27 * sizeof(real) * kp.plane, (unsigned)rows);
    }
    // vo: byte offset of the node's row position, (y kMState nx + x) S
    __device__ real ld(int m, unsigned vo) const { return bld((real *)nullptr, r, vo, (unsigned)m * nxS); }
    __device__ void st(int m, unsigned vo, real x) const { bst<kPopStore>(x, r, vo, (unsigned)m * nxS); }
};

template <int P, int MODE, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_mstate(KP kp, const void *sin_q, void *out_q, const double *__restrict__ mu,
                                               const void *Fq, const void *Qq, double *__restrict__ rho, void *jq,
                                               double *__restrict__ mu0, int *flag, int cz) {
    using G = Geo<TX, TY, NT>;
    using real = typename Pol<P>::real;
    constexpr unsigned S = sizeof(real);
    __shared__ Plane<P, G::NR> pl;

    const Chunk ch = chunk_of<TX, TY>(kp, cz);
    const int x0 = ch.x0, y0 = ch.y0, zs = ch.zs, ze = ch.ze;
    const int k = threadIdx.x;
    const unsigned nx = (unsigned)kp.nx;
    // source role: ring-inclusive node (a, b), a in [-1, TX], b in [-1, TY],
    // at LDS index k; lanes past the ring read nothing
    const bool src = k < G::NR;
    const unsigned cxg = (unsigned)wrapi(x0 + k % G::WX - 1, kp.nx), cyg = (unsigned)wrapi(y0 + k / G::WX - 1, kp.ny);
    const unsigned vs = src ? (cyg * kMState * nx + cxg) * S : kOOB;
    // owned column (oa, ob) at LDS index (ob + 1) WX + oa + 1
    const int oa = k % TX, ob = k / TX;
    const bool owner = k < TX * TY && x0 + oa < kp.nx && y0 + ob < kp.ny;
    const unsigned ox = (unsigned)(x0 + oa), oy = (unsigned)(y0 + ob);
    const int oc = owner ? (ob + 1) * G::WX + oa + 1 : G::WX + 1;
    const unsigned vso = owner ? (oy * kMState * nx + ox) * S : kOOB;                   // state lattice
    const unsigned vo = owner ? (oy * Code<P>::NS * nx + ox) * Code<P>::S : kOOB;      // population lattice
    const unsigned vn8 = owner ? (oy * nx + ox) * 8u : kOOB, vnr = owner ? (oy * nx + ox) * S : kOOB;  // fields

    const size_t N = kp.N, plane = kp.plane;
    const unsigned b8 = 8u * kp.plane, br = S * kp.plane;
    const real *F = (const real *)Fq, *Qa = (const real *)Qq;
    real *J = (real *)jq;

    auto fluid = [&](int s) { return kp.walls ? (s >= 1 && s <= kp.nz - 2) : true; };
    auto zw = [&](int s) { return s < 0 ? s + kp.nz : (s >= kp.nz ? s - kp.nz : s); };

    // prefetched state of the next source plane (zeros where ok is false)
    real mn[kMState];
    auto load = [&](int s, bool ok) {
        const StatePlane<P> L(sin_q, kp, ok ? zw(s) : zs);
        const unsigned a = ok ? vs : kOOB;
#pragma unroll
        for (int m = 0; m < kMState; ++m) mn[m] = L.ld(m, a);
    };
    // collide mode: prefetched mu, F, Q of the owned node in plane s
    double fmu = 0;
    real ff[6] = {0, 0, 0, 0, 0, 0};
    auto load_fields = [&](int s, bool ok) {
        const size_t pb = (size_t)(ok ? s : zs) * plane;
        const unsigned a8 = ok ? vn8 : kOOB, ar = ok ? vnr : kOOB;
        fmu = bld((double *)nullptr, rsrc(mu + pb, b8), a8, 0);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            ff[c] = bld((real *)nullptr, rsrc(F + c * N + pb, br), ar, 0);
            ff[3 + c] = bld((real *)nullptr, rsrc(Qa + c * N + pb, br), ar, 0);
        }
    };

    // One layer (cz = c) of the values that arrive at the owned column from
    // the LDS plane, val[3 (cx + 1) + (cy + 1)] for direction (cx, cy, c);
    // with refl (c = -1 at the bottom wall, c = +1 at the top wall) instead
    // the node's own values of direction (-cx, -cy, c), which the wall
    // reflects into slot (cx, cy, -c) of the same node (halfway bounce-back):
    // then val[..] is for direction (cx, cy, -c).  In kPops mode the values
    // are also stored to plane L at offset v (kOOB: not stored).
    auto gather = [&](auto cc, bool refl, real(&val)[9], unsigned v, unsigned v0, const void *Lp, int z) {
        constexpr int c = decltype(cc)::value;
#pragma unroll
        for (int cx = -1; cx <= 1; ++cx)
#pragma unroll
            for (int cy = -1; cy <= 1; ++cy) {
                const int jj = 3 * (cx + 1) + (cy + 1);
                const int in = dir(cx, cy, c), ir = dir(-cx, -cy, c);
                const bool rf = c != 0 && refl;
                const int kk = rf ? oc : oc - cy * G::WX - cx;
                val[jj] = rf ? pl.get(ir, kk) : pl.get(in, kk);
                if constexpr (MODE == kPops) {
                    const LatPlane<P> L(Lp, kp, z);
                    pl.store(L, rf ? 26 - ir : in, rf ? ir : in, kk, v, v0);
                }
            }
    };
    // moment partials of one layer in the order of moments()
    auto layer = [&](const real(&val)[9]) {
        double R[3], X[3];
#pragma unroll
        for (int cy = -1; cy <= 1; ++cy)
            xpartial((double)val[3 + cy + 1], (double)val[6 + cy + 1], (double)val[cy + 1], R[cy + 1], X[cy + 1]);
        return layer_of(R, X);
    };
    bool bad = false;  // some owned density left the EOS domain (flag set at the end)
    auto output = [&](bool ok, int z, const Acc &A, double Lm) {
        ok = ok && owner;
        const size_t pb = (size_t)z * plane;
        const unsigned o8 = ok ? vn8 : kOOB, orr = ok ? vnr : kOOB;
        const double r = A.r + Lm;
        bst(r, rsrc(rho + pb, b8), o8, 0);
        bst(mu_bulk(kp, r), rsrc(mu0 + pb, b8), o8, 0);
        bst((real)A.jx, rsrc(J + pb, br), orr, 0);
        bst((real)A.jy, rsrc(J + N + pb, br), orr, 0);
        bst((real)(A.lp - Lm), rsrc(J + 2 * N + pb, br), orr, 0);
        bad = bad || (ok && !(r > 0.0 && kp.b * r < 1.0));
    };

    // moments modes: partial sums of destination planes s (cur) and s-1 (prev)
    Acc prev{0, 0, 0, 0}, cur{0, 0, 0, 0};
    // collide mode: arrived layers of destination s-1 (cz = +1: up, cz = 0:
    // mid) and of destination s (cz = +1: nxt, or the bottom-wall reflection)
    real up[9], mid[9], nxt[9];
#pragma unroll
    for (int j = 0; j < 9; ++j) up[j] = mid[j] = nxt[j] = 0;

    // As in the fused kernel, every global access sits outside lane-divergent
    // branches (masked lanes carry kOOB) and every plane issues the same
    // number of them, so the next plane's loads stay in flight through the
    // rebuild and the gathers.
    load(zs - 1, fluid(zs - 1));
    for (int s = zs - 1; s <= ze; ++s) {
        const bool sf = fluid(s);
        real m[kMState];
#pragma unroll
        for (int q = 0; q < kMState; ++q) m[q] = mn[q];
        load(s + 1, s + 1 <= ze && fluid(s + 1));
        double cmu = 0;
        real cf[6];
        if constexpr (MODE == kCollide) {
            cmu = fmu;
#pragma unroll
            for (int q = 0; q < 6; ++q) cf[q] = ff[q];
            load_fields(s, s >= zs && s < ze && sf);
        }
        if (sf && src) {
            real f[27];
            state_populations(kp, m, f);
#pragma unroll
            for (int i = 0; i < 27; ++i) pl.put(i, k, f[i]);
        }
        __syncthreads();
        if (k < TX * TY) {  // the waves that hold owned columns (wave-uniform)
            const int zm = s - 1, zp = s + 1;
            const bool wall_lo = kp.walls && s == 1, wall_hi = kp.walls && s == kp.nz - 2;
            const bool top = kp.walls && s == kp.nz - 1;
            const bool own_m = sf && zm >= zs && zm < ze && fluid(zm);
            const bool own_0 = sf && s >= zs && s < ze;
            const bool own_p = sf && zp >= zs && zp < ze && fluid(zp);
            const bool st_m = wall_lo ? own_0 : own_m, st_p = wall_hi ? own_0 : own_p;
            real vm[9], v0[9], vp[9];
            gather(std::integral_constant<int, -1>{}, wall_lo, vm, st_m ? vo : kOOB, kOOB, out_q,
                   zw(wall_lo ? s : zm));
            gather(std::integral_constant<int, 0>{}, false, v0, own_0 ? vo : kOOB, kOOB, out_q, zw(s));
            gather(std::integral_constant<int, 1>{}, wall_hi, vp, st_p ? vo : kOOB, kOOB, out_q,
                   zw(wall_hi ? s : zp));
            if constexpr (MODE == kCollide) {
                // destination s-1 is complete with its cz = -1 layer (from this
                // plane, or next to the top wall the reflection held in nxt)
                const bool ok = top ? zm >= zs && zm < ze : own_m;
                real f[27];
#pragma unroll
                for (int j = 0; j < 9; ++j) {
                    f[3 * j + 2] = up[j];
                    f[3 * j + 1] = mid[j];
                    f[3 * j] = top ? nxt[j] : vm[j];
                }
                real st[kMState];
                collide_to_state(kp, f, cmu, cf[0], cf[1], cf[2], cf[3], cf[4], cf[5], st);
                const StatePlane<P> O(out_q, kp, zw(zm));
                const unsigned a = ok && owner ? vso : kOOB;
#pragma unroll
                for (int q = 0; q < kMState; ++q) O.st(q, a, st[q]);
#pragma unroll
                for (int j = 0; j < 9; ++j) {
                    up[j] = wall_lo ? vm[j] : nxt[j];
                    mid[j] = v0[j];
                    nxt[j] = vp[j];
                }
            } else {
                const Layer Lm = layer(vm), L0 = layer(v0), Lp = layer(vp);
                // plane s-1 is complete with the layer cz = -1 of this plane;
                // next to the top wall with the reflection left in cur
                {
                    const Layer Lc = top ? Layer{cur.r, cur.jx, cur.jy} : Lm;
                    Acc A = prev;
                    A.jx += Lc.JX;
                    A.jy += Lc.JY;
                    output(top ? zm >= zs && zm < ze : own_m, zw(zm), A, Lc.L);
                }
                if (wall_lo) cur = Acc{Lm.L, Lm.JX, Lm.JY, Lm.L};
                cur.r += L0.L;
                cur.jx += L0.JX;
                cur.jy += L0.JY;
                prev = cur;
                cur = Acc{Lp.L, Lp.JX, Lp.JY, Lp.L};
            }
        }
        __syncthreads();
    }
    if constexpr (MODE != kCollide) {
        if (bad) *flag = 1;
    }
}

// Entry into the state form: the collision of the populations f[cur] with
// the current mu, F, Q, ending at the state (no streaming).  One thread per
// fluid node; the state is written in the layout of StatePlane.
template <int P>
__global__ __launch_bounds__(kBlock) void k_mstate_first(KP kp, const void *fin_q, void *sout_q,
                                                         const double *__restrict__ mu, const void *Fq,
                                                         const void *Qq) {
    using real = typename Pol<P>::real;
    const unsigned idx = tile_id(kp) * kBlock + threadIdx.x;
    if (idx >= kp.nfluid) return;
    const unsigned n = (unsigned)kp.z0 * kp.plane + idx;
    const unsigned row = n / (unsigned)kp.nx, x = n - row * (unsigned)kp.nx;
    const unsigned z = n / kp.plane, y = row - z * (unsigned)kp.ny;
    const Pops<P> fin(fin_q, kp);
    real f[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) f[i] = fin.ld(i, row, x);
    const real *F = (const real *)Fq, *Qa = (const real *)Qq;
    const size_t N = kp.N;
    real st[kMState];
    collide_to_state(kp, f, mu[n], F[n], F[N + n], F[2 * N + n], Qa[n], Qa[N + n], Qa[2 * N + n], st);
    real *out = (real *)sout_q + (size_t)z * 27 * kp.plane + (size_t)y * kMState * kp.nx + x;
#pragma unroll
    for (int q = 0; q < kMState; ++q) __builtin_nontemporal_store(st[q], out + (size_t)q * kp.nx);
}

constexpr int kTX = 32, kTY = 12, kNT = 512;

template <int P, int MODE> hipError_t launch(hipStream_t s, const KP &kp, const Bufs &b, const void *sin, void *out) {
    const unsigned ntx = (kp.nx + kTX - 1) / kTX, nty = (kp.ny + kTY - 1) / kTY;
    const int cz = chunk_planes(kp, ntx * nty);
    const int nzf = kp.z1 - kp.z0;
    const dim3 grid(ntx * nty, (nzf + cz - 1) / cz);
    k_mstate<P, MODE, kTX, kTY, kNT><<<grid, kNT, 0, s>>>(kp, sin, out, b.mu, b.F, b.Q, b.rho, b.j, b.mu0, b.flag, cz);
    return hipGetLastError();
}

template <int P> hipError_t launch_mode(hipStream_t s, int mode, const KP &kp, const Bufs &b, const void *sin,
                                        void *out) {
    switch (mode) {
        case kMoments: return launch<P, kMoments>(s, kp, b, sin, out);
        case kPops: return launch<P, kPops>(s, kp, b, sin, out);
        default: return launch<P, kCollide>(s, kp, b, sin, out);
    }
}

}  // namespace

bool state_plane_ok(int prec, size_t plane) {
    // one z-plane of the population rows (kPops) and of the state below the
    // 32-bit offsets of the buffer descriptors
    return plane * 27 * real_bytes(prec) < kOOB;
}

hipError_t launch_state_pass(hipStream_t s, int prec, int mode, const KP &kp, const Bufs &b, const void *sin,
                             void *out) {
    if (prec == LBFE_FP64) return launch_mode<LBFE_FP64>(s, mode, kp, b, sin, out);
    if (prec == LBFE_FP32) return launch_mode<LBFE_FP32>(s, mode, kp, b, sin, out);
    return hipErrorInvalidValue;
}

hipError_t launch_state_first(hipStream_t s, int prec, const KP &kp, const Bufs &b, const void *fin, void *sout) {
    const unsigned g = nblocks(kp.nfluid);
    if (prec == LBFE_FP64)
        k_mstate_first<LBFE_FP64><<<g, kBlock, 0, s>>>(kp, fin, sout, b.mu, b.F, b.Q);
    else if (prec == LBFE_FP32)
        k_mstate_first<LBFE_FP32><<<g, kBlock, 0, s>>>(kp, fin, sout, b.mu, b.F, b.Q);
    else
        return hipErrorInvalidValue;
    return hipGetLastError();
}

}  // namespace lbfe
