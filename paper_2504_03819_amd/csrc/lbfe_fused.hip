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

#include "lbfe_plane.h"

namespace lbfe {
namespace {

using namespace plane;

template <int P, int TX, int TY, int NT>
__global__ __launch_bounds__(NT) void k_fused(KP kp, const void *fin_q, void *fout_q, const double *__restrict__ mu,
                                              const void *Fq, const void *Qq, double *__restrict__ rho, void *jq,
                                              double *__restrict__ mu0, int *flag, int cz) {
    using G = Geo<TX, TY, NT>;
    using C = Code<P>;
    using real = typename Pol<P>::real;
    __shared__ Plane<P, G::NR> pl;

    const Chunk ch = chunk_of<TX, TY>(kp, cz);
    const int x0 = ch.x0, y0 = ch.y0, zs = ch.zs, ze = ch.ze;

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

template <int P, int TX, int TY, int NT> hipError_t launch(hipStream_t s, const KP &kp, const Bufs &b, int cur) {
    const unsigned ntx = (kp.nx + TX - 1) / TX, nty = (kp.ny + TY - 1) / TY;
    const int cz = chunk_planes(kp, ntx * nty);
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
