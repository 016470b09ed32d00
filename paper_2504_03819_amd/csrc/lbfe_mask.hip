// Arbitrary solid voxel masks (curved or patterned substrates) on gfx950:
// the halfway bounce-back of Eq. (10) and the wetting boundary of
// Eqs. (36)-(38) at every solid node x_s of a mask, which the paper writes
// for a general x_s (Sec. III C).  The flat walls of the z-plane path are the
// special case of a mask holding the two planes.
//
// Every node carries one 32-bit neighbour word: bit i (i = 0..26) is set
// when x + c_i is solid, so bit 13 tells whether the node itself is solid.
// It is built once per mask; all kernels below work per node over the whole
// grid and read it (the _m kernels gather their neighbours through L1/L2,
// the _z stencils stage their input field in the z-marching LDS ring of
// lbfe_zring.h):
//   k_moments_m     rho, j of the fluid nodes (order of moments())
//   k_wall_rho_m    rho at solid nodes with a fluid neighbour, Eqs. (37)-(38)
//   k_mu_z          mu = mu0(rho) - kappa lap_h rho at fluid nodes, Eq. (32)
//                   (k_mu_m for the initialiser)
//   k_wall_mu_m     mu at solid nodes, Eq. (36)
//   k_fphi_z        G = grad_h mu, F = (1/3 - rho) G, u = (j + F/2)/rho,
//                   phi = (p_m - rho/3) u at fluid nodes, Eqs. (11)-(12), (27)
//   k_q_z / k_q_m   Q_aa = -3 d_a phi_a at fluid nodes, Eq. (27) (FP64 /
//                   FP32 phi)
//   k_collide_m     collision and push-streaming; a link that ends on a
//                   solid node returns into slot opp(i) of its own node
// Solid nodes hold no populations (their slots stay zero) and zero j, F,
// phi, Q; a solid node with no fluid neighbour gets rho = mu = 0 and is read
// by no fluid stencil.
#include "lbfe_device.h"
#include "lbfe_zring.h"

namespace lbfe {
namespace {

template <int P> using real_t = typename Pol<P>::real;

constexpr unsigned kSelf = 1u << kRest;

__device__ inline bool solid_at(unsigned w) { return (w & kSelf) != 0; }

__global__ __launch_bounds__(kBlock) void k_mask_prep(KP kp, const uint8_t *solid, unsigned *nbr) {
    const unsigned n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    int x, y, z;
    decompose(kp, n, x, y, z);
    const Nb nb(kp, x, y, z);
    unsigned w = 0;
#pragma unroll
    for (int i = 0; i < 27; ++i)
        if (solid[nb.at(cxi(i), cyi(i), czi(i))]) w |= 1u << i;
    nbr[n] = w;
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_moments_m(KP kp, const unsigned *nbr, const void *fq, double *rho,
                                                      void *jq, int *flag) {
    using real = real_t<P>;
    const unsigned n = tile_id(kp) * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    // the population loads do not wait for the neighbour word (a solid
    // node's slots hold zeros); only the stores depend on it
    const unsigned w = nbr[n];
    const unsigned row = n / (unsigned)kp.nx, x = n - row * (unsigned)kp.nx;
    const Pops<P> f(fq, kp);
    real v[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) v[i] = f.ld(i, row, x);
    double r;
    real jx, jy, jz;
    moments(v, r, jx, jy, jz);
    if (solid_at(w)) return;
    rho[n] = r;
    real *j = (real *)jq;
    j[n] = jx;
    j[kp.N + n] = jy;
    j[2 * (size_t)kp.N + n] = jz;
    if (!(r > 0.0 && kp.b * r < 1.0)) *flag = 1;
}

// Weighted average over the fluid neighbours of a solid node (Eqs. (36),
// (37)), in direction order; 0 when there is none.
__device__ inline double fluid_average(const KP &kp, unsigned w, const double *g, unsigned n) {
    int x, y, z;
    decompose(kp, n, x, y, z);
    const Nb nb(kp, x, y, z);
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        if (w & (1u << i)) continue;
        const double wt = wi(i);
        num += wt * g[nb.at(cxi(i), cyi(i), czi(i))];
        den += wt;
    }
    return den > 0.0 ? num / den : 0.0;
}

__global__ __launch_bounds__(kBlock) void k_wall_rho_m(KP kp, const unsigned *nbr, double *rho) {
    const unsigned n = tile_id(kp) * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    const unsigned w = nbr[n];
    if (!solid_at(w)) return;
    const double rave = fluid_average(kp, w, rho, n);
    double out = rave;
    if (rave >= kp.lo && rave <= kp.hi) {  // contact-line window
        if (kp.wet_mode == LBFE_WET_PHI)
            out = fmin(fmax(kp.wet_value * rave, kp.lo), kp.hi);
        else if (kp.wet_mode == LBFE_WET_DELTA)
            out = fmin(fmax(rave - kp.wet_value, kp.lo), kp.hi);
    }
    rho[n] = out;
}

// mu = mu0(rho) - kappa lap_h rho, lap_h g = 6 sum_i w_i (g(x+c_i) - g(x))
__global__ __launch_bounds__(kBlock) void k_mu_m(KP kp, const unsigned *nbr, const double *rho, double *mu) {
    const unsigned n = tile_id(kp) * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    const bool solid = solid_at(nbr[n]);
    int x, y, z;
    decompose(kp, n, x, y, z);
    const Nb nb(kp, x, y, z);
    const double r0 = rho[n];
    double s = 0.0;
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        if (i == kRest) continue;
        s += wi(i) * (rho[nb.at(cxi(i), cyi(i), czi(i))] - r0);
    }
    if (solid) return;
    mu[n] = mu_bulk(kp, r0) - kp.kappa * 6.0 * s;
}

__global__ __launch_bounds__(kBlock) void k_wall_mu_m(KP kp, const unsigned *nbr, double *mu) {
    const unsigned n = tile_id(kp) * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    const unsigned w = nbr[n];
    if (!solid_at(w)) return;
    mu[n] = fluid_average(kp, w, mu, n);
}

// Q_aa = -3 d_a,h phi_a = -9 sum_i w_i c_ia phi_a(x + c_i)
template <int P>
__global__ __launch_bounds__(kBlock) void k_q_m(KP kp, const unsigned *nbr, const void *phiq, void *Qq) {
    using real = real_t<P>;
    const unsigned n = tile_id(kp) * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    const size_t N = kp.N;
    real *Q = (real *)Qq;
    const bool solid = solid_at(nbr[n]);
    int x, y, z;
    decompose(kp, n, x, y, z);
    const Nb nb(kp, x, y, z);
    const real *phi = (const real *)phiq;
    real sx = 0, sy = 0, sz = 0;
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        if (i == kRest) continue;
        const unsigned m = nb.at(cxi(i), cyi(i), czi(i));
        const real wt = (real)wi(i);
        if (cxi(i)) sx += (real)cxi(i) * wt * phi[m];
        if (cyi(i)) sy += (real)cyi(i) * wt * phi[N + m];
        if (czi(i)) sz += (real)czi(i) * wt * phi[2 * N + m];
    }
    const real h = (real)(-9.0);
    Q[n] = solid ? (real)0 : h * sx;
    Q[N + n] = solid ? (real)0 : h * sy;
    Q[2 * N + n] = solid ? (real)0 : h * sz;
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_collide_m(KP kp, const unsigned *nbr, const void *fin_q, void *fout_q,
                                                      const double *mu, const void *Fq, const void *Qq) {
    using real = real_t<P>;
    const unsigned n = tile_id(kp) * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    const unsigned w = nbr[n];
    int x, y, z;
    decompose(kp, n, x, y, z);
    const Nb nb(kp, x, y, z);
    const Pops<P> fin(fin_q, kp);
    const Pops<P> fout(fout_q, kp);
    const unsigned row = nb.row(0, 0);
    real f[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) f[i] = fin.ld(i, row, (unsigned)x);
    if (solid_at(w)) return;
    const real *F = (const real *)Fq, *Qa = (const real *)Qq;
    collide_node(kp, f, mu[n], F[n], F[kp.N + n], F[2 * (size_t)kp.N + n], Qa[n], Qa[kp.N + n],
                 Qa[2 * (size_t)kp.N + n]);
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        if (w & (1u << i))
            fout.st(26 - i, row, (unsigned)x, f[i]);
        else
            fout.st(i, nb.row(cyi(i), czi(i)), nb.xo(cxi(i)), f[i]);
    }
}

// Initial populations of the fluid nodes (Eq. (20) equilibrium at rho0, u0,
// p_m(mu)); solid nodes get zeros.
template <int P>
__global__ __launch_bounds__(kBlock) void k_init_m(KP kp, const unsigned *nbr, const double *rho0, const double *u0,
                                                   const double *mu, void *fq) {
    using real = real_t<P>;
    const unsigned n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    const Pops<P> f(fq, kp);
    const unsigned row = n / (unsigned)kp.nx, x = n - row * (unsigned)kp.nx;
    real k[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) k[i] = 0;
    if (!solid_at(nbr[n])) {
        const real pm = (real)((1.0 + mu[n]) / 3.0);
        k[K(0, 0, 0)] = (real)rho0[n];
        k[K(2, 0, 0)] = k[K(0, 2, 0)] = k[K(0, 0, 2)] = pm;
        k[K(2, 2, 0)] = k[K(2, 0, 2)] = k[K(0, 2, 2)] = pm * (real)(1.0 / 3.0);
        k[K(2, 2, 2)] = pm * (real)(1.0 / 9.0);
        real ux = 0, uy = 0, uz = 0;
        if (u0) {
            ux = (real)u0[n];
            uy = (real)u0[kp.N + n];
            uz = (real)u0[2 * (size_t)kp.N + n];
        }
        cm_inverse(k, ux, uy, uz);
#pragma unroll
        for (int i = 0; i < 27; ++i) f.st(i, row, x, k[i]);
    } else {
#pragma unroll
        for (int i = 0; i < 27; ++i) f.st(i, row, x, (real)0);
    }
}

__global__ __launch_bounds__(kBlock) void k_copy_fluid_m(KP kp, const unsigned *nbr, const double *src, double *dst) {
    const unsigned n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    dst[n] = solid_at(nbr[n]) ? 0.0 : src[n];
}

__global__ __launch_bounds__(kBlock) void k_check_rho_m(KP kp, const unsigned *nbr, const double *rho, int *flag) {
    const unsigned n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= kp.N || solid_at(nbr[n])) return;
    const double r = rho[n];
    if (!(r > 0.0 && kp.b * r < 1.0)) *flag = 1;
}

// The same Q for FP64 phi, whose per-node gathers (54 eight-byte loads per
// node) miss L1 more than the FP32 ones: the three components of four
// consecutive planes of a 32 x 16 tile (plus a one-node halo) are staged in
// an LDS ring and each point reads its stencil there.
__global__ __launch_bounds__(ZCB) void k_q_z(KP kp, const unsigned *nbr, const double *phi, double *Q, int cz) {
    __shared__ double lds[4][3][ZNR];
    int x0, y0, zs, ze;
    ztile(kp, cz, 0, kp.nz, x0, y0, zs, ze);
    const size_t N = kp.N;
    ZRing<3> R;
    R.init(kp, lds, x0, y0);
    for (int c = 0; c < 3; ++c) R.src[c] = phi + c * N;
    R.march(zs, ze, [&](int k) {
        if (!R.own) return;
        double sx = 0.0, sy = 0.0, sz = 0.0;
#pragma unroll
        for (int a = -1; a <= 1; ++a)
#pragma unroll
            for (int c = -1; c <= 1; ++c) {
                const double w = w1(a) * w1(c) / 6.0;
                sx += w * (R.at(0, k + c, 1, a) - R.at(0, k + c, -1, a));
                sy += w * (R.at(1, k + c, a, 1) - R.at(1, k + c, a, -1));
                sz += w * (R.at(2, k + 1, a, c) - R.at(2, k - 1, a, c));
            }
        const size_t n = (size_t)k * kp.plane + R.node;
        const bool solid = solid_at(nbr[n]);
        Q[n] = solid ? 0.0 : -9.0 * sx;
        Q[N + n] = solid ? 0.0 : -9.0 * sy;
        Q[2 * N + n] = solid ? 0.0 : -9.0 * sz;
    });
}

// The step's mu (the sums of k_mu_m, in the same order) and its force,
// velocity and phi, with the stencil field (rho, mu) staged in an LDS ring:
// grad_h mu = 3 sum_i w_i c_i mu(x + c_i), F = (1/3 - rho) grad_h mu,
// u = (j + F/2)/rho, phi = (p_m - rho/3) u; F = phi = 0 at solid nodes.
__global__ __launch_bounds__(ZCB) void k_mu_z(KP kp, const unsigned *nbr, const double *rho, double *mu, int cz) {
    __shared__ double lds[4][1][ZNR];
    int x0, y0, zs, ze;
    ztile(kp, cz, 0, kp.nz, x0, y0, zs, ze);
    ZRing<1> R;
    R.init(kp, lds, x0, y0);
    R.src[0] = rho;
    R.march(zs, ze, [&](int k) {
        if (!R.own) return;
        const size_t n = (size_t)k * kp.plane + R.node;
        if (solid_at(nbr[n])) return;
        const double r0 = R.at(0, k, 0, 0);
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            if (i == kRest) continue;
            s += wi(i) * (R.at(0, k + czi(i), cxi(i), cyi(i)) - r0);
        }
        mu[n] = mu_bulk(kp, r0) - kp.kappa * 6.0 * s;
    });
}

template <int P>
__global__ __launch_bounds__(ZCB) void k_fphi_z(KP kp, const unsigned *nbr, const double *rho, const void *jq,
                                                const double *mu, void *Fq, void *phiq, int cz) {
    using real = real_t<P>;
    __shared__ double lds[4][1][ZNR];
    int x0, y0, zs, ze;
    ztile(kp, cz, 0, kp.nz, x0, y0, zs, ze);
    const size_t N = kp.N;
    real *F = (real *)Fq, *phi = (real *)phiq;
    const real *j = (const real *)jq;
    ZRing<1> R;
    R.init(kp, lds, x0, y0);
    R.src[0] = mu;
    R.march(zs, ze, [&](int k) {
        if (!R.own) return;
        const size_t n = (size_t)k * kp.plane + R.node;
        if (solid_at(nbr[n])) {
            for (int a = 0; a < 3; ++a) F[a * N + n] = phi[a * N + n] = (real)0;
            return;
        }
        double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            if (i == kRest) continue;
            const double v = 3.0 * wi(i) * R.at(0, k + czi(i), cxi(i), cyi(i));
            if (cxi(i)) gx += cxi(i) * v;
            if (cyi(i)) gy += cyi(i) * v;
            if (czi(i)) gz += czi(i) * v;
        }
        const double rd = rho[n];
        const double c1 = 1.0 / 3.0 - rd;
        const real Fx = (real)(c1 * gx), Fy = (real)(c1 * gy), Fz = (real)(c1 * gz);
        const real ir = (real)1 / (real)rd;
        const real ux = (j[n] + (real)0.5 * Fx) * ir;
        const real uy = (j[N + n] + (real)0.5 * Fy) * ir;
        const real uz = (j[2 * N + n] + (real)0.5 * Fz) * ir;
        const real c2 = (real)((1.0 + R.at(0, k, 0, 0) - rd) * (1.0 / 3.0));  // p_m - rho/3
        F[n] = Fx;
        F[N + n] = Fy;
        F[2 * N + n] = Fz;
        phi[n] = c2 * ux;
        phi[N + n] = c2 * uy;
        phi[2 * N + n] = c2 * uz;
    });
}

template <int P> void chain_m(hipStream_t s, const KP &kp, const Bufs &b) {
    const unsigned g = nblocks(kp.N);
    const dim3 gz = zgrid(kp, 0, kp.nz);
    k_mu_z<<<gz, ZCB, 0, s>>>(kp, b.nbr, b.rho, b.mu, kZChunk);
    k_wall_mu_m<<<g, kBlock, 0, s>>>(kp, b.nbr, b.mu);
    k_fphi_z<P><<<gz, ZCB, 0, s>>>(kp, b.nbr, b.rho, b.j, b.mu, b.F, b.phi, kZChunk);
    if constexpr (P == LBFE_FP64)
        k_q_z<<<zgrid(kp, 0, kp.nz), ZCB, 0, s>>>(kp, b.nbr, (const double *)b.phi, (double *)b.Q, kZChunk);
    else
        k_q_m<P><<<g, kBlock, 0, s>>>(kp, b.nbr, b.phi, b.Q);
}

template <class Fn> hipError_t dispatch(int prec, Fn &&fn) {
    switch (prec) {
        case LBFE_FP64: return fn(std::integral_constant<int, LBFE_FP64>{});
        case LBFE_FP32: return fn(std::integral_constant<int, LBFE_FP32>{});
        case LBFE_FP16_DEV: return fn(std::integral_constant<int, LBFE_FP16_DEV>{});
        default: return fn(std::integral_constant<int, LBFE_FP16_DEV_F0FP32>{});
    }
}

}  // namespace

hipError_t launch_mask_prep(hipStream_t s, const KP &kp, const Bufs &b, const uint8_t *solid) {
    k_mask_prep<<<nblocks(kp.N), kBlock, 0, s>>>(kp, solid, b.nbr);
    return hipGetLastError();
}

hipError_t launch_aux_mask(hipStream_t s, int prec, const KP &kp, const Bufs &b, int cur) {
    return dispatch(prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        const unsigned g = nblocks(kp.N);
        k_moments_m<P><<<g, kBlock, 0, s>>>(kp, b.nbr, b.f[cur], b.rho, b.j, b.flag);
        k_wall_rho_m<<<g, kBlock, 0, s>>>(kp, b.nbr, b.rho);
        chain_m<P>(s, kp, b);
        return hipGetLastError();
    });
}

hipError_t launch_step_mask(hipStream_t s, int prec, const KP &kp, const Bufs &b, int cur, hipEvent_t *ev) {
    return dispatch(prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        const unsigned g = nblocks(kp.N);
        auto mark = [&](int k) {
            if (ev) (void)hipEventRecord(ev[k], s);
        };
        mark(0);
        k_moments_m<P><<<g, kBlock, 0, s>>>(kp, b.nbr, b.f[cur], b.rho, b.j, b.flag);
        k_wall_rho_m<<<g, kBlock, 0, s>>>(kp, b.nbr, b.rho);
        mark(1);
        chain_m<P>(s, kp, b);
        mark(2);
        k_collide_m<P><<<g, kBlock, 0, s>>>(kp, b.nbr, b.f[cur], b.f[1 - cur], b.mu, b.F, b.Q);
        mark(3);
        mark(4);
        return hipGetLastError();
    });
}

hipError_t launch_init_mask(hipStream_t s, int prec, const KP &kp, const Bufs &b, int cur, const double *rho0,
                            const double *u0) {
    return dispatch(prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        const unsigned g = nblocks(kp.N);
        k_copy_fluid_m<<<g, kBlock, 0, s>>>(kp, b.nbr, rho0, b.rho);
        k_wall_rho_m<<<g, kBlock, 0, s>>>(kp, b.nbr, b.rho);
        k_mu_m<<<g, kBlock, 0, s>>>(kp, b.nbr, b.rho, b.mu);
        k_init_m<P><<<g, kBlock, 0, s>>>(kp, b.nbr, b.rho, u0, b.mu, b.f[cur]);
        return hipGetLastError();
    });
}

hipError_t launch_init_aux_mask(hipStream_t s, const KP &kp, const Bufs &b, const double *rho0) {
    const unsigned g = nblocks(kp.N);
    k_copy_fluid_m<<<g, kBlock, 0, s>>>(kp, b.nbr, rho0, b.rho);
    k_wall_rho_m<<<g, kBlock, 0, s>>>(kp, b.nbr, b.rho);
    k_mu_m<<<g, kBlock, 0, s>>>(kp, b.nbr, b.rho, b.mu);
    return hipGetLastError();
}

hipError_t launch_check_rho0_mask(hipStream_t s, const KP &kp, const Bufs &b, const double *rho0, int *flag) {
    k_check_rho_m<<<nblocks(kp.N), kBlock, 0, s>>>(kp, b.nbr, rho0, flag);
    return hipGetLastError();
}

}  // namespace lbfe
