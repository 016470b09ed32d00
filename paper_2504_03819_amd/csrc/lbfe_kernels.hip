// Forward kernels of the D3Q27 chemical-potential free-energy LB step
// (arXiv:2504.03819, Sec. II B and Sec. III C) for gfx950.
//
// One time step t -> t+1 on the post-streaming state f(t):
//   k_chain     mu, mu at walls, F, u, phi and Q from rho, j, mu0 with
//               LDS-staged stencils (lbfe_chain.hip)
//                                              Eqs. (12), (27), (32), (36)
//   k_fused     CM transform, collision, inverse, push-stream with halfway
//               bounce-back, and rho, j, mu0 of f(t+1) (lbfe_fused.hip)
//                                  Eqs. (10), (11), (21)-(26), (28), (32)
//   k_wall_rho  density of the solid nodes (walls only)         Eqs. (37)-(38)
// k_moments forms rho (double), j = sum f c and mu0(rho) from stored
// populations when they were set from outside (Eqs. (11), (32)); k_collide
// is the collide-stream alone, for the unfused reference path.  Populations are row-blocked
// (each x-row holds its 27 populations as 27 contiguous runs); one thread per
// node, x fastest, so every population load and store of a wave64 is one
// contiguous 64-element run.
#include <mutex>
#include <type_traits>

#include "lbfe_device.h"

namespace lbfe {

// Scratch of the allocation-free reduction (lbfe_reduce_into): the block
// partials of k_reduce_part, one record of 8 doubles per workgroup of
// kBlock fluid nodes.  File-scope device memory that every GPU the library
// runs on holds until the process ends; host code reaches it only through
// the per-device address from hipGetSymbolAddress (the array's name is a
// host-side stand-in, not a device address).  Every record a call reads is
// written by that call first, so nothing needs clearing between calls.
static __device__ __align__(256) double scratch[8 * (size_t)kScratchPartials];

namespace {

template <int P> using real_t = typename Pol<P>::real;

// --------------------------------------------------------------------------
__global__ void k_fill(uint4 *p, size_t n16) {
    const size_t stride = (size_t)gridDim.x * blockDim.x;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

// --------------------------------------------------------------------------
template <int P>
__global__ __launch_bounds__(kBlock) void k_moments(KP kp, const void *fq, double *rho, void *jq, double *mu0,
                                                    int *flag) {
    using real = real_t<P>;
    const unsigned idx = tile_id(kp) * kBlock + threadIdx.x;
    if (idx >= kp.nfluid) return;
    const unsigned n = (unsigned)kp.z0 * kp.plane + idx;
    const unsigned row = n / (unsigned)kp.nx, x = n - row * (unsigned)kp.nx;
    const Pops<P> f(fq, kp);
    real v[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) v[i] = f.ld(i, row, x);
    double r;
    real jx, jy, jz;
    moments(v, r, jx, jy, jz);
    rho[n] = r;
    mu0[n] = mu_bulk(kp, r);
    real *j = (real *)jq;
    j[n] = jx;
    j[kp.N + n] = jy;
    j[2 * (size_t)kp.N + n] = jz;
    if (!(r > 0.0 && kp.b * r < 1.0)) *flag = 1;
}

// Weighted average over fluid neighbours of a solid node (Eqs. (36)/(37));
// neighbours outside the box or on the solid planes have s_w = 0.
__device__ inline double wall_average(const KP &kp, const double *g, int x, int y, int zs) {
    const int xm = x == 0 ? kp.nx - 1 : x - 1, xp = x == kp.nx - 1 ? 0 : x + 1;
    const int ym = y == 0 ? kp.ny - 1 : y - 1, yp = y == kp.ny - 1 ? 0 : y + 1;
    const int X[3] = {xm, x, xp}, Y[3] = {ym, y, yp};
    double num = 0.0, den = 0.0;
#pragma unroll
    for (int cz = -1; cz <= 1; ++cz) {
        const int zz = zs + cz;
        if (zz < 1 || zz > kp.nz - 2) continue;
#pragma unroll
        for (int cy = -1; cy <= 1; ++cy)
#pragma unroll
            for (int cx = -1; cx <= 1; ++cx) {
                const double w = wq(cx, cy, cz);
                num += w * g[(size_t)zz * kp.plane + (unsigned)Y[cy + 1] * kp.nx + X[cx + 1]];
                den += w;
            }
    }
    return num / den;
}

__global__ __launch_bounds__(kBlock) void k_wall_rho(KP kp, double *rho) {
    const unsigned idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= 2 * kp.plane) return;
    const int side = idx >= kp.plane;
    const unsigned p = idx - (side ? kp.plane : 0u);
    const int y = (int)(p / (unsigned)kp.nx), x = (int)(p - (unsigned)y * kp.nx);
    const int zs = side ? kp.nz - 1 : 0;
    const double rave = wall_average(kp, rho, x, y, zs);
    double out = rave;
    if (rave >= kp.lo && rave <= kp.hi) {  // contact-line window
        if (kp.wet_mode == LBFE_WET_PHI)
            out = fmin(fmax(kp.wet_value * rave, kp.lo), kp.hi);
        else if (kp.wet_mode == LBFE_WET_DELTA)
            out = fmin(fmax(rave - kp.wet_value, kp.lo), kp.hi);
    }
    rho[(size_t)zs * kp.plane + p] = out;
}

// mu = mu0(rho) - kappa lap_h rho, lap_h g = 6 sum_i w_i (g(x+c_i) - g(x)).
__global__ __launch_bounds__(kBlock) void k_mu(KP kp, const double *rho, double *mu) {
    const unsigned idx = tile_id(kp) * kBlock + threadIdx.x;
    if (idx >= kp.nfluid) return;
    const unsigned n = (unsigned)kp.z0 * kp.plane + idx;
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
    mu[n] = mu_bulk(kp, r0) - kp.kappa * 6.0 * s;
}

// Fused collide + stream of one fluid node (push: f*_i(x) -> x + c_i, or
// -> slot opp(i) of x when x + c_i is solid: halfway bounce-back).
template <int P>
__global__ __launch_bounds__(kBlock) void k_collide(KP kp, const void *fin_q, void *fout_q, const double *mu,
                                                    const void *Fq, const void *Qq) {
    using real = real_t<P>;
    const unsigned idx = tile_id(kp) * kBlock + threadIdx.x;
    if (idx >= kp.nfluid) return;
    const unsigned n = (unsigned)kp.z0 * kp.plane + idx;
    int x, y, z;
    decompose(kp, n, x, y, z);
    const Nb nb(kp, x, y, z);
    const Pops<P> fin(fin_q, kp);
    const Pops<P> fout(fout_q, kp);
    const unsigned row = nb.row(0, 0);

    real f[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) f[i] = fin.ld(i, row, (unsigned)x);
    const real *F = (const real *)Fq, *Qa = (const real *)Qq;
    // the aux fields are read once; non-temporal in the FP64 and FP32 forms
    // (measured neutral to slightly slower in the FP16 forms)
    constexpr bool nt = P == LBFE_FP64 || P == LBFE_FP32;
    auto ld = [&](const auto *p) { return nt ? ldnt(p) : *p; };
    collide_node(kp, f, ld(mu + n), ld(F + n), ld(F + kp.N + n), ld(F + 2 * (size_t)kp.N + n), ld(Qa + n),
                 ld(Qa + kp.N + n), ld(Qa + 2 * (size_t)kp.N + n));

    const bool wall_lo = kp.walls && z == 1;
    const bool wall_hi = kp.walls && z == kp.nz - 2;
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const int cz = czi(i);
        if ((cz < 0 && wall_lo) || (cz > 0 && wall_hi))
            fout.st(26 - i, row, (unsigned)x, f[i]);
        else
            fout.st(i, nb.row(cyi(i), cz), nb.xo(cxi(i)), f[i]);
    }
}

// Moving walls (after k_collide): the populations reflected at a wall of
// velocity u_w take the odd part of the Eq. (20) equilibrium at u_w,
// f_opp(i)(x, t+1) = f*_i(x) - [f^eq_i - f^eq_opp(i)](rho(x), p_m(x), u_w), for
// the first and last fluid planes (2 nx ny threads).  rho and mu are those
// of f(t), the state k_collide collided.
template <int P> __global__ __launch_bounds__(kBlock) void k_wall_move(KP kp, void *fq, const double *rho,
                                                                       const double *mu) {
    using real = real_t<P>;
    const unsigned idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= 2 * kp.plane) return;
    const int side = idx >= kp.plane;  // 0: next to the bottom wall, 1: top
    const unsigned p = idx - (side ? kp.plane : 0u);
    const int z = side ? kp.nz - 2 : 1;
    if (side && z == 1) return;  // one fluid plane: both walls handled by side 0
    const unsigned y = p / (unsigned)kp.nx, x = p - y * (unsigned)kp.nx;
    const size_t n = (size_t)z * kp.plane + p;
    const unsigned row = (unsigned)z * (unsigned)kp.ny + y;
    const Pops<P> f(fq, kp);
    const real r = (real)rho[n], pm = (real)((1.0 + mu[n]) * (1.0 / 3.0));
    real fe[27];
    for (int w = 0; w < 2; ++w) {  // bottom, top
        const bool hit = w == 0 ? z == 1 : z == kp.nz - 2;
        if (!hit) continue;
        wall_equilibrium(r, pm, (real)kp.wall_u[2 * w], (real)kp.wall_u[2 * w + 1], fe);
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const int cz = czi(i);
            if ((w == 0 && cz < 0) || (w == 1 && cz > 0))
                f.st(26 - i, row, x, f.ld(26 - i, row, x) - (fe[i] - fe[26 - i]));
        }
    }
}

// Moving walls on the fused path.  k_fused reflects at the walls without the
// wall-velocity term and overwrites rho of the first and last fluid planes
// with rho(t+1).  k_wall_keep first copies rho(t) of those planes into the
// density slots of the adjacent solid planes, which nothing reads before
// k_wall_rho refills them; k_wall_move_fused then applies the term exactly
// as k_wall_move does and forms rho, j, mu0 of the corrected nodes again
// from their stored populations, as k_moments would (so the fused path with
// moving walls gives the two-pass path's bits).
__global__ __launch_bounds__(kBlock) void k_wall_keep(KP kp, double *rho) {
    const unsigned p = blockIdx.x * kBlock + threadIdx.x;
    if (p >= kp.plane) return;
    rho[p] = rho[kp.plane + p];
    rho[(size_t)(kp.nz - 1) * kp.plane + p] = rho[(size_t)(kp.nz - 2) * kp.plane + p];
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_wall_move_fused(KP kp, void *fq, double *rho, const double *mu, void *jq,
                                                          double *mu0, int *flag) {
    using real = real_t<P>;
    const unsigned idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= 2 * kp.plane) return;
    const int side = idx >= kp.plane;
    const unsigned p = idx - (side ? kp.plane : 0u);
    const int z = side ? kp.nz - 2 : 1;
    if (side && z == 1) return;  // one fluid plane: both walls handled by side 0
    const unsigned y = p / (unsigned)kp.nx, x = p - y * (unsigned)kp.nx;
    const size_t n = (size_t)z * kp.plane + p;
    const unsigned row = (unsigned)z * (unsigned)kp.ny + y;
    const Pops<P> f(fq, kp);
    const double rt = rho[(size_t)(side ? kp.nz - 1 : 0) * kp.plane + p];  // rho(t), kept by k_wall_keep
    const real r = (real)rt, pm = (real)((1.0 + mu[n]) * (1.0 / 3.0));
    real fe[27];
    for (int w = 0; w < 2; ++w) {  // bottom, top
        const bool hit = w == 0 ? z == 1 : z == kp.nz - 2;
        if (!hit) continue;
        wall_equilibrium(r, pm, (real)kp.wall_u[2 * w], (real)kp.wall_u[2 * w + 1], fe);
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const int cz = czi(i);
            if ((w == 0 && cz < 0) || (w == 1 && cz > 0))
                f.st(26 - i, row, x, f.ld(26 - i, row, x) - (fe[i] - fe[26 - i]));
        }
    }
    real v[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) v[i] = f.ld(i, row, x);
    double rn;
    real jx, jy, jz;
    moments(v, rn, jx, jy, jz);
    rho[n] = rn;
    mu0[n] = mu_bulk(kp, rn);
    real *j = (real *)jq;
    j[n] = jx;
    j[kp.N + n] = jy;
    j[2 * (size_t)kp.N + n] = jz;
    if (!(rn > 0.0 && kp.b * rn < 1.0)) *flag = 1;
}

// Initial populations: inverse CM transform of the Eq. (20) equilibrium.
template <int P>
__global__ __launch_bounds__(kBlock) void k_init(KP kp, const double *rho0, const double *u0, const double *mu,
                                                 void *fq) {
    using real = real_t<P>;
    const unsigned idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= kp.nfluid) return;
    const unsigned n = (unsigned)kp.z0 * kp.plane + idx;
    real k[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) k[i] = 0;
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
    const Pops<P> f(fq, kp);
    const unsigned row = n / (unsigned)kp.nx, x = n - row * (unsigned)kp.nx;
#pragma unroll
    for (int i = 0; i < 27; ++i) f.st(i, row, x, k[i]);
}

__global__ __launch_bounds__(kBlock) void k_copy_fluid(KP kp, const double *src, double *dst) {
    const unsigned idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= kp.nfluid) return;
    const unsigned n = (unsigned)kp.z0 * kp.plane + idx;
    dst[n] = src[n];
}

__global__ __launch_bounds__(kBlock) void k_check_rho(KP kp, const double *rho, int *flag) {
    const unsigned idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= kp.nfluid) return;
    const double r = rho[(unsigned)kp.z0 * kp.plane + idx];
    if (!(r > 0.0 && kp.b * r < 1.0)) *flag = 1;
}

// Field export of the current state (aux arrays already evaluated).
template <int P>
__global__ __launch_bounds__(kBlock) void k_export(KP kp, int which, const double *rho, const void *jq,
                                                   const double *mu, const void *Fq, const void *Qq,
                                                   const unsigned *nbr, double *out) {
    using real = real_t<P>;
    const unsigned n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    int x, y, z;
    decompose(kp, n, x, y, z);
    const bool fluid = kp.masked ? !(nbr[n] & (1u << kRest)) : (z >= kp.z0 && z < kp.z1);
    const size_t N = kp.N;
    const real *F = (const real *)Fq;
    switch (which) {
        case LBFE_FIELD_RHO: out[n] = rho[n]; break;
        case LBFE_FIELD_MU: out[n] = mu[n]; break;
        case LBFE_FIELD_PM: out[n] = (1.0 + mu[n]) / 3.0; break;
        case LBFE_FIELD_F:
            for (int a = 0; a < 3; ++a) out[a * N + n] = fluid ? (double)F[a * N + n] : 0.0;
            break;
        case LBFE_FIELD_U: {
            const real *j = (const real *)jq;
            const real rr = (real)rho[n];
            for (int a = 0; a < 3; ++a)
                out[a * N + n] = fluid ? (double)((j[a * N + n] + (real)0.5 * F[a * N + n]) / rr) : 0.0;
            break;
        }
        case LBFE_FIELD_Q: {
            const real *Qa = (const real *)Qq;
            for (int a = 0; a < 3; ++a) out[a * N + n] = fluid ? (double)Qa[a * N + n] : 0.0;
            break;
        }
        default: break;
    }
}

// Deterministic reductions: fixed per-block tree, then one block over the
// block partials in a fixed order.
template <int P>
__global__ __launch_bounds__(kBlock) void k_reduce_part(KP kp, const double *rho, const void *jq, const void *Fq,
                                                        const unsigned *nbr, double *part) {
    using real = real_t<P>;
    __shared__ double s[8][kBlock];
    const unsigned idx = blockIdx.x * kBlock + threadIdx.x;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    if (idx < kp.nfluid && !(kp.masked && (nbr[(unsigned)kp.z0 * kp.plane + idx] & (1u << kRest)))) {
        const unsigned n = (unsigned)kp.z0 * kp.plane + idx;
        const size_t N = kp.N;
        const real *j = (const real *)jq, *F = (const real *)Fq;
        const double r = rho[n];
        v[0] = r;
        double u2 = 0.0;
        for (int a = 0; a < 3; ++a) {
            v[1 + a] = (double)j[a * N + n];
            v[4 + a] = (double)F[a * N + n];
            const double u = ((double)j[a * N + n] + 0.5 * (double)F[a * N + n]) / r;
            u2 += u * u;
        }
        v[7] = sqrt(u2);
    }
    for (int k = 0; k < 8; ++k) s[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            for (int k = 0; k < 7; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + h];
            s[7][threadIdx.x] = fmax(s[7][threadIdx.x], s[7][threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 8) part[(size_t)blockIdx.x * 8 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(kBlock) void k_reduce_final(unsigned nblk, const double *part, double *out) {
    __shared__ double s[8][kBlock];
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    for (unsigned b = threadIdx.x; b < nblk; b += kBlock) {
        for (int k = 0; k < 7; ++k) v[k] += part[(size_t)b * 8 + k];
        v[7] = fmax(v[7], part[(size_t)b * 8 + 7]);
    }
    for (int k = 0; k < 8; ++k) s[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            for (int k = 0; k < 7; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + h];
            s[7][threadIdx.x] = fmax(s[7][threadIdx.x], s[7][threadIdx.x + h]);
        }
        __syncthreads();
    }
    if (threadIdx.x < 8) out[threadIdx.x] = s[threadIdx.x][0];
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_get_pop(KP kp, const void *fq, const unsigned *nbr, double *out) {
    const unsigned n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    const unsigned z = n / kp.plane;
    const bool fluid = kp.masked ? !(nbr[n] & (1u << kRest)) : ((int)z >= kp.z0 && (int)z < kp.z1);
    const Pops<P> f(fq, kp);
    const unsigned row = n / (unsigned)kp.nx, x = n - row * (unsigned)kp.nx;
#pragma unroll
    for (int i = 0; i < 27; ++i) out[(size_t)i * kp.N + n] = fluid ? (double)f.ld(i, row, x) : 0.0;
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_set_pop(KP kp, void *fq, const unsigned *nbr, const double *in) {
    const unsigned idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= kp.nfluid) return;
    const unsigned n = (unsigned)kp.z0 * kp.plane + idx;
    const bool solid = kp.masked && (nbr[n] & (1u << kRest));  // solid nodes hold no populations
    const Pops<P> f(fq, kp);
    const unsigned row = n / (unsigned)kp.nx, x = n - row * (unsigned)kp.nx;
#pragma unroll
    for (int i = 0; i < 27; ++i) f.st(i, row, x, solid ? (real_t<P>)0 : (real_t<P>)in[(size_t)i * kp.N + n]);
}

// --------------------------------------------------------------------------
// One step's launches.  With `ev` non-null, HIP events ev[0..4] bracket the
// four kernel classes in the order: moments (with the wall density that
// follows them), chain, collide-stream, wall density after the step.
template <int P>
hipError_t aux_impl(hipStream_t s, const KP &kp, const Bufs &b, int cur) {
    const unsigned gf = nblocks(kp.nfluid), gw = nblocks(2 * (size_t)kp.plane);
    k_moments<P><<<gf, kBlock, 0, s>>>(kp, b.f[cur], b.rho, b.j, b.mu0, b.flag);
    if (kp.walls) k_wall_rho<<<gw, kBlock, 0, s>>>(kp, b.rho);
    hipError_t e = launch_chain(s, P, kp, b);
    if (e != hipSuccess) return e;
    return hipGetLastError();
}

// Fused path: rho, j, mu0 of f[cur] are current unless `refresh`; the fused
// kernel leaves them current for f[1 - cur].
template <int P>
hipError_t step_impl(hipStream_t s, const KP &kp, const Bufs &b, int cur, bool fused, bool refresh,
                     hipEvent_t *ev) {
    const unsigned gf = nblocks(kp.nfluid), gw = nblocks(2 * (size_t)kp.plane);
    auto mark = [&](int k) {
        if (ev) (void)hipEventRecord(ev[k], s);
    };
    mark(0);
    if (refresh || !fused) {
        k_moments<P><<<gf, kBlock, 0, s>>>(kp, b.f[cur], b.rho, b.j, b.mu0, b.flag);
        if (kp.walls) k_wall_rho<<<gw, kBlock, 0, s>>>(kp, b.rho);
    }
    mark(1);
    hipError_t e = launch_chain(s, P, kp, b);
    if (e != hipSuccess) return e;
    mark(2);
    if (fused) {
        if (kp.moving) k_wall_keep<<<nblocks(kp.plane), kBlock, 0, s>>>(kp, b.rho);
        e = launch_fused(s, P, kp, b, cur);
        if (e != hipSuccess) return e;
        if (kp.moving) k_wall_move_fused<P><<<gw, kBlock, 0, s>>>(kp, b.f[1 - cur], b.rho, b.mu, b.j, b.mu0, b.flag);
    } else {
        k_collide<P><<<nblocks(kp.nfluid), kBlock, 0, s>>>(kp, b.f[cur], b.f[1 - cur], b.mu, b.F, b.Q);
        if (kp.moving) k_wall_move<P><<<gw, kBlock, 0, s>>>(kp, b.f[1 - cur], b.rho, b.mu);
    }
    mark(3);
    if (fused && kp.walls) k_wall_rho<<<gw, kBlock, 0, s>>>(kp, b.rho);
    mark(4);
    return hipGetLastError();
}

template <int P>
hipError_t init_impl(hipStream_t s, const KP &kp, const Bufs &b, int cur, const double *rho0, const double *u0) {
    const unsigned gf = nblocks(kp.nfluid), gw = nblocks(2 * (size_t)kp.plane);
    k_copy_fluid<<<gf, kBlock, 0, s>>>(kp, rho0, b.rho);
    if (kp.walls) k_wall_rho<<<gw, kBlock, 0, s>>>(kp, b.rho);
    k_mu<<<gf, kBlock, 0, s>>>(kp, b.rho, b.mu);
    k_init<P><<<gf, kBlock, 0, s>>>(kp, b.rho, u0, b.mu, b.f[cur]);
    return hipGetLastError();
}

// Run f(std::integral_constant<int, P>) for the storage form P = prec.
template <class Fn> hipError_t dispatch(int prec, Fn &&fn) {
    switch (prec) {
        case LBFE_FP64: return fn(std::integral_constant<int, LBFE_FP64>{});
        case LBFE_FP32: return fn(std::integral_constant<int, LBFE_FP32>{});
        case LBFE_FP16_DEV: return fn(std::integral_constant<int, LBFE_FP16_DEV>{});
        default: return fn(std::integral_constant<int, LBFE_FP16_DEV_F0FP32>{});
    }
}

}  // namespace

hipError_t launch_fill(hipStream_t s, void *p, size_t bytes) {
    const size_t n16 = bytes / 16;
    if (!n16) return hipSuccess;
    unsigned g = (unsigned)((n16 + kBlock - 1) / kBlock);
    if (g > 65536) g = 65536;
    k_fill<<<g, kBlock, 0, s>>>((uint4 *)p, n16);
    return hipGetLastError();
}

hipError_t launch_init(hipStream_t s, int prec, const KP &kp, const Bufs &b, int cur, const double *rho0,
                       const double *u0) {
    if (kp.masked) return launch_init_mask(s, prec, kp, b, cur, rho0, u0);
    return dispatch(prec, [&](auto pc) { return init_impl<decltype(pc)::value>(s, kp, b, cur, rho0, u0); });
}

hipError_t launch_aux(hipStream_t s, int prec, const KP &kp, const Bufs &b, int cur) {
    if (kp.masked) return launch_aux_mask(s, prec, kp, b, cur);
    return dispatch(prec, [&](auto pc) { return aux_impl<decltype(pc)::value>(s, kp, b, cur); });
}

hipError_t launch_step(hipStream_t s, int prec, const KP &kp, const Bufs &b, int cur, bool fused, bool refresh,
                       hipEvent_t *ev5) {
    if (kp.masked) return launch_step_mask(s, prec, kp, b, cur, ev5);
    return dispatch(prec,
                    [&](auto pc) { return step_impl<decltype(pc)::value>(s, kp, b, cur, fused, refresh, ev5); });
}

// Moment-state launch groups (the kernels are in lbfe_moment.hip)
hipError_t launch_state_enter(hipStream_t s, int prec, const KP &kp, const Bufs &b, int cur, bool refresh,
                              hipEvent_t *ev) {
    const unsigned gf = nblocks(kp.nfluid), gw = nblocks(2 * (size_t)kp.plane);
    if (ev) (void)hipEventRecord(ev[0], s);
    if (refresh) {
        hipError_t e = dispatch(prec, [&](auto pc) {
            k_moments<decltype(pc)::value><<<gf, kBlock, 0, s>>>(kp, b.f[cur], b.rho, b.j, b.mu0, b.flag);
            return hipGetLastError();
        });
        if (e != hipSuccess) return e;
        if (kp.walls) k_wall_rho<<<gw, kBlock, 0, s>>>(kp, b.rho);
    }
    hipError_t e = launch_chain(s, prec, kp, b);
    if (e != hipSuccess) return e;
    if (ev) (void)hipEventRecord(ev[1], s);
    e = launch_state_first(s, prec, kp, b, b.f[cur], b.f[1 - cur]);
    if (ev) (void)hipEventRecord(ev[2], s);
    return e;
}

hipError_t launch_state_moments(hipStream_t s, int prec, const KP &kp, const Bufs &b, int a, bool pops,
                                hipEvent_t *ev) {
    if (ev) (void)hipEventRecord(ev[0], s);
    hipError_t e = launch_state_pass(s, prec, pops ? kStatePops : kStateMoments, kp, b, b.f[a], pops ? b.f[1 - a] : nullptr);
    if (e != hipSuccess) return e;
    if (kp.walls) k_wall_rho<<<nblocks(2 * (size_t)kp.plane), kBlock, 0, s>>>(kp, b.rho);
    if (ev) (void)hipEventRecord(ev[1], s);
    return hipGetLastError();
}

hipError_t launch_state_collide(hipStream_t s, int prec, const KP &kp, const Bufs &b, int a, hipEvent_t *ev) {
    if (ev) (void)hipEventRecord(ev[0], s);
    hipError_t e = launch_chain(s, prec, kp, b);
    if (e != hipSuccess) return e;
    if (ev) (void)hipEventRecord(ev[1], s);
    e = launch_state_pass(s, prec, kStateCollide, kp, b, b.f[a], b.f[1 - a]);
    if (ev) (void)hipEventRecord(ev[2], s);
    return e;
}

hipError_t launch_export(hipStream_t s, int prec, const KP &kp, const Bufs &b, int which, double *out) {
    return dispatch(prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        k_export<P><<<nblocks(kp.N), kBlock, 0, s>>>(kp, which, b.rho, b.j, b.mu, b.F, b.Q, b.nbr, out);
        return hipGetLastError();
    });
}

hipError_t launch_reduce(hipStream_t s, int prec, const KP &kp, const Bufs &b) {
    const unsigned g = nblocks(kp.nfluid);
    return dispatch(prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        k_reduce_part<P><<<g, kBlock, 0, s>>>(kp, b.rho, b.j, b.F, b.nbr, b.part);
        k_reduce_final<<<1, kBlock, 0, s>>>(g, b.part, b.red);
        return hipGetLastError();
    });
}

hipError_t scratch_partials(int device, double **out) {
    static std::mutex mu;
    static double *ptr[kMaxDevices] = {};
    if (device < 0 || device >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(mu);
    if (!ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess) return e;
        ptr[device] = (double *)p;
    }
    *out = ptr[device];
    return hipSuccess;
}

hipError_t launch_reduce_into(hipStream_t s, int prec, const KP &kp, const Bufs &b, double *part, double *out) {
    const unsigned g = nblocks(kp.nfluid);
    if (g > kScratchPartials) return hipErrorInvalidValue;
    return dispatch(prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        k_reduce_part<P><<<g, kBlock, 0, s>>>(kp, b.rho, b.j, b.F, b.nbr, part);
        k_reduce_final<<<1, kBlock, 0, s>>>(g, part, out);
        return hipGetLastError();
    });
}

hipError_t launch_get_pop(hipStream_t s, int prec, const KP &kp, const Bufs &b, const void *f, double *out) {
    return dispatch(prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        k_get_pop<P><<<nblocks(kp.N), kBlock, 0, s>>>(kp, f, b.nbr, out);
        return hipGetLastError();
    });
}

hipError_t launch_set_pop(hipStream_t s, int prec, const KP &kp, const Bufs &b, void *f, const double *in) {
    return dispatch(prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        k_set_pop<P><<<nblocks(kp.nfluid), kBlock, 0, s>>>(kp, f, b.nbr, in);
        return hipGetLastError();
    });
}

hipError_t launch_init_aux(hipStream_t s, const KP &kp, const Bufs &b, const double *rho0) {
    if (kp.masked) return launch_init_aux_mask(s, kp, b, rho0);
    const unsigned gf = nblocks(kp.nfluid), gw = nblocks(2 * (size_t)kp.plane);
    k_copy_fluid<<<gf, kBlock, 0, s>>>(kp, rho0, b.rho);
    if (kp.walls) k_wall_rho<<<gw, kBlock, 0, s>>>(kp, b.rho);
    k_mu<<<gf, kBlock, 0, s>>>(kp, b.rho, b.mu);
    return hipGetLastError();
}

hipError_t launch_check_rho0(hipStream_t s, const KP &kp, const double *rho0, int *flag) {
    k_check_rho<<<nblocks(kp.nfluid), kBlock, 0, s>>>(kp, rho0, flag);
    return hipGetLastError();
}

}  // namespace lbfe
