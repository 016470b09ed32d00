// Fused collide + push-stream + next-step moments of one time step on gfx950
// (Eqs. (10), (11), (21)-(26), (28), (32); halfway bounce-back at the walls).
//
// The step's population traffic is one read and one write of the 27
// populations per node: besides colliding and streaming its nodes, each
// workgroup forms the density and momentum of the next step, rho(t+1) =
// sum_i f*_i(x - c_i) and j(t+1) = sum_i c_i f*_i(x - c_i), from the
// post-collision values of its own nodes and of a one-node ring around them,
// so no separate pass has to read the streamed populations back.  It also
// writes mu0(rho(t+1)) for the stencil chain of the next step.
//
// Tile: 32 columns x RY rows, marching in z over a chunk of planes.  Wave w
// < RY/2 holds two interior rows (lanes 0-31 and 32-63), the next wave the
// two ring rows y0-1 and y0+RY, the last wave the 2 (RY+2) ring nodes at
// x0-1 and x0+32.  Every lane collides its node; interior lanes also push
// their populations to global memory.  The sums are taken in the order of
// moments() (lbfe_device.h):
//   x: a lane's right and left neighbours' populations arrive by DPP
//      whole-wave shifts, the tile-edge lanes take them from the x-ring
//      values in LDS; each lane forms the x-partials R, X of its 9 (cy, cz)
//      rows;
//   y: the partials with cy = +-1 go through LDS to the lanes one row up or
//      down;
//   z: three destination planes are in flight in registers; plane s-1 is
//      complete once source plane s has been added.
// The ring nodes are collided by the neighbouring tiles too (about 25% more
// collisions); their populations come mostly from L2.
#include <type_traits>

#include "lbfe_device.h"
#include "lbfe_dpp.h"

namespace lbfe {
namespace {

constexpr int FX = 32;  // interior columns of a tile (one half wave)

template <int RY> struct Geo {
    static_assert(RY % 2 == 0 && 2 * (RY + 2) <= 64, "tile rows");
    static constexpr int YR = RY / 2;      // the y-ring wave
    static constexpr int XR = RY / 2 + 1;  // the x-ring wave
    static constexpr int NT = 64 * (RY / 2 + 2);
    static constexpr int NROW = RY + 2;    // rows -1 .. RY
};

// Ordinary (cached) population loads: unlike the single-pass kernels, this
// one reads the one-node ring of its tile that the neighbouring tiles read
// too, and those re-reads should hit the cache.
__device__ inline double ld_cached(const Pops<LBFE_FP64> &f, int i, unsigned row, unsigned x) {
    return f.p[f.off(i, row, x)];
}
__device__ inline float ld_cached(const Pops<LBFE_FP32> &f, int i, unsigned row, unsigned x) {
    return f.p[f.off(i, row, x)];
}
__device__ inline float ld_cached(const Pops<LBFE_FP16_DEV> &f, int i, unsigned row, unsigned x) {
    return dec16(i, f.p[f.off(i, row, x)]);
}
__device__ inline float ld_cached(const Pops<LBFE_FP16_DEV_F0FP32> &f, int i, unsigned row, unsigned x) {
    return i == kRest ? f.p0[(size_t)row * f.nx + x] : dec16(i, f.p[f.off(i, row, x)]);
}

__device__ inline int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

struct Acc {  // partial moments of one destination plane
    double r, jx, jy, lp;
};

// Reflected layer of a node next to a wall: the populations that left
// toward the solid plane (direction cz = -side) come back as direction
// (-cx, -cy, side).
template <class real> __device__ inline Layer reflected_layer(const real (&q)[27], int side) {
    double R[3], X[3];
#pragma unroll
    for (int cy = -1; cy <= 1; ++cy)
        xpartial((double)q[dir(0, -cy, -side)], (double)q[dir(-1, -cy, -side)], (double)q[dir(1, -cy, -side)],
                 R[cy + 1], X[cy + 1]);
    return layer_of(R, X);
}

template <int P, int RY>
__global__ __launch_bounds__(Geo<RY>::NT) void k_fused(KP kp, const void *fin_q, void *fout_q,
                                                       const double *__restrict__ mu, const void *Fq, const void *Qq,
                                                       double *__restrict__ rho, void *jq, double *__restrict__ mu0,
                                                       int *flag, int cz) {
    using G = Geo<RY>;
    using real = typename Pol<P>::real;
    // y-exchange: [row + 1][slot][column], slot 2k (R) / 2k+1 (X) with
    // k = cz + 1 for the cy = +1 rows and k = 4 + cz for the cy = -1 rows
    __shared__ double ypart[G::NROW][12][FX];
    // x-ring populations entering the tile: [row + 1][0: from x0-1, 1: from x0+32][3 (cy+1) + cz+1]
    __shared__ real xring[G::NROW][2][9];

    const int ntx = (kp.nx + FX - 1) / FX;
    const unsigned ntiles = gridDim.x, nb = gridDim.x * gridDim.y;
    const unsigned hw = blockIdx.y * gridDim.x + blockIdx.x;
    const unsigned qq = nb >> 3, rem = nb & 7u, xcd = hw & 7u;
    const unsigned lid = xcd * qq + (xcd < rem ? xcd : rem) + (hw >> 3);  // XCD-contiguous order
    const int tile = (int)(lid % ntiles), chunk = (int)(lid / ntiles);
    const int x0 = (tile % ntx) * FX, y0 = (tile / ntx) * RY;
    const int zs = kp.z0 + chunk * cz;
    const int ze = min(zs + cz, kp.z1);

    const int w = threadIdx.x >> 6, l = threadIdx.x & 63;
    int a, b;
    bool live = true;
    if (w < G::YR) {
        b = 2 * w + (l >> 5);
        a = l & 31;
    } else if (w == G::YR) {
        b = l < 32 ? -1 : RY;
        a = l & 31;
    } else if (l < 2 * G::NROW) {
        b = (l >> 1) - 1;
        a = (l & 1) ? FX : -1;
    } else {
        b = 0;
        a = 0;
        live = false;
    }
    const bool inner = w < G::YR;
    const int x = wrapi(x0 + a, kp.nx), y = wrapi(y0 + b, kp.ny);
    const bool owner = inner && x0 + a < kp.nx && y0 + b < kp.ny;  // writes populations and moments
    const unsigned xo[3] = {(unsigned)(x == 0 ? kp.nx - 1 : x - 1), (unsigned)x,
                            (unsigned)(x == kp.nx - 1 ? 0 : x + 1)};
    const unsigned yo[3] = {(unsigned)(y == 0 ? kp.ny - 1 : y - 1), (unsigned)y,
                            (unsigned)(y == kp.ny - 1 ? 0 : y + 1)};
    const size_t N = kp.N;
    const Pops<P> fin(fin_q, kp), fout(fout_q, kp);
    const real *F = (const real *)Fq, *Qa = (const real *)Qq;
    real *J = (real *)jq;

    auto fluid = [&](int s) { return kp.walls ? (s >= 1 && s <= kp.nz - 2) : true; };
    auto zw = [&](int s) { return s < 0 ? s + kp.nz : (s >= kp.nz ? s - kp.nz : s); };  // |s| within one period

    real f[27];
    double m;
    real Fx, Fy, Fz, q200, q020, q002;
    auto load = [&](int s) {
        const int zz = zw(s);
        const unsigned row = (unsigned)zz * (unsigned)kp.ny + (unsigned)y;
#pragma unroll
        for (int i = 0; i < 27; ++i) f[i] = ld_cached(fin, i, row, (unsigned)x);
        const size_t n = (size_t)row * kp.nx + x;
        m = mu[n];
        Fx = F[n];
        Fy = F[N + n];
        Fz = F[2 * N + n];
        q200 = Qa[n];
        q020 = Qa[N + n];
        q002 = Qa[2 * N + n];
    };
    auto output = [&](int s, const Acc &A, double Lm) {
        const size_t n = ((size_t)s * kp.ny + y) * kp.nx + x;
        const double r = A.r + Lm;
        rho[n] = r;
        mu0[n] = mu_bulk(kp, r);
        J[n] = (real)A.jx;
        J[N + n] = (real)A.jy;
        J[2 * N + n] = (real)(A.lp - Lm);
        if (!(r > 0.0 && kp.b * r < 1.0)) *flag = 1;
    };

    Acc prev{0, 0, 0, 0}, cur{0, 0, 0, 0};
    if (fluid(zs - 1)) load(zs - 1);
    for (int s = zs - 1; s <= ze; ++s) {
        const bool sf = fluid(s);
        Layer Rb{0, 0, 0}, Rt{0, 0, 0};  // reflected layers at the bottom / top wall
        if (sf) {
            collide_node(kp, f, m, Fx, Fy, Fz, q200, q020, q002);
            const bool wall_lo = kp.walls && s == 1, wall_hi = kp.walls && s == kp.nz - 2;
            if (owner && s >= zs && s < ze) {
                const int zz = zw(s);
                const unsigned rz[3] = {(unsigned)zw(s - 1) * (unsigned)kp.ny, (unsigned)zz * (unsigned)kp.ny,
                                        (unsigned)zw(s + 1) * (unsigned)kp.ny};
#pragma unroll
                for (int i = 0; i < 27; ++i) {
                    const int cx = cxi(i), cy = cyi(i), c = czi(i);
                    if ((c < 0 && wall_lo) || (c > 0 && wall_hi))
                        fout.st(26 - i, rz[1] + yo[1], (unsigned)x, f[i]);
                    else
                        fout.st(i, rz[c + 1] + yo[cy + 1], xo[cx + 1], f[i]);
                }
            }
#pragma unroll
            for (int i = 0; i < 27; ++i) f[i] = Pops<P>::quant(i, f[i]);
            if (wall_lo) Rb = reflected_layer(f, 1);
            if (wall_hi) Rt = reflected_layer(f, -1);
            if (w == G::XR && live) {
                const int side = a < 0 ? 0 : 1, cx = a < 0 ? 1 : -1;
#pragma unroll
                for (int cy = -1; cy <= 1; ++cy)
#pragma unroll
                    for (int c = -1; c <= 1; ++c) xring[b + 1][side][3 * (cy + 1) + c + 1] = f[dir(cx, cy, c)];
            }
        }
        __syncthreads();

        double R0[3], X0[3];
        if (sf && w <= G::YR) {
#pragma unroll
            for (int cy = -1; cy <= 1; ++cy)
#pragma unroll
                for (int c = -1; c <= 1; ++c) {
                    real fp = shr1(f[dir(1, cy, c)]);
                    real fm = shl1(f[dir(-1, cy, c)]);
                    if (a == 0) fp = xring[b + 1][0][3 * (cy + 1) + c + 1];
                    if (a == FX - 1) fm = xring[b + 1][1][3 * (cy + 1) + c + 1];
                    double R, X;
                    xpartial((double)f[dir(0, cy, c)], (double)fp, (double)fm, R, X);
                    if (cy == 0) {
                        R0[c + 1] = R;
                        X0[c + 1] = X;
                    } else {
                        const int k = cy > 0 ? c + 1 : 4 + c;
                        ypart[b + 1][2 * k][a] = R;
                        ypart[b + 1][2 * k + 1][a] = X;
                    }
                }
        }
        // the populations of this plane are consumed: fetch the next plane
        if (s + 1 <= ze && fluid(s + 1)) load(s + 1);
        __syncthreads();

        if (sf && inner) {
            Layer Ly[3];
#pragma unroll
            for (int c = -1; c <= 1; ++c) {
                const double R[3] = {ypart[b + 2][2 * (4 + c)][a], R0[c + 1], ypart[b][2 * (c + 1)][a]};
                const double X[3] = {ypart[b + 2][2 * (4 + c) + 1][a], X0[c + 1], ypart[b][2 * (c + 1) + 1][a]};
                Ly[c + 1] = layer_of(R, X);
            }
            // plane s-1 is complete with the layer cz = -1 of this plane
            if (owner && s - 1 >= zs && s - 1 < ze && fluid(s - 1)) {
                Acc A = prev;
                A.jx += Ly[0].JX;
                A.jy += Ly[0].JY;
                output(zw(s - 1), A, Ly[0].L);
            }
            // plane s: its cz = +1 layer came from plane s-1, or from the
            // reflection at the bottom wall
            if (kp.walls && s == 1) cur = Acc{Rb.L, Rb.JX, Rb.JY, Rb.L};
            cur.r += Ly[1].L;
            cur.jx += Ly[1].JX;
            cur.jy += Ly[1].JY;
            if (kp.walls && s == kp.nz - 2 && owner && s >= zs && s < ze) {
                Acc A = cur;
                A.jx += Rt.JX;
                A.jy += Rt.JY;
                output(s, A, Rt.L);
            }
            prev = cur;
            cur = Acc{Ly[2].L, Ly[2].JX, Ly[2].JY, Ly[2].L};
        }
    }
}

// Planes per workgroup: long chunks amortise the two ring planes; enough
// workgroups to give every CU one.
int fused_chunk(const KP &kp, unsigned tiles) {
    const int nzf = kp.z1 - kp.z0;
    int cz = 64;
    while (cz > 8 && (size_t)tiles * ((nzf + cz - 1) / cz) < 256) cz /= 2;
    return cz;
}

template <int P, int RY> hipError_t launch(hipStream_t s, const KP &kp, const Bufs &b, int cur) {
    const unsigned ntx = (kp.nx + FX - 1) / FX, nty = (kp.ny + RY - 1) / RY;
    const int cz = fused_chunk(kp, ntx * nty);
    const int nzf = kp.z1 - kp.z0;
    const dim3 grid(ntx * nty, (nzf + cz - 1) / cz);
    k_fused<P, RY><<<grid, Geo<RY>::NT, 0, s>>>(kp, b.f[cur], b.f[1 - cur], b.mu, b.F, b.Q, b.rho, b.j, b.mu0,
                                                 b.flag, cz);
    return hipGetLastError();
}

}  // namespace

hipError_t launch_fused(hipStream_t s, int prec, const KP &kp, const Bufs &b, int cur) {
    switch (prec) {
        case LBFE_FP64: return launch<LBFE_FP64, 12>(s, kp, b, cur);
        case LBFE_FP32: return launch<LBFE_FP32, 16>(s, kp, b, cur);
        case LBFE_FP16_DEV: return launch<LBFE_FP16_DEV, 16>(s, kp, b, cur);
        default: return launch<LBFE_FP16_DEV_F0FP32, 16>(s, kp, b, cur);
    }
}

}  // namespace lbfe
