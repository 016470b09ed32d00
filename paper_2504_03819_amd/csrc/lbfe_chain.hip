// The stencil chain of one step on gfx950, one kernel:
//   rho  -> mu = mu0(rho) - kappa lap_h rho                 (Eq. (32))
//        -> solid-node mu by the wall average              (Eq. (36))
//   mu   -> G = grad_h mu, F = (1/3 - rho) G,               (Eq. (12))
//           u = (j + F/2)/rho, phi = (p_m - rho/3) u
//   phi  -> Q_aa = -3 d_a phi_a                              (Eq. (27))
// Each workgroup owns a TX x TY column tile and marches in z over a chunk
// of planes.  Three plane rings live in LDS: rho on the tile with a 4-node
// halo, mu with 3, phi with 1, so every neighbour read of the three
// 27-point stencils is an LDS read and each plane of rho is read from
// global memory once per tile.  mu is evaluated on a 2-node halo, or on the
// full 3-node halo next to a solid plane, whose wall average (Eq. (36)) is
// then needed on a 2-node halo.  The z-pipeline of iteration k loads
// rho(k+3), evaluates mu(k+2), then F, phi at k+1 and Q at k; the first
// chunk planes are recomputed as the pipeline fills.
// Outputs per fluid node: mu (double), F and Q (compute precision); mu is
// also written at the solid planes.
#include <type_traits>

#include "lbfe_device.h"

namespace lbfe {
namespace {

constexpr int TX = 16, TY = 16;
constexpr int WR = TX + 8, HR = TY + 8, NR = WR * HR;  // rho region (halo 4)
constexpr int WM = TX + 6, HM = TY + 6, NM = WM * HM;  // mu region (halo 3)
constexpr int WP = TX + 2, HP = TY + 2, NP = WP * HP;  // phi region (halo 1)

__device__ inline int wrap(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}
__device__ inline int slot3(int p) { return ((p % 3) + 3) % 3; }

template <int P>
__global__ __launch_bounds__(kBlock) void k_chain(KP kp, const double *__restrict__ rho, const void *jq,
                                                  double *__restrict__ mu, void *Fq, void *Qq, int cz) {
    using real = typename Pol<P>::real;
    __shared__ double sr[3][NR];
    __shared__ double sm[3][NM];
    __shared__ real sp[3][3][NP];

    // Workgroups are dealt round-robin to the 8 XCDs in linear order; the
    // linear id is remapped so that each XCD runs a contiguous range of
    // (chunk, tile) pairs, tiles of one chunk consecutively: neighbouring
    // tiles then share their halo planes through that XCD's L2.
    const int ntx = (kp.nx + TX - 1) / TX;
    const unsigned ntiles = gridDim.x, nb = gridDim.x * gridDim.y;
    const unsigned hw = blockIdx.y * gridDim.x + blockIdx.x;
    const unsigned q = nb >> 3, rem = nb & 7u, xcd = hw & 7u;
    const unsigned lid = xcd * q + (xcd < rem ? xcd : rem) + (hw >> 3);
    const int tile = (int)(lid % ntiles), chunk = (int)(lid / ntiles);
    const int x0 = (tile % ntx) * TX, y0 = (tile / ntx) * TY;
    const int zs = kp.z0 + chunk * cz;
    const int ze = min(zs + cz, kp.z1);
    const int tid = threadIdx.x;
    const size_t N = kp.N;
    const real *j = (const real *)jq;
    real *F = (real *)Fq;
    real *Q = (real *)Qq;

    auto fluid = [&](int p) { return kp.walls ? (p >= 1 && p <= kp.nz - 2) : true; };
    auto gplane = [&](int p) { return (size_t)wrap(p, kp.nz) * kp.plane; };
    auto interior = [&](int a, int b) { return x0 + a < kp.nx && y0 + b < kp.ny; };
    // global node of an interior tile point (never wraps)
    auto inode = [&](int a, int b, int p) {
        return gplane(p) + (size_t)(y0 + b) * kp.nx + (x0 + a);
    };
    // wall average of mu over the mu-region ring slot of fluid plane pf into
    // slot of solid plane ps, at region points with halo >= 1
    auto wall_mu = [&](int ps, int pf, bool write_out) {
        const int ss = slot3(ps), sf = slot3(pf);
        for (int r = tid; r < NM; r += kBlock) {
            const int a = r % WM, b = r / WM;
            if (a < 1 || a > WM - 2 || b < 1 || b > HM - 2) continue;
            double acc = 0.0;
#pragma unroll
            for (int cy = -1; cy <= 1; ++cy)
#pragma unroll
                for (int cx = -1; cx <= 1; ++cx) acc += w1(cx) * w1(cy) * sm[sf][(b + cy) * WM + a + cx];
            sm[ss][r] = acc;
            if (write_out && a >= 3 && b >= 3 && a < TX + 3 && b < TY + 3 && interior(a - 3, b - 3))
                mu[inode(a - 3, b - 3, ps)] = acc;
        }
    };

    // Global loads run one iteration ahead: rho(k+4) and j(k+2) are issued
    // into registers while iteration k computes from LDS, and committed to
    // LDS (rho) or used directly (j, by the thread that owns the point) in
    // iteration k+1.
    constexpr int MR = (NR + kBlock - 1) / kBlock, MP = (NP + kBlock - 1) / kBlock;
    // In-plane offsets of the region points this thread owns are the same on
    // every plane: computed once, with the periodic wrap, before the march.
    unsigned offr[MR], offp[MP];
#pragma unroll
    for (int m = 0; m < MR; ++m) {
        const int r = min(tid + m * kBlock, NR - 1);
        offr[m] = (unsigned)wrap(y0 + r / WR - 4, kp.ny) * kp.nx + wrap(x0 + r % WR - 4, kp.nx);
    }
#pragma unroll
    for (int m = 0; m < MP; ++m) {
        const int r = min(tid + m * kBlock, NP - 1);
        offp[m] = (unsigned)wrap(y0 + r / WP - 1, kp.ny) * kp.nx + wrap(x0 + r % WP - 1, kp.nx);
    }
    double pr[MR];
    real pj[MP][3];
    auto issue_rho = [&](int p) {
        if (kp.walls && (p < 0 || p > kp.nz - 1)) return;
        const size_t base = gplane(p);
#pragma unroll
        for (int m = 0; m < MR; ++m) {
            const int r = tid + m * kBlock;
            if (r < NR) pr[m] = rho[base + offr[m]];
        }
    };
    auto commit_rho = [&](int p) {
        if (kp.walls && (p < 0 || p > kp.nz - 1)) return;
        const int s = slot3(p);
#pragma unroll
        for (int m = 0; m < MR; ++m) {
            const int r = tid + m * kBlock;
            if (r < NR) sr[s][r] = pr[m];
        }
    };
    auto issue_j = [&](int p) {
        if (!fluid(p)) return;
        const size_t base = gplane(p);
#pragma unroll
        for (int m = 0; m < MP; ++m) {
            const int r = tid + m * kBlock;
            if (r < NP) {
                const size_t g = base + offp[m];
                pj[m][0] = j[g];
                pj[m][1] = j[N + g];
                pj[m][2] = j[2 * N + g];
            }
        }
    };
    real cj[MP][3];  // j of the plane stage C works on

    issue_rho(zs - 3);
    for (int k = zs - 6; k < ze; ++k) {
        // A: commit rho(k+3) (halo-4 region); take j(k+1); prefetch the next
        commit_rho(k + 3);
#pragma unroll
        for (int m = 0; m < MP; ++m)
            for (int c = 0; c < 3; ++c) cj[m][c] = pj[m][c];
        __syncthreads();
        issue_rho(k + 4);
        if (k + 2 >= zs - 1) issue_j(k + 2);
        // B: mu(k+2) on the halo-2 (or halo-3) region
        {
            const int p = k + 2;
            if (p >= zs - 2) {
                const bool out_plane = (p >= zs && p < ze) || (kp.walls && (p == zs - 1 || p == ze) && !fluid(p));
                if (fluid(p)) {
                    const int s0 = slot3(p - 1), s1 = slot3(p), s2 = slot3(p + 1), sd = slot3(p);
                    // full 3-node halo only where a wall average follows
                    const bool full = kp.walls && (p == 1 || p == kp.nz - 2);
                    for (int r = tid; r < NM; r += kBlock) {
                        const int a = r % WM, b = r / WM;
                        if (!full && (a < 1 || a > WM - 2 || b < 1 || b > HM - 2)) continue;
                        const int c = (b + 1) * WR + (a + 1);  // same point in the rho region
                        const double r0 = sr[s1][c];
                        double s = 0.0;
#pragma unroll
                        for (int i = 0; i < 27; ++i) {
                            if (i == kRest) continue;
                            const int ss = czi(i) < 0 ? s0 : (czi(i) > 0 ? s2 : s1);
                            s += wi(i) * (sr[ss][c + cyi(i) * WR + cxi(i)] - r0);
                        }
                        const double m = mu_bulk(kp, r0) - kp.kappa * 6.0 * s;
                        sm[sd][r] = m;
                        if (out_plane && a >= 3 && b >= 3 && a < TX + 3 && b < TY + 3 && interior(a - 3, b - 3))
                            mu[inode(a - 3, b - 3, p)] = m;
                    }
                    if (kp.walls && p == 1) {  // bottom solid plane from the first fluid plane
                        __syncthreads();
                        wall_mu(0, 1, zs - 1 == 0);
                    }
                } else if (kp.walls && p == kp.nz - 1) {  // top solid plane
                    wall_mu(p, p - 1, out_plane);
                }
            }
        }
        __syncthreads();
        // C: F, phi at k+1 on the halo-1 region
        {
            const int p = k + 1;
            if (p >= zs - 1) {
                const int sd = slot3(p);
                if (fluid(p)) {
                    const int s0 = slot3(p - 1), s1 = slot3(p), s2 = slot3(p + 1);
                    const bool out_plane = p >= zs && p < ze;
#pragma unroll
                    for (int m = 0; m < MP; ++m) {
                        const int r = tid + m * kBlock;
                        if (r >= NP) continue;
                        const int a = r % WP, b = r / WP;
                        const int cm = (b + 2) * WM + (a + 2);  // point in the mu region
                        double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
                        for (int i = 0; i < 27; ++i) {
                            if (i == kRest) continue;
                            const int ss = czi(i) < 0 ? s0 : (czi(i) > 0 ? s2 : s1);
                            const double m = wi(i) * sm[ss][cm + cyi(i) * WM + cxi(i)];
                            if (cxi(i)) gx += cxi(i) * m;
                            if (cyi(i)) gy += cyi(i) * m;
                            if (czi(i)) gz += czi(i) * m;
                        }
                        const double rd = sr[s1][(b + 3) * WR + (a + 3)];
                        const double c1 = 1.0 / 3.0 - rd;
                        const real Fx = (real)(c1 * 3.0 * gx), Fy = (real)(c1 * 3.0 * gy), Fz = (real)(c1 * 3.0 * gz);
                        const real rr = (real)rd;
                        const real ux = (cj[m][0] + (real)0.5 * Fx) / rr;
                        const real uy = (cj[m][1] + (real)0.5 * Fy) / rr;
                        const real uz = (cj[m][2] + (real)0.5 * Fz) / rr;
                        const double pm = (1.0 + sm[s1][cm]) / 3.0;
                        const real c2 = (real)(pm - rd / 3.0);
                        sp[sd][0][r] = c2 * ux;
                        sp[sd][1][r] = c2 * uy;
                        sp[sd][2][r] = c2 * uz;
                        if (out_plane && a >= 1 && b >= 1 && a <= TX && b <= TY && interior(a - 1, b - 1)) {
                            const size_t g = inode(a - 1, b - 1, p);
                            F[g] = Fx;
                            F[N + g] = Fy;
                            F[2 * N + g] = Fz;
                        }
                    }
                } else {
                    for (int r = tid; r < NP; r += kBlock) sp[sd][0][r] = sp[sd][1][r] = sp[sd][2][r] = (real)0;
                }
            }
        }
        __syncthreads();
        // D: Q at k on the tile
        {
            const int p = k;
            if (p >= zs && fluid(p)) {
                const int s0 = slot3(p - 1), s1 = slot3(p), s2 = slot3(p + 1);
                for (int r = tid; r < TX * TY; r += kBlock) {
                    const int a = r % TX, b = r / TX;
                    if (!interior(a, b)) continue;
                    const int c = (b + 1) * WP + (a + 1);
                    real sx = 0, sy = 0, sz = 0;
#pragma unroll
                    for (int u = -1; u <= 1; ++u)
#pragma unroll
                        for (int v = -1; v <= 1; ++v) {
                            const real w = (real)(w1(u) * w1(v));
                            // d_x phi_x: y offset u, z offset v
                            const int sv = v < 0 ? s0 : (v > 0 ? s2 : s1);
                            sx += w * (sp[sv][0][c + u * WP + 1] - sp[sv][0][c + u * WP - 1]);
                            // d_y phi_y: x offset u, z offset v
                            sy += w * (sp[sv][1][c + WP + u] - sp[sv][1][c - WP + u]);
                            // d_z phi_z: x offset u, y offset v
                            sz += w * (sp[s2][2][c + v * WP + u] - sp[s0][2][c + v * WP + u]);
                        }
                    const size_t g = inode(a, b, p);
                    Q[g] = (real)(-1.5) * sx;
                    Q[N + g] = (real)(-1.5) * sy;
                    Q[2 * N + g] = (real)(-1.5) * sz;
                }
            }
        }
        // no barrier here: the next writes to the phi ring (stage C of k+1)
        // come after two barriers
    }
}

}  // namespace

// Planes per workgroup: enough workgroups to fill the chip (>= ~2048),
// otherwise as long as possible to amortise the six pipeline-fill planes.
static int chain_chunk(const KP &kp, unsigned tiles) {
    const int nzf = kp.z1 - kp.z0;
    int cz = 32;
    while (cz > 8 && (size_t)tiles * ((nzf + cz - 1) / cz) < 2048) cz /= 2;
    return cz;
}

hipError_t launch_chain(hipStream_t s, int prec, const KP &kp, const Bufs &b) {
    const unsigned ntx = (kp.nx + TX - 1) / TX, nty = (kp.ny + TY - 1) / TY;
    const int cz = chain_chunk(kp, ntx * nty);
    const int nzf = kp.z1 - kp.z0;
    const dim3 grid(ntx * nty, (nzf + cz - 1) / cz);
    switch (prec) {
        case LBFE_FP64: k_chain<LBFE_FP64><<<grid, kBlock, 0, s>>>(kp, b.rho, b.j, b.mu, b.F, b.Q, cz); break;
        case LBFE_FP32: k_chain<LBFE_FP32><<<grid, kBlock, 0, s>>>(kp, b.rho, b.j, b.mu, b.F, b.Q, cz); break;
        case LBFE_FP16_DEV: k_chain<LBFE_FP16_DEV><<<grid, kBlock, 0, s>>>(kp, b.rho, b.j, b.mu, b.F, b.Q, cz); break;
        default: k_chain<LBFE_FP16_DEV_F0FP32><<<grid, kBlock, 0, s>>>(kp, b.rho, b.j, b.mu, b.F, b.Q, cz); break;
    }
    return hipGetLastError();
}

}  // namespace lbfe
