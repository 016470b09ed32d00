// The stencil chain of one step on gfx950, one kernel:
//   rho  -> mu = mu0 - kappa lap_h rho                      (Eq. (32))
//           (mu0 = mu0(rho) per node comes from the moments kernel)
//        -> solid-node mu by the wall average              (Eq. (36))
//   mu   -> G = grad_h mu, F = (1/3 - rho) G,               (Eq. (12))
//           u = (j + F/2)/rho, phi = (p_m - rho/3) u
//   phi  -> Q_aa = -3 d_a phi_a                              (Eq. (27))
//
// Each workgroup owns a 64 x 16 column tile and marches in z over a chunk of
// planes.  The isotropic D3Q27 stencils factor into D1Q3 pieces (weights
// 1/6, 2/3, 1/6 along each axis), so every stencil is evaluated as an
// in-plane part, read from one LDS plane, and a z part, combined in a
// three-plane register ring that each thread keeps for the columns it owns:
//   lap_h g = 6 (Wz (Wx Wy g) - g)
//   d_x g   = 1/2 Wz (Dx Wy g),  d_y g = 1/2 Wz (Wx Dy g),  d_z g = 1/2 Dz (Wx Wy g)
// with W the D1Q3 weights and D g = g(+1) - g(-1).  LDS holds a ring of three
// rho planes (tile + 4-node halo), two mu planes (3-node halo) and one phi
// plane (1-node halo).  Iteration k of the march loads rho(k+3), evaluates
// mu(k+2) and the in-plane parts of mu(k+2), then F and phi at k+1 and the
// in-plane parts of phi(k+1), and Q at k; global loads run ahead of their
// use.  Outputs per fluid node: mu (double), F and Q (compute precision);
// mu is also written at the solid planes.
#include <type_traits>

#include "lbfe_device.h"

namespace lbfe {
namespace {

constexpr int TX = 64, TY = 16;  // 1024 threads, one workgroup per CU (LDS)
constexpr int CB = TX * TY;                            // threads: one per tile column
constexpr int WR = TX + 8, HR = TY + 8, NR = WR * HR;  // rho region (halo 4)
constexpr int WM = TX + 6, HM = TY + 6, NM = WM * HM;  // mu region (halo 3)
constexpr int WP = TX + 2, HP = TY + 2, NP = WP * HP;  // phi region (halo 1)
constexpr int MR = (NR + CB - 1) / CB;         // rho points per thread
constexpr int MM = (NM + CB - 1) / CB;         // mu points per thread
constexpr int MP = (NP + CB - 1) / CB;         // phi points per thread
constexpr int NRP = MR * CB;                   // rho plane in LDS, padded to whole rounds
constexpr double A1 = 1.0 / 6.0, A0 = 2.0 / 3.0;       // D1Q3 weights

// Branch-free global access: raw buffer loads/stores through a descriptor
// of one plane; masked lanes use an offset past the plane, which the
// hardware drops (stores) or reads as zero (loads).  Keeping every global
// access outside lane-divergent branches lets the compiler count outstanding
// memory operations instead of draining them all at each plane.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr unsigned kOOB = 0x80000000u;
__device__ inline __amdgpu_buffer_rsrc_t plane_rsrc(const void *base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}
// The outputs mu, F, Q are stored non-temporal (cache-policy bit 2): the
// collide pass reads them once, after the whole chain, and the L2 is left to
// the stencil halos.
constexpr int kStoreNT = 2;
__device__ inline void bstore(double v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, v), r, off, 0, kStoreNT);
}
__device__ inline void bstore(float v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, v), r, off, 0, kStoreNT);
}
__device__ inline void bload(double &v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    v = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, off, 0, 0));
}
__device__ inline void bload(float &v, __amdgpu_buffer_rsrc_t r, unsigned off) {
    v = __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, off, 0, 0));
}

__device__ inline int wrap(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}
__device__ inline int slot3(int p) { return ((p % 3) + 3) % 3; }

// Wx Wy g of the 3x3 in-plane neighbourhood of index c in a row-major LDS
// plane with row stride W.
template <int W> __device__ inline double smooth2(const double *g, int c) {
    const double r0 = A1 * g[c - W - 1] + A0 * g[c - W] + A1 * g[c - W + 1];
    const double r1 = A1 * g[c - 1] + A0 * g[c] + A1 * g[c + 1];
    const double r2 = A1 * g[c + W - 1] + A0 * g[c + W] + A1 * g[c + W + 1];
    return A1 * r0 + A0 * r1 + A1 * r2;
}

template <int P, bool WALLS>
__global__ __launch_bounds__(CB) void k_chain(KP kp, const double *__restrict__ rho, const double *__restrict__ mu0,
                                              const void *jq, double *__restrict__ mu, void *Fq, void *Qq, int cz) {
    using real = typename Pol<P>::real;
    __shared__ double sr[3][NRP];
    __shared__ double sm[2][NM];
    __shared__ real sp[3][NP];

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

    // WALLS: solid planes z = 0 and z = nz-1 (kp.walls; a template argument,
    // so the periodic kernel carries none of the wall code)
    auto fluid = [&](int p) { return WALLS ? (p >= 1 && p <= kp.nz - 2) : true; };
    auto valid = [&](int p) { return !WALLS || (p >= 0 && p <= kp.nz - 1); };
    auto interior = [&](int a, int b) { return x0 + a < kp.nx && y0 + b < kp.ny; };
    // plane indices wrap periodically; inside the march they advance by one
    auto next = [&](int g) { return g + 1 == kp.nz ? 0 : g + 1; };
    auto pbase = [&](int g) { return (size_t)g * kp.plane; };

    // in-plane byte offsets of the owned rho-, mu- and phi-region points
    // (kOOB for lanes past the region)
    unsigned offr[MR], offm[MM], offp[MP];
#pragma unroll
    for (int m = 0; m < MR; ++m) {
        const int r = tid + m * CB;
        offr[m] = r < NR ? 8u * ((unsigned)wrap(y0 + r / WR - 4, kp.ny) * kp.nx + wrap(x0 + r % WR - 4, kp.nx)) : kOOB;
    }
#pragma unroll
    for (int m = 0; m < MM; ++m) {
        const int r = tid + m * CB;
        offm[m] = r < NM ? 8u * ((unsigned)wrap(y0 + r / WM - 3, kp.ny) * kp.nx + wrap(x0 + r % WM - 3, kp.nx)) : kOOB;
    }
#pragma unroll
    for (int m = 0; m < MP; ++m) {
        const int r = tid + m * CB;
        offp[m] = r < NP ? (unsigned)sizeof(real) *
                               ((unsigned)wrap(y0 + r / WP - 1, kp.ny) * kp.nx + wrap(x0 + r % WP - 1, kp.nx))
                         : kOOB;
    }
    const unsigned pbytes8 = kp.plane * 8u, pbytesr = kp.plane * (unsigned)sizeof(real);
    // byte offset of an interior tile point inside its plane, or kOOB
    auto ioff = [&](bool ok, int a, int b, unsigned esize) {
        return ok ? esize * ((unsigned)(y0 + b) * kp.nx + (x0 + a)) : kOOB;
    };
    // the store offsets of the owned mu-, phi- and tile points, once per
    // march (kOOB: not a point of the tile inside the grid)
    unsigned omu[MM], ofp[MP];
#pragma unroll
    for (int m = 0; m < MM; ++m) {
        const int r = tid + m * CB, a = r % WM, b = r / WM;
        omu[m] = ioff(r < NM && a >= 3 && b >= 3 && a < TX + 3 && b < TY + 3 && interior(a - 3, b - 3), a - 3, b - 3, 8u);
    }
#pragma unroll
    for (int m = 0; m < MP; ++m) {
        const int r = tid + m * CB, a = r % WP, b = r / WP;
        ofp[m] = ioff(r < NP && a >= 1 && b >= 1 && a <= TX && b <= TY && interior(a - 1, b - 1), a - 1, b - 1,
                      (unsigned)sizeof(real));
    }
    const unsigned oq = ioff(interior(tid % TX, tid / TX), tid % TX, tid / TX, (unsigned)sizeof(real));

    // Global loads run ahead of their use: rho one iteration ahead, mu0 and
    // j issued right after the stage that consumed the previous plane.
    // Loads of every plane index are issued (planes outside a walled box
    // wrap to valid memory and their values are never used).
    double pr[MR], m0[MM];
    real pj[MP][3];
    auto issue_rho = [&](int g) {
        const __amdgpu_buffer_rsrc_t rr = plane_rsrc(rho + pbase(g), pbytes8);
#pragma unroll
        for (int m = 0; m < MR; ++m) bload(pr[m], rr, offr[m]);
    };
    auto issue_mu0 = [&](int g) {
        const __amdgpu_buffer_rsrc_t rr = plane_rsrc(mu0 + pbase(g), pbytes8);
#pragma unroll
        for (int m = 0; m < MM; ++m) bload(m0[m], rr, offm[m]);
    };
    auto issue_j = [&](int g) {
        const size_t base = pbase(g);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const __amdgpu_buffer_rsrc_t rj = plane_rsrc(j + c * N + base, pbytesr);
#pragma unroll
            for (int m = 0; m < MP; ++m) bload(pj[m][c], rj, offp[m]);
        }
    };
    // every lane writes (the padding takes the lanes past the region, and a
    // plane outside a walled box is written but never read), so the commit
    // has no lane-divergent branch around the wait for its loads
    auto commit_rho = [&](int p) {
        const int s = slot3(p);
#pragma unroll
        for (int m = 0; m < MR; ++m) sr[s][tid + m * CB] = pr[m];
    };

    // register rings, index 0/1/2 = planes p-1, p, p+1 of the consumer
    double Pr[MM][3];                        // Wx Wy rho at owned mu points
    double Ar[MP][3], Br[MP][3], Cr[MP][3];  // Dx Wy mu, Wx Dy mu, Wx Wy mu at owned phi points
    real Xr[3], Yr[3], Zr[3];                // in-plane parts of the Q stencils at the tile point
#pragma unroll
    for (int m = 0; m < MM; ++m) Pr[m][0] = Pr[m][1] = Pr[m][2] = 0.0;
#pragma unroll
    for (int m = 0; m < MP; ++m)
#pragma unroll
        for (int t = 0; t < 3; ++t) Ar[m][t] = Br[m][t] = Cr[m][t] = 0.0;
#pragma unroll
    for (int t = 0; t < 3; ++t) Xr[t] = Yr[t] = Zr[t] = (real)0;

    // wall average (Eq. (36)) of mu plane pf into mu plane ps, on the points
    // with a halo of at most 2
    auto wall_mu = [&](int ps, int pf, bool write_out) {
        const int ss = ps & 1, sf = pf & 1;
        for (int r = tid; r < NM; r += CB) {
            const int a = r % WM, b = r / WM;
            if (a < 1 || a > WM - 2 || b < 1 || b > HM - 2) continue;
            const double v = smooth2<WM>(sm[sf], r);
            sm[ss][r] = v;
            if (write_out && a >= 3 && b >= 3 && a < TX + 3 && b < TY + 3 && interior(a - 3, b - 3))
                mu[pbase(ps) + (size_t)(y0 + b - 3) * kp.nx + (x0 + a - 3)] = v;
        }
    };
    // in-plane parts of grad mu from mu plane p at the owned phi point m
    auto abc = [&](int p, int m, double &Av, double &Bv, double &Cv) {
        const int r = tid + m * CB;
        const int c = (r / WP + 2) * WM + (r % WP + 2);
        const double *g = sm[p & 1];
        const double l0 = g[c - WM - 1], l1 = g[c - WM], l2 = g[c - WM + 1];
        const double m0 = g[c - 1], m1 = g[c], m2 = g[c + 1];
        const double h0 = g[c + WM - 1], h1 = g[c + WM], h2 = g[c + WM + 1];
        Av = A1 * (l2 - l0) + A0 * (m2 - m0) + A1 * (h2 - h0);
        Bv = A1 * (h0 - l0) + A0 * (h1 - l1) + A1 * (h2 - l2);
        Cv = A1 * (A1 * l0 + A0 * l1 + A1 * l2) + A0 * (A1 * m0 + A0 * m1 + A1 * m2) +
             A1 * (A1 * h0 + A0 * h1 + A1 * h2);
    };

    // wrapped indices of planes k, k+1, k+2, k+3, k+4
    int g0 = wrap(zs - 6, kp.nz);
    int g1 = next(g0), g2 = next(g1), g3 = next(g2), g4 = next(g3);
    issue_rho(g3);      // rho(zs - 3)
    issue_mu0(g2);      // mu0(zs - 4)
    issue_j(g1);        // j(zs - 5)
    for (int k = zs - 6; k < ze; ++k) {
        // ---- A: commit rho(k+3); prefetch rho(k+4)
        commit_rho(k + 3);
        __syncthreads();
        issue_rho(g4);

        // ---- B: Wx Wy rho(k+3) on the mu region; mu(k+2)
        {
            const int q3 = k + 3, p = k + 2;
            const bool pv = valid(q3);
            const int s3 = slot3(q3), s2 = slot3(p);
            const bool do_mu = p >= zs - 2 && fluid(p);
            const bool out_plane = p >= zs && p < ze;
            const bool full = WALLS && (p == 1 || p == kp.nz - 2);
            const __amdgpu_buffer_rsrc_t rmu = plane_rsrc(mu + pbase(g2), pbytes8);
#pragma unroll
            for (int m = 0; m < MM; ++m) {
                const int r = tid + m * CB;
                Pr[m][0] = Pr[m][1];
                Pr[m][1] = Pr[m][2];
                const int a = r % WM, b = r / WM;
                double v = 0.0;
                bool out = false;
                if (r < NM) {
                    const int c = (b + 1) * WR + (a + 1);  // the same point in the rho region
                    if (pv) Pr[m][2] = smooth2<WR>(sr[s3], c);
                    if (do_mu && (full || (a >= 1 && a <= WM - 2 && b >= 1 && b <= HM - 2))) {
                        const double r0 = sr[s2][c];
                        const double s27 = A1 * Pr[m][0] + A0 * Pr[m][1] + A1 * Pr[m][2];
                        v = m0[m] - kp.kappa * 6.0 * (s27 - r0);
                        sm[p & 1][r] = v;
                        out = out_plane;
                    }
                }
                bstore(v, rmu, out ? omu[m] : kOOB);
            }
            issue_mu0(g3);
            if constexpr (WALLS) {
                if (p == 1 && p >= zs - 2) {  // bottom solid plane, from the first fluid plane
                    __syncthreads();
                    wall_mu(0, 1, zs - 1 == 0);
                } else if (p == kp.nz - 1 && p >= zs - 2) {  // top solid plane
                    wall_mu(p, p - 1, p == ze);
                }
            }
        }
        __syncthreads();

        // ---- C: in-plane parts of mu(k+2); F and phi at k+1
        {
            const int p2 = k + 2, p1 = k + 1;
            const bool do_abc = p2 >= zs - 2 && valid(p2);
            const bool do_phi = p1 >= zs - 1;
            const bool fl1 = fluid(p1);
            const bool out_plane = p1 >= zs && p1 < ze;
            const size_t base1 = pbase(g1);
            const __amdgpu_buffer_rsrc_t rF0 = plane_rsrc(F + base1, pbytesr);
            const __amdgpu_buffer_rsrc_t rF1 = plane_rsrc(F + N + base1, pbytesr);
            const __amdgpu_buffer_rsrc_t rF2 = plane_rsrc(F + 2 * N + base1, pbytesr);
#pragma unroll
            for (int m = 0; m < MP; ++m) {
                const int r = tid + m * CB;
                Ar[m][0] = Ar[m][1];
                Ar[m][1] = Ar[m][2];
                Br[m][0] = Br[m][1];
                Br[m][1] = Br[m][2];
                Cr[m][0] = Cr[m][1];
                Cr[m][1] = Cr[m][2];
                const int a = r % WP, b = r / WP;
                real Fx = 0, Fy = 0, Fz = 0;
                bool out = false;
                if (r < NP) {
                    if (do_abc) abc(p2, m, Ar[m][2], Br[m][2], Cr[m][2]);
                    // the bottom solid plane's mu only exists from the step
                    // that evaluated the first fluid plane: refresh its entry
                    if (do_abc && WALLS && p2 == 1) abc(0, m, Ar[m][1], Br[m][1], Cr[m][1]);
                    if (do_phi && !fl1) sp[0][r] = sp[1][r] = sp[2][r] = (real)0;
                    if (do_phi && fl1) {
                        const double gx = 0.5 * (A1 * Ar[m][0] + A0 * Ar[m][1] + A1 * Ar[m][2]);
                        const double gy = 0.5 * (A1 * Br[m][0] + A0 * Br[m][1] + A1 * Br[m][2]);
                        const double gz = 0.5 * (Cr[m][2] - Cr[m][0]);
                        const double rd = sr[slot3(p1)][(b + 3) * WR + (a + 3)];
                        const double c1 = 1.0 / 3.0 - rd;
                        Fx = (real)(c1 * gx);
                        Fy = (real)(c1 * gy);
                        Fz = (real)(c1 * gz);
                        const real ir = (real)1 / (real)rd;
                        const real ux = (pj[m][0] + (real)0.5 * Fx) * ir;
                        const real uy = (pj[m][1] + (real)0.5 * Fy) * ir;
                        const real uz = (pj[m][2] + (real)0.5 * Fz) * ir;
                        // p_m - rho/3 with p_m = (1 + mu)/3
                        const real c2 = (real)((1.0 + sm[p1 & 1][(b + 2) * WM + (a + 2)] - rd) * (1.0 / 3.0));
                        sp[0][r] = c2 * ux;
                        sp[1][r] = c2 * uy;
                        sp[2][r] = c2 * uz;
                        out = out_plane;
                    }
                }
                const unsigned o = out ? ofp[m] : kOOB;
                bstore(Fx, rF0, o);
                bstore(Fy, rF1, o);
                bstore(Fz, rF2, o);
            }
            issue_j(g2);
        }
        __syncthreads();

        // ---- D: in-plane parts of phi(k+1); Q at k
        {
            const int p1 = k + 1, p0 = k;
            Xr[0] = Xr[1];
            Xr[1] = Xr[2];
            Yr[0] = Yr[1];
            Yr[1] = Yr[2];
            Zr[0] = Zr[1];
            Zr[1] = Zr[2];
            const int a = tid % TX, b = tid / TX;
            const int c = (b + 1) * WP + (a + 1);
            const real w1r = (real)A1, w0r = (real)A0;
            if (p1 >= zs - 1) {
                const real *gx = sp[0], *gy = sp[1], *gz = sp[2];
                Xr[2] = w1r * (gx[c - WP + 1] - gx[c - WP - 1]) + w0r * (gx[c + 1] - gx[c - 1]) +
                        w1r * (gx[c + WP + 1] - gx[c + WP - 1]);
                Yr[2] = w1r * (gy[c + WP - 1] - gy[c - WP - 1]) + w0r * (gy[c + WP] - gy[c - WP]) +
                        w1r * (gy[c + WP + 1] - gy[c - WP + 1]);
                Zr[2] = w1r * (w1r * gz[c - WP - 1] + w0r * gz[c - WP] + w1r * gz[c - WP + 1]) +
                        w0r * (w1r * gz[c - 1] + w0r * gz[c] + w1r * gz[c + 1]) +
                        w1r * (w1r * gz[c + WP - 1] + w0r * gz[c + WP] + w1r * gz[c + WP + 1]);
            }
            {
                const real h = (real)(-1.5);
                const size_t base0 = pbase(g0);
                const unsigned o = p0 >= zs && fluid(p0) ? oq : kOOB;
                bstore(h * (w1r * Xr[0] + w0r * Xr[1] + w1r * Xr[2]), plane_rsrc(Q + base0, pbytesr), o);
                bstore(h * (w1r * Yr[0] + w0r * Yr[1] + w1r * Yr[2]), plane_rsrc(Q + N + base0, pbytesr), o);
                bstore(h * (Zr[2] - Zr[0]), plane_rsrc(Q + 2 * N + base0, pbytesr), o);
            }
        }
        // no barrier: the next writes to the phi plane (stage C of k+1) and
        // to the mu ring (stage B of k+1) come after at least one barrier
        g0 = g1;
        g1 = g2;
        g2 = g3;
        g3 = g4;
        g4 = next(g4);
    }
}

}  // namespace

// Planes per workgroup.  One workgroup fits a CU (LDS), and every march
// starts with six pipeline-fill planes, so chunks of c planes cost the
// busiest CU ceil(workgroups / CUs) x (c + 6) plane iterations; the chunk
// length from 64 down to 1 that minimises it is taken (the longer on ties).
// (128-plane chunks, which the count favours at 512^3, measured slower.)
constexpr unsigned kCUs = 256;  // MI355X
static int chain_chunk(const KP &kp, unsigned tiles) {
    const int nzf = kp.z1 - kp.z0;
    auto iters = [&](int c) {
        const size_t wg = (size_t)tiles * ((nzf + c - 1) / c);
        return ((wg + kCUs - 1) / kCUs) * (size_t)(c + 6);
    };
    int cz = 64;
    for (int c = 32; c >= 1; c /= 2)
        if (iters(c) < iters(cz)) cz = c;
    return cz;
}

int chain_chunk_for(const KP &kp) {
    const unsigned ntx = (kp.nx + TX - 1) / TX, nty = (kp.ny + TY - 1) / TY;
    return kp.chain_cz > 0 ? kp.chain_cz : chain_chunk(kp, ntx * nty);
}

hipError_t launch_chain(hipStream_t s, int prec, const KP &kp, const Bufs &b) {
    const unsigned ntx = (kp.nx + TX - 1) / TX, nty = (kp.ny + TY - 1) / TY;
    const int cz = chain_chunk_for(kp);
    const int nzf = kp.z1 - kp.z0;
    const dim3 grid(ntx * nty, (nzf + cz - 1) / cz);
    auto go = [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        if (kp.walls)
            k_chain<P, true><<<grid, CB, 0, s>>>(kp, b.rho, b.mu0, b.j, b.mu, b.F, b.Q, cz);
        else
            k_chain<P, false><<<grid, CB, 0, s>>>(kp, b.rho, b.mu0, b.j, b.mu, b.F, b.Q, cz);
    };
    switch (prec) {
        case LBFE_FP64: go(std::integral_constant<int, LBFE_FP64>{}); break;
        case LBFE_FP32: go(std::integral_constant<int, LBFE_FP32>{}); break;
        case LBFE_FP16_DEV: go(std::integral_constant<int, LBFE_FP16_DEV>{}); break;
        default: go(std::integral_constant<int, LBFE_FP16_DEV_F0FP32>{}); break;
    }
    return hipGetLastError();
}

}  // namespace lbfe
