// Discrete adjoint of the D3Q27 free-energy LB step: lambda(t) =
// (d f(t+1) / d f(t))^T lambda(t+1) for the forward map of lbfe_kernels.hip,
// plus the adjoint of the initialiser and the parameter gradients
// dL/dkappa, dL/d(wet_value), dL/dnu.  (The adjoint is not part of the
// paper; it differentiates the paper's discrete update exactly.)
//
// Per adjoint step, after the forward auxiliary fields of f(t) have been
// recomputed (launch_aux):
//   k_adj_collide   pull-gather lambda*(x) = lambda(t+1)(x + c_i) (or the
//                   bounce-back slot), local collision adjoint in central-
//                   moment space; writes the direct part of lambda(t) and
//                   the adjoints of u, F, Q, p_m (and rho, nu via omega_1)
//   k_adj_wall_move (moving walls) the wall-velocity term of the reflected
//                   populations transposed into rho_bar and p_m_bar
//   k_adj_phimu     transposed Q stencil -> adjoint of phi; back through
//                   phi = (p_m - rho/3) u, u = (j + F/2)/rho, F = (1/3-rho) G;
//                   then the transposed gradient stencil -> adjoint of mu
//                   (all nodes), in one z-march with G_bar kept in LDS
//   k_adj_wall_gather (walls) wall average of Eq. (36) transposed
//   k_adj_rho       mu0'(rho) and the (symmetric) Laplacian transposed
//   k_adj_wall_rho_solid, k_adj_wall_gather (walls) limiter/window of
//                   Eqs. (37)-(38) transposed
//   k_adj_pack      (rho_bar_total, j_bar) per node, for the next step's gather
//   k_adj_final     lambda_i(t) += rho_bar + c_i . j_bar, applied when lambda
//                   is read out; between adjoint steps this term is added by
//                   the next step's gather instead
//   k_adj_reduce*   deterministic parameter-gradient accumulation
// With a solid voxel mask the collision adjoint takes its bounce-back links
// from the neighbour words, solid nodes hold no lambda and no source
// adjoints, and the wall averages and window of every solid node are
// transposed per node (k_adj_wall_gather_m, k_adj_wall_rho_solid_m).  With
// moving walls k_adj_wall_move transposes the wall-velocity term of the
// reflected populations.
#include <type_traits>

#include "lbfe_device.h"
#include "lbfe_dpp.h"
#include "lbfe_zring.h"

namespace lbfe {
namespace {

template <int P> using real_t = typename Pol<P>::real;

constexpr unsigned kSelfBit = 1u << kRest;  // neighbour word: the node itself is solid
// a fluid node: inside the fluid planes, and not solid in a voxel mask
__device__ inline bool fluid_node(const KP &kp, const Bufs &b, size_t n) {
    if (kp.masked) return !(b.nbr[n] & kSelfBit);
    const int z = (int)(n / kp.plane);
    return z >= kp.z0 && z < kp.z1;
}

// Adjoint auxiliary arrays inside Bufs::abuf, in slots of N doubles.  The
// slots marked (real) hold planes in the compute precision (three float
// planes use half of their three slots): those values are formed in that
// precision, so keeping them narrower loses nothing.
enum : int {
    A_UB = 0,    // 3 (real): u_bar
    A_FB = 3,    // 3 (real): F_bar
    A_QB = 6,    // 3 (real): Q_bar (after folding the fourth-order terms)
    A_PMB = 9,   // p_m bar
    A_RHOB = 10, // rho bar (local part)
    A_JB = 11,   // 3 (real): j bar, rounded to the compute precision
    A_MUB = 14,  // mu bar (all nodes; the wall and mask transposes)
    A_KAPC = 15, // per-node dL/dkappa contribution
    A_NUC = 16,  // per-node dL/dnu contribution
    A_WETC = 17, // dL/d(wet) contribution per wall node, 2 planes packed
    A_RAVEB = 18,// rho_ave bar at solid nodes
    A_RHOBT = 19,// rho bar total (all nodes)
    A_MUBT = 20, // mu bar total (all nodes)
    A_PACK = 21, // 4 planes: (rho_bar_total, j_bar) per node as 4 compute-precision values
    A_COUNT = 25
};

// Adjoint (lambda) storage: same row-blocked layout as the populations, in
// the compute precision.
template <class real> struct Lam {
    real *p;
    unsigned nx;
    __device__ Lam(void *q, const KP &kp) : p((real *)q), nx((unsigned)kp.nx) {}
    __device__ size_t off(int i, unsigned row, unsigned x) const { return ((size_t)row * 27 + i) * nx + x; }
    __device__ real ld(int i, unsigned row, unsigned x) const { return p[off(i, row, x)]; }
    __device__ void st(int i, unsigned row, unsigned x, real v) const { p[off(i, row, x)] = v; }
};

// Plane c of a (real) slot group.
template <class real> __device__ inline real *aplane(void *abuf, int slot, int c, size_t N) {
    return (real *)((double *)abuf + (size_t)slot * N) + (size_t)c * N;
}

// ---- transposed 1-D transforms -------------------------------------------
// Transpose of the inverse map (k0,k1,k2) -> (f-,f0,f+) (see inv3).
template <class real> __device__ inline void inv3_T(real &lm, real &l0, real &lp, real u) {
    const real s = lp + lm, d = lp - lm;
    const real k0 = l0 + u * u * ((real)0.5 * s - l0) + (real)0.5 * u * d;
    const real k1 = u * (s - (real)2 * l0) + (real)0.5 * d;
    const real k2 = (real)0.5 * s - l0;
    lm = k0;
    l0 = k1;
    lp = k2;
}
// Transpose of the forward map (f-,f0,f+) -> (k0,k1,k2): g_c = m0 + (c-u) m1 + (c-u)^2 m2.
template <class real> __device__ inline void fwd3_T(real &a, real &b, real &c, real u) {
    const real m0 = a, m1 = b, m2 = c;
    const real em = (real)-1 - u, e0 = -u, ep = (real)1 - u;
    a = m0 + em * m1 + em * em * m2;
    b = m0 + e0 * m1 + e0 * e0 * m2;
    c = m0 + ep * m1 + ep * ep * m2;
}
// lambda_hat = T(u)^{-T} lambda*  (slots: directions in, central moments out)
template <class real> __device__ inline void cm_inverse_T(real (&l)[27], real ux, real uy, real uz) {
#pragma unroll
    for (int p = 0; p < 9; ++p) inv3_T(l[3 * p], l[3 * p + 1], l[3 * p + 2], uz);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int g = 0; g < 3; ++g) inv3_T(l[9 * a + g], l[9 * a + 3 + g], l[9 * a + 6 + g], uy);
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int g = 0; g < 3; ++g) inv3_T(l[3 * b + g], l[9 + 3 * b + g], l[18 + 3 * b + g], ux);
}
// g = T(u)^T m  (slots: central moments in, directions out)
template <class real> __device__ inline void cm_forward_T(real (&m)[27], real ux, real uy, real uz) {
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int g = 0; g < 3; ++g) fwd3_T(m[3 * b + g], m[9 + 3 * b + g], m[18 + 3 * b + g], ux);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int g = 0; g < 3; ++g) fwd3_T(m[9 * a + g], m[9 * a + 3 + g], m[9 * a + 6 + g], uy);
#pragma unroll
    for (int p = 0; p < 9; ++p) fwd3_T(m[3 * p], m[3 * p + 1], m[3 * p + 2], uz);
}

// sum_{abg} lam_{abg} (S_x k)_{abg} with (S_x k)_{abg} = a k_{(a-1)bg}; S_y, S_z alike.
template <class real>
__device__ inline void shift_dot(const real (&lam)[27], const real (&k)[27], real &sx, real &sy, real &sz) {
    real ax = 0, ay = 0, az = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
#pragma unroll
            for (int g = 0; g < 3; ++g) {
                if (a > 0) ax += (real)a * lam[K(a, b, g)] * k[K(a - 1, b, g)];
                if (b > 0) ay += (real)b * lam[K(a, b, g)] * k[K(a, b - 1, g)];
                if (g > 0) az += (real)g * lam[K(a, b, g)] * k[K(a, b, g - 1)];
            }
    sx = ax;
    sy = ay;
    sz = az;
}

// Transpose of the collision's linear part D (Eqs. (21)-(26) at zero
// sources), in place on lambda_hat -> D^T lambda_hat, with the adjoints of
// the sources: F, the six Q terms, p_m and omega_1 (which also multiplies
// pre-collision moments k).
template <class real> struct SrcBar {
    real F[3], Q[6], pm, om1;
};

template <class real>
__device__ inline void collide_T(real (&l)[27], const real (&k)[27], const Rates<real> &R, real q200, real q020,
                                 real q002, SrcBar<real> &sb) {
    const real one = 1, half = 0.5, third = (real)(1.0 / 3.0), ninth = (real)(1.0 / 9.0);
    const real *w = R.w;
    for (int a = 0; a < 3; ++a) sb.F[a] = 0;
    for (int a = 0; a < 6; ++a) sb.Q[a] = 0;
    sb.pm = 0;
    sb.om1 = 0;
    // first order
    {
        const real r0 = one - w[0], c0 = one - half * w[0];
        sb.F[0] += c0 * l[K(1, 0, 0)];
        sb.F[1] += c0 * l[K(0, 1, 0)];
        sb.F[2] += c0 * l[K(0, 0, 1)];
        l[K(1, 0, 0)] *= r0;
        l[K(0, 1, 0)] *= r0;
        l[K(0, 0, 1)] *= r0;
    }
    // second order, off-diagonal
    sb.om1 -= l[K(1, 1, 0)] * k[K(1, 1, 0)] + l[K(0, 1, 1)] * k[K(0, 1, 1)] + l[K(1, 0, 1)] * k[K(1, 0, 1)];
    l[K(1, 1, 0)] *= (one - w[1]);
    l[K(0, 1, 1)] *= (one - w[1]);
    l[K(1, 0, 1)] *= (one - w[1]);
    // second order, diagonal: (A, B, S) combinations
    {
        const real l200 = l[K(2, 0, 0)], l020 = l[K(0, 2, 0)], l002 = l[K(0, 0, 2)];
        const real Ab = third * (l200 - (real)2 * l020 + l002);
        const real Bb = third * (l200 + l020 - (real)2 * l002);
        const real Sb = third * (l200 + l020 + l002);
        const real A = k[K(2, 0, 0)] - k[K(0, 2, 0)], B = k[K(2, 0, 0)] - k[K(0, 0, 2)];
        sb.om1 += Ab * (-A - half * (q200 - q020)) + Bb * (-B - half * (q200 - q002));
        const real c1 = one - half * w[1], c2 = one - half * w[2];
        sb.Q[0] += c1 * (Ab + Bb) + c2 * Sb;
        sb.Q[1] += -c1 * Ab + c2 * Sb;
        sb.Q[2] += -c1 * Bb + c2 * Sb;
        sb.pm += (real)3 * w[2] * Sb;
        const real Ap = (one - w[1]) * Ab, Bp = (one - w[1]) * Bb, Sp = (one - w[2]) * Sb;
        l[K(2, 0, 0)] = Ap + Bp + Sp;
        l[K(0, 2, 0)] = -Ap + Sp;
        l[K(0, 0, 2)] = -Bp + Sp;
    }
    // third order
    {
        const real r3 = one - w[3], r4 = one - w[4], c3 = (one - half * w[3]) * (real)(2.0 / 3.0);
        auto pair = [&](int ia, int ib, int comp) {
            const real Pb = half * (l[ia] + l[ib]), Mb = half * (l[ia] - l[ib]);
            sb.F[comp] += c3 * Pb;
            l[ia] = r3 * Pb + r4 * Mb;
            l[ib] = r3 * Pb - r4 * Mb;
        };
        pair(K(1, 2, 0), K(1, 0, 2), 0);
        pair(K(2, 1, 0), K(0, 1, 2), 1);
        pair(K(2, 0, 1), K(0, 2, 1), 2);
        l[K(1, 1, 1)] *= (one - w[5]);
    }
    // fourth order: (D1, D2, S4) combinations
    {
        const real l220 = l[K(2, 2, 0)], l202 = l[K(2, 0, 2)], l022 = l[K(0, 2, 2)];
        const real D1b = third * (l220 - l202), D2b = third * (l220 - l022), S4b = third * (l220 + l202 + l022);
        const real c6 = one - half * w[6], c7 = one - half * w[7];
        sb.Q[3] += c6 * (D1b + D2b) + c7 * S4b;
        sb.Q[4] += c6 * (-(real)2 * D1b + D2b) + c7 * S4b;
        sb.Q[5] += c6 * (D1b - (real)2 * D2b) + c7 * S4b;
        sb.pm += w[7] * S4b;
        const real D1p = (one - w[6]) * D1b, D2p = (one - w[6]) * D2b, S4p = (one - w[7]) * S4b;
        l[K(2, 2, 0)] = D1p + D2p + S4p;
        l[K(2, 0, 2)] = -(real)2 * D1p + D2p + S4p;
        l[K(0, 2, 2)] = D1p - (real)2 * D2p + S4p;
        l[K(2, 1, 1)] *= (one - w[8]);
        l[K(1, 2, 1)] *= (one - w[8]);
        l[K(1, 1, 2)] *= (one - w[8]);
    }
    // fifth order
    {
        const real c9 = (one - half * w[9]) * ninth, r9 = one - w[9];
        sb.F[0] += c9 * l[K(1, 2, 2)];
        sb.F[1] += c9 * l[K(2, 1, 2)];
        sb.F[2] += c9 * l[K(2, 2, 1)];
        l[K(1, 2, 2)] *= r9;
        l[K(2, 1, 2)] *= r9;
        l[K(2, 2, 1)] *= r9;
    }
    // sixth order
    sb.pm += w[10] * ninth * l[K(2, 2, 2)];
    l[K(2, 2, 2)] *= (one - w[10]);
}

// The last term of lambda(t): lambda_i(x) = direct part + rho_bar_total(x)
// + c_i . j_bar(x) at fluid nodes.  It is either applied in place
// (k_adj_final) or, while the next adjoint step follows, added to each value
// as that step gathers it (k_adj_collide with PEND): the same expression in
// the same order, so both give lambda bit for bit.
template <class real> __device__ inline real final_term(real rb, real jx, real jy, real jz, int i) {
    real add = rb;
    if (cxi(i)) add += (real)cxi(i) * jx;
    if (cyi(i)) add += (real)cyi(i) * jy;
    if (czi(i)) add += (real)czi(i) * jz;
    return add;
}
// the same four values packed per node (k_adj_pack), one vector load
template <class real> using Pack4 = std::conditional_t<std::is_same_v<real, double>, double4, float4>;
template <class real> __device__ inline real final_term(const Pack4<real> *pk, int i, size_t m) {
    const Pack4<real> t = pk[m];
    return final_term<real>(t.x, t.y, t.z, t.w, i);
}

template <class real> __device__ inline void store_pack(void *abuf, size_t N, size_t n, double rhobt) {
    Pack4<real> t;
    t.x = (real)rhobt;
    t.y = aplane<real>(abuf, A_JB, 0, N)[n];
    t.z = aplane<real>(abuf, A_JB, 1, N)[n];
    t.w = aplane<real>(abuf, A_JB, 2, N)[n];
    ((Pack4<real> *)((double *)abuf + A_PACK * N))[n] = t;
}

template <int P> __global__ __launch_bounds__(kBlock) void k_adj_pack(KP kp, Bufs b) {
    using real = real_t<P>;
    const unsigned idx = tile_id(kp) * kBlock + threadIdx.x;
    if (idx >= kp.nfluid) return;
    const size_t n = (size_t)kp.z0 * kp.plane + idx, N = kp.N;
    store_pack<real>(b.abuf, N, n, ((const double *)b.abuf)[A_RHOBT * N + n]);
}

// ---------------------------------------------------------------------------
// PEND: lam_in holds only the direct part of lambda(t+1); its last term is
// added during the gather from the (rho_bar_total, j_bar) pack that the
// previous adjoint step left (this kernel does not write it).
template <int P, bool PEND, bool MASK>
__global__ __launch_bounds__(kBlock) void k_adj_collide(KP kp, Bufs b, const void *ft, const void *lam_in,
                                                        void *lam_out) {
    using real = real_t<P>;
    const unsigned idx = tile_id(kp) * kBlock + threadIdx.x;
    if (idx >= kp.nfluid) return;
    const unsigned n = (unsigned)kp.z0 * kp.plane + idx;
    int x, y, z;
    decompose(kp, n, x, y, z);
    const Nb nb(kp, x, y, z);
    const unsigned row = nb.row(0, 0);
    const Pops<P> fin(ft, kp);
    const Lam<real> lin(const_cast<void *>(lam_in), kp), lout(lam_out, kp);
    // solid mask: bit i of the neighbour word marks a link that ends on a
    // solid node (bounce-back); a solid node holds no lambda
    const unsigned wm = MASK ? b.nbr[n] : 0u;
    if (MASK && (wm & kSelfBit)) {
#pragma unroll
        for (int i = 0; i < 27; ++i) lout.st(i, row, (unsigned)x, (real)0);
        return;
    }

    // forward recomputation at x: the moments, kinematics and collision of
    // k_collide (the same device functions, so the same roundings)
    real k[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) k[i] = fin.ld(i, row, (unsigned)x);
    double rd;
    real jx, jy, jz;
    moments(k, rd, jx, jy, jz);
    const real *F = (const real *)b.F;
    const real Fx = F[n], Fy = F[kp.N + n], Fz = F[2 * (size_t)kp.N + n];
    const Kin<real> kin = kinematics(kp, rd, jx, jy, jz, Fx, Fy, Fz, b.mu[n]);
    const real ux = kin.ux, uy = kin.uy, uz = kin.uz, pm = kin.pm;
    const real *Qa = (const real *)b.Q;
    const real q200 = Qa[n], q020 = Qa[kp.N + n], q002 = Qa[2 * (size_t)kp.N + n];
    real q220 = 0, q202 = 0, q022 = 0;
    const real third = (real)(1.0 / 3.0);
    if (kp.corr4) {
        q220 = (q200 + q020) * third;
        q202 = (q200 + q002) * third;
        q022 = (q020 + q002) * third;
    }
    Rates<real> R;
#pragma unroll
    for (int q = 0; q < 11; ++q) R.w[q] = (real)kp.om[q];
    const real om1 = kin.om1;
    R.w[1] = om1;
    cm_forward(k, ux, uy, uz);  // k: pre-collision central moments
    real ks[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) ks[i] = k[i];
    collide(ks, R, Fx, Fy, Fz, pm, q200, q020, q002, q220, q202, q022);

    // reverse streaming: lambda*_i(x) = lambda_i(t+1)(x + c_i), or the
    // bounce-back partner at x when x + c_i is solid
    const bool wall_lo = kp.walls && z == 1;
    const bool wall_hi = kp.walls && z == kp.nz - 2;
    real l[27];
    const Pack4<real> *pk = (const Pack4<real> *)((const double *)b.abuf + A_PACK * (size_t)kp.N);
    auto bounce = [&](int i) {
        const int cz = czi(i);
        if constexpr (MASK) return ((wm >> i) & 1u) != 0;
        return (cz < 0 && wall_lo) || (cz > 0 && wall_hi);
    };
    if constexpr (PEND && (sizeof(real) == 8 || MASK)) {
        // FP64: the pending (rho_bar_total, j_bar) of each link's neighbour
        // with one vector load per link, beside the link's lambda (the
        // lane-shift form below needs more registers than an FP64 wave has
        // at two waves per SIMD)
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const int cz = czi(i);
            if (bounce(i))
                l[i] = lin.ld(26 - i, row, (unsigned)x) + final_term<real>(pk, 26 - i, n);
            else
                l[i] = lin.ld(i, nb.row(cyi(i), cz), nb.xo(cxi(i))) +
                       final_term<real>(pk, i, nb.at(cxi(i), cyi(i), cz));
        }
    } else {
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const int cz = czi(i);
            if (bounce(i))
                l[i] = lin.ld(26 - i, row, (unsigned)x);
            else
                l[i] = lin.ld(i, nb.row(cyi(i), cz), nb.xo(cxi(i)));
        }
    }
    if constexpr (PEND && sizeof(real) == 4 && !MASK) {
        // The pending (rho_bar_total, j_bar) of the 27 neighbours, one row
        // (cy, cz) at a time: the x - 1 and x + 1 values are those of the
        // adjacent lanes (a wave holds consecutive nodes), loaded only by
        // the lanes at a wave's or a row's ends.  The last active lane of
        // a partial wave has x = nx - 1 (fluid rows are whole).
        const unsigned lane = threadIdx.x & 63u;
        const bool own_m = lane == 0u || x == 0, own_p = lane == 63u || x == kp.nx - 1;
        const Pack4<real> c0 = pk[n];
#pragma unroll
        for (int r = 0; r < 9; ++r) {
            const int cy = r / 3 - 1, cz = r % 3 - 1;
            const Pack4<real> c = pk[nb.at(0, cy, cz)];
            Pack4<real> m, p;
            m.x = shr1(c.x), m.y = shr1(c.y), m.z = shr1(c.z), m.w = shr1(c.w);
            p.x = shl1(c.x), p.y = shl1(c.y), p.z = shl1(c.z), p.w = shl1(c.w);
            if (own_m) m = pk[nb.at(-1, cy, cz)];
            if (own_p) p = pk[nb.at(1, cy, cz)];
            const bool bb = (cz < 0 && wall_lo) || (cz > 0 && wall_hi);
#pragma unroll
            for (int cx = -1; cx <= 1; ++cx) {
                const int i = 9 * (cx + 1) + 3 * (cy + 1) + (cz + 1);
                const Pack4<real> t = cx < 0 ? m : (cx > 0 ? p : c);
                l[i] += bb ? final_term<real>(c0.x, c0.y, c0.z, c0.w, 26 - i)
                           : final_term<real>(t.x, t.y, t.z, t.w, i);
            }
        }
    }
    // (moving walls: the wall term's adjoint is added by k_adj_wall_move)
    cm_inverse_T(l, ux, uy, uz);  // l = lambda_hat (adjoint of k*)
    real ubx, uby, ubz;
    shift_dot(l, ks, ubx, uby, ubz);  // lambda_hat . S k*
    SrcBar<real> sb;
    collide_T(l, k, R, q200, q020, q002, sb);  // l = D^T lambda_hat
    real tx, ty, tz;
    shift_dot(l, k, tx, ty, tz);  // (D^T lambda_hat) . S k
    ubx -= tx;
    uby -= ty;
    ubz -= tz;
    cm_forward_T(l, ux, uy, uz);  // direct part of lambda(t)
#pragma unroll
    for (int i = 0; i < 27; ++i) lout.st(i, row, (unsigned)x, l[i]);

    // fold the fourth-order correction (Eq. (28)) into Q_bar
    real qb0 = sb.Q[0], qb1 = sb.Q[1], qb2 = sb.Q[2];
    if (kp.corr4) {
        qb0 += third * (sb.Q[3] + sb.Q[4]);
        qb1 += third * (sb.Q[3] + sb.Q[5]);
        qb2 += third * (sb.Q[4] + sb.Q[5]);
    }
    // omega_1 = 1 / (rho nu / p_m + 1/2)
    const double o = (double)om1, dpm = (double)pm, rr = rd;
    const double om1b = (double)sb.om1;
    const double rhob = -om1b * o * o * kp.nu / dpm;
    const double pmb = (double)sb.pm + om1b * o * o * rr * kp.nu / (dpm * dpm);
    const double nub = -om1b * o * o * rr / dpm;
    const size_t N = kp.N;
    double *A = (double *)b.abuf;
    aplane<real>(A, A_UB, 0, N)[n] = ubx;
    aplane<real>(A, A_UB, 1, N)[n] = uby;
    aplane<real>(A, A_UB, 2, N)[n] = ubz;
    aplane<real>(A, A_FB, 0, N)[n] = sb.F[0];
    aplane<real>(A, A_FB, 1, N)[n] = sb.F[1];
    aplane<real>(A, A_FB, 2, N)[n] = sb.F[2];
    aplane<real>(A, A_QB, 0, N)[n] = qb0;
    aplane<real>(A, A_QB, 1, N)[n] = qb1;
    aplane<real>(A, A_QB, 2, N)[n] = qb2;
    A[A_PMB * N + n] = pmb;
    A[A_RHOB * N + n] = rhob;
    A[A_NUC * N + n] = nub;
}

// Moving walls: a reflected population carries -[f^eq_i - f^eq_opp(i)](rho,
// p_m, u_w) (k_wall_move), which is linear in (rho, p_m) at a given u_w; its
// adjoint adds to rho_bar and p_m_bar of the wall-adjacent nodes, from the
// lambda* that k_adj_collide gathered on the reflected links (a kernel of its
// own, after k_adj_collide: the wall equilibria would raise the collision
// adjoint's register count past two waves per SIMD in FP64).
template <int P, bool PEND>
__global__ __launch_bounds__(kBlock) void k_adj_wall_move(KP kp, Bufs b, const void *lam_in) {
    using real = real_t<P>;
    const unsigned idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= 2 * kp.plane) return;
    const int side = idx >= kp.plane;
    if (side && kp.nz - 2 == 1) return;  // one fluid plane: both walls by side 0
    const unsigned p = idx - (side ? kp.plane : 0u);
    const int y = (int)(p / (unsigned)kp.nx), x = (int)(p - (unsigned)y * kp.nx);
    const int z = side ? kp.nz - 2 : 1;
    const size_t n = (size_t)z * kp.plane + p;
    const Nb nb(kp, x, y, z);
    const unsigned row = nb.row(0, 0);
    const Lam<real> lin(const_cast<void *>(lam_in), kp);
    const Pack4<real> *pk = (const Pack4<real> *)((const double *)b.abuf + A_PACK * (size_t)kp.N);
    const bool wall_lo = z == 1, wall_hi = z == kp.nz - 2;
    double wrb = 0.0, wpb = 0.0;
    for (int w = 0; w < 2; ++w) {
        if (!(w == 0 ? wall_lo : wall_hi)) continue;
        real ea[27], eb[27];
        const real uwx = (real)kp.wall_u[2 * w], uwy = (real)kp.wall_u[2 * w + 1];
        wall_equilibrium((real)1, (real)0, uwx, uwy, ea);
        wall_equilibrium((real)0, (real)1, uwx, uwy, eb);
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const int cz = czi(i);
            if ((w == 0 && cz < 0) || (w == 1 && cz > 0)) {
                // lambda*_i at a reflected link: the node's own value of the
                // opposite direction, plus its pending last term
                real li = lin.ld(26 - i, row, (unsigned)x);
                if constexpr (PEND) li = li + final_term<real>(pk, 26 - i, n);
                wrb -= (double)li * (double)(ea[i] - ea[26 - i]);
                wpb -= (double)li * (double)(eb[i] - eb[26 - i]);
            }
        }
    }
    double *A = (double *)b.abuf;
    A[A_RHOB * kp.N + n] += wrb;
    A[A_PMB * kp.N + n] += wpb;
}

// The transposed Q and gradient stencils in one z-march:
//   phi part, at fluid nodes: phi_bar_a = transpose of Q_a = -9 sum_i w_i
//     c_ia phi_a(x + c_i) = 9 sum_i w_i c_ia Q_bar_a(x + c_i), then back
//     through phi = (p_m - rho/3) u, u = (j + F/2)/rho, F = (1/3 - rho) G:
//     j_bar, rho_bar (local part), G_bar and the local part of mu_bar;
//   mu part, at every node: mu_bar(y) = local part (fluid) - 3 sum_i w_i
//     c_i . G_bar(y + c_i) (G_bar is zero at solid nodes), into A_MUBT.
// A workgroup owns a 32 x 16 tile of mu_bar planes [zs, ze).  Iteration k
// evaluates the phi part at plane k+1 on the tile and its one-node ring (Q_bar
// and mu staged with a two-node halo in a three-plane LDS ring), which leaves
// G_bar of those 34 x 18 nodes in a three-plane LDS ring, then sums mu_bar of
// plane k on the tile.  G_bar never goes to HBM; the owned node's j_bar and
// rho_bar do, the ring nodes only give G_bar.
constexpr int PWX = ZTX + 4, PNR = PWX * (ZTY + 4);  // Q_bar and mu region: tile + 2-node halo
constexpr int GWX = ZTX + 2, GNR = GWX * (ZTY + 2);  // G_bar region: tile + 1-node ring
constexpr int PCB = ZCB + 128;                       // threads: the tile's nodes, then the ring's
constexpr int PPT = (PNR + PCB - 1) / PCB;           // Q_bar / mu region points per thread
static_assert(GNR <= PCB, "one G_bar node per thread");

__device__ inline int zslot3(int p) { return ((p % 3) + 3) % 3; }

template <int P, bool MASK> __global__ __launch_bounds__(PCB) void k_adj_phimu(KP kp, Bufs b, int cz) {
    using real = real_t<P>;
    __shared__ double sq[3][4][PNR];  // Q_bar x, y, z and mu of planes p (slot p mod 3)
    __shared__ double sg[3][3][GNR];  // G_bar of planes p (slot p mod 3)
    int x0, y0, zs, ze;
    ztile(kp, cz, 0, kp.nz, x0, y0, zs, ze);
    const size_t N = kp.N;
    const unsigned plane = kp.plane;
    double *A = (double *)b.abuf;
    const real *j = (const real *)b.j, *F = (const real *)b.F;
    const real *qb[3] = {aplane<real>(A, A_QB, 0, N), aplane<real>(A, A_QB, 1, N), aplane<real>(A, A_QB, 2, N)};
    const int tid = threadIdx.x;
    const int ta = tid % ZTX, tb = tid / ZTX;  // the tile node of threads below ZCB
    const bool own = tid < ZCB && x0 + ta < kp.nx && y0 + tb < kp.ny;

    // Q_bar / mu region points of this thread, in-plane node index
    unsigned qoff[PPT];
    bool qhas[PPT];
#pragma unroll
    for (int m = 0; m < PPT; ++m) {
        const int r = tid + m * PCB;
        qhas[m] = r < PNR;
        const int rr = qhas[m] ? r : 0;
        qoff[m] = (unsigned)zwrap(y0 + rr / PWX - 2, kp.ny) * kp.nx + zwrap(x0 + rr % PWX - 2, kp.nx);
    }
    double qpre[4][PPT];
    auto load = [&](int p) {
        const size_t base = (size_t)zwrap(p, kp.nz) * plane;
#pragma unroll
        for (int m = 0; m < PPT; ++m)
            if (qhas[m]) {
#pragma unroll
                for (int c = 0; c < 3; ++c) qpre[c][m] = (double)qb[c][base + qoff[m]];
                qpre[3][m] = b.mu[base + qoff[m]];
            }
    };
    auto commit = [&](int p) {
        const int sl = zslot3(p);
#pragma unroll
        for (int m = 0; m < PPT; ++m)
            if (qhas[m]) {
#pragma unroll
                for (int f = 0; f < 4; ++f) sq[sl][f][tid + m * PCB] = qpre[f][m];
            }
    };

    // the phi part at plane p for G-region node (ga, gb): G_bar into LDS;
    // for an owned node of a plane of this chunk also j_bar and rho_bar to
    // HBM (the fill planes at both ends belong to the neighbouring chunks),
    // and the local part of mu_bar returned
    auto phi_node = [&](int p, int ga, int gb, bool owned) -> double {
        const int zz = zwrap(p, kp.nz);
        const int sm = zslot3(p - 1), s0 = zslot3(p), sp = zslot3(p + 1);
        const int g = gb * GWX + ga;
        const int cq = (gb + 1) * PWX + ga + 1;  // the node in the Q_bar / mu region
        auto at = [&](int f, int dz, int dx, int dy) {
            return sq[dz < 0 ? sm : (dz > 0 ? sp : s0)][f][cq + dy * PWX + dx];
        };
        const size_t n = (size_t)zz * plane + (unsigned)zwrap(y0 + gb - 1, kp.ny) * kp.nx +
                         (unsigned)zwrap(x0 + ga - 1, kp.nx);
        bool fl = zz >= kp.z0 && zz < kp.z1;
        if constexpr (MASK) fl = fl && !(b.nbr[n] & kSelfBit);
        if (!fl) {  // solid: no G_bar, no local mu_bar, nothing stored
            sg[s0][0][g] = sg[s0][1][g] = sg[s0][2][g] = 0.0;
            return 0.0;
        }
        double px = 0, py = 0, pz = 0;
#pragma unroll
        for (int a = -1; a <= 1; ++a)
#pragma unroll
            for (int c = -1; c <= 1; ++c) {
                const double w = w1(a) * w1(c) / 6.0;
                px += w * (at(0, c, 1, a) - at(0, c, -1, a));
                py += w * (at(1, c, a, 1) - at(1, c, a, -1));
                pz += w * (at(2, 1, a, c) - at(2, -1, a, c));
            }
        px *= 9.0;
        py *= 9.0;
        pz *= 9.0;
        const double r = b.rho[n], mu = at(3, 0, 0, 0);
        const real ir = (real)1 / (real)r;
        const double ux = (double)((j[n] + (real)0.5 * F[n]) * ir);
        const double uy = (double)((j[N + n] + (real)0.5 * F[N + n]) * ir);
        const double uz = (double)((j[2 * N + n] + (real)0.5 * F[2 * N + n]) * ir);
        const double c2 = (double)(real)((1.0 + mu - r) * (1.0 / 3.0));
        const double pu = px * ux + py * uy + pz * uz;
        const double utx = (double)aplane<real>(A, A_UB, 0, N)[n] + c2 * px;
        const double uty = (double)aplane<real>(A, A_UB, 1, N)[n] + c2 * py;
        const double utz = (double)aplane<real>(A, A_UB, 2, N)[n] + c2 * pz;
        // u = (j + F/2)/rho: j_bar = u_tilde/rho, F_bar += j_bar/2 (halving
        // the quotient rounds as dividing the halved numerator does)
        const double jbx = utx / r, jby = uty / r, jbz = utz / r;
        const double Fbx = (double)aplane<real>(A, A_FB, 0, N)[n] + 0.5 * jbx;
        const double Fby = (double)aplane<real>(A, A_FB, 1, N)[n] + 0.5 * jby;
        const double Fbz = (double)aplane<real>(A, A_FB, 2, N)[n] + 0.5 * jbz;
        const double c1 = 1.0 / 3.0 - r;
        sg[s0][0][g] = c1 * Fbx;
        sg[s0][1][g] = c1 * Fby;
        sg[s0][2][g] = c1 * Fbz;
        if (!owned) return 0.0;
        double pmb = A[A_PMB * N + n], rhob = A[A_RHOB * N + n];
        pmb += pu;
        rhob -= pu / 3.0;
        aplane<real>(A, A_JB, 0, N)[n] = (real)jbx;
        aplane<real>(A, A_JB, 1, N)[n] = (real)jby;
        aplane<real>(A, A_JB, 2, N)[n] = (real)jbz;
        rhob -= (utx * ux + uty * uy + utz * uz) / r;
        double gx = 0.0, gy = 0.0, gz = 0.0;
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            if (i == kRest) continue;
            const double m = wi(i) * at(3, czi(i), cxi(i), cyi(i));
            if (cxi(i)) gx += cxi(i) * m;
            if (cyi(i)) gy += cyi(i) * m;
            if (czi(i)) gz += czi(i) * m;
        }
        gx *= 3.0;
        gy *= 3.0;
        gz *= 3.0;
        rhob -= Fbx * gx + Fby * gy + Fbz * gz;
        A[A_RHOB * N + n] = rhob;
        return pmb / 3.0;  // p_m = (1 + mu)/3
    };
    // ring-only G-region node q of thread ZCB + q
    auto ring_node = [&](int q, int &ga, int &gb) {
        if (q < GWX) {
            ga = q, gb = 0;
        } else if (q < 2 * GWX) {
            ga = q - GWX, gb = ZTY + 1;
        } else if (q < 2 * GWX + ZTY) {
            ga = 0, gb = q - 2 * GWX + 1;
        } else {
            ga = GWX - 1, gb = q - 2 * GWX - ZTY + 1;
        }
    };

    double mloc_k = 0.0;  // local mu_bar of the owned node, plane k
    load(zs - 2);
    commit(zs - 2);
    load(zs - 1);
    commit(zs - 1);
    load(zs);
    for (int k = zs - 2; k < ze; ++k) {
        commit(k + 2);
        __syncthreads();
        if (k + 3 <= ze + 1) load(k + 3);
        // phi part at plane k+1: the tile's nodes and the ring's, one per thread
        double mloc_next = 0.0;
        if (tid < ZCB) {
            mloc_next = phi_node(k + 1, ta + 1, tb + 1, own && k + 1 >= zs && k + 1 < ze);
        } else if (tid < GNR) {
            int ga, gb;
            ring_node(tid - ZCB, ga, gb);
            phi_node(k + 1, ga, gb, false);
        }
        __syncthreads();
        if (k >= zs && own) {
            const int sm = zslot3(k - 1), s0 = zslot3(k), sp = zslot3(k + 1);
            const int g = (tb + 1) * GWX + ta + 1;
            double sum = 0.0;
#pragma unroll
            for (int i = 0; i < 27; ++i) {
                if (i == kRest) continue;
                const int sl = czi(i) < 0 ? sm : (czi(i) > 0 ? sp : s0);
                const int gi = g + cyi(i) * GWX + cxi(i);
                double d = 0.0;
                if (cxi(i)) d += cxi(i) * sg[sl][0][gi];
                if (cyi(i)) d += cyi(i) * sg[sl][1][gi];
                if (czi(i)) d += czi(i) * sg[sl][2][gi];
                sum += wi(i) * d;
            }
            const size_t n = (size_t)k * plane + (unsigned)(y0 + tb) * kp.nx + (x0 + ta);
            const bool fluid = k >= kp.z0 && k < kp.z1;
            A[A_MUBT * N + n] = (fluid ? mloc_k : 0.0) - 3.0 * sum;
        }
        mloc_k = mloc_next;
    }
}

// Normalising weight sum of the wall average at solid node (x, y, zs).
__device__ inline double wall_den(const KP &kp, int zs) {
    double den = 0.0;
    for (int cz = -1; cz <= 1; ++cz) {
        const int zz = zs + cz;
        if (zz < 1 || zz > kp.nz - 2) continue;
        for (int cy = -1; cy <= 1; ++cy)
            for (int cx = -1; cx <= 1; ++cx) den += wq(cx, cy, cz);
    }
    return den;
}

// Transpose of a wall average (Eqs. (36)/(37)) for the fluid first layers:
// dst(y) += sum over solid neighbours s of w(y - s) / den(s) * src(s).
__global__ __launch_bounds__(kBlock) void k_adj_wall_gather(KP kp, const double *src, double *dst) {
    const unsigned idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= 2 * kp.plane) return;
    const int side = idx >= kp.plane;
    if (side && kp.nz - 2 == 1) return;  // one fluid layer: both walls handled by side 0
    const unsigned p = idx - (side ? kp.plane : 0u);
    const int y = (int)(p / (unsigned)kp.nx), x = (int)(p - (unsigned)y * kp.nx);
    const int zf = side ? kp.nz - 2 : 1;  // fluid layer next to a wall
    const Nb nb(kp, x, y, zf);
    double acc = 0.0;
    for (int cz = -1; cz <= 1; ++cz) {
        const int zs = zf + cz;
        if (zs != 0 && zs != kp.nz - 1) continue;  // only solid neighbours
        const double inv = 1.0 / wall_den(kp, zs);
        for (int cy = -1; cy <= 1; ++cy)
            for (int cx = -1; cx <= 1; ++cx) acc += wq(cx, cy, cz) * inv * src[nb.at(cx, cy, cz)];
    }
    dst[(size_t)zf * kp.plane + p] += acc;
}

// rho_bar_total(y) = [fluid: rho_bar + mu_bar mu0'(rho)] - kappa L[mu_bar_fluid](y);
// per-node dL/dkappa = -mu_bar L[rho].  `mub` is the total mu_bar (solid
// entries are ignored: the Laplacian's adjoint sees fluid mu_bar only).
template <bool MASK>
__global__ __launch_bounds__(ZCB) void k_adj_rho(KP kp, const double *mub, const double *rhob_local,
                                                 const double *rho, double *rhobt, double *kapc, int cz,
                                                 const unsigned *nbr) {
    __shared__ double lds[4][2][ZNR];
    int x0, y0, zs, ze;
    ztile(kp, cz, 0, kp.nz, x0, y0, zs, ze);
    ZRing<2> R;
    R.init(kp, lds, x0, y0);
    R.src[0] = mub;
    R.src[1] = rho;
    R.zmask = 1u;  // mu_bar of solid planes reads as zero
    R.march(zs, ze, [&](int k) {
        if (!R.own) return;
        const double m0 = R.at(0, k, 0, 0);
        const double r0 = R.at(1, k, 0, 0);
        double lm = 0.0, lr = 0.0;
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            if (i == kRest) continue;
            const int p = k + czi(i);
            lm += wi(i) * (R.at(0, p, cxi(i), cyi(i)) - m0);
            lr += wi(i) * (R.at(1, p, cxi(i), cyi(i)) - r0);
        }
        lm *= 6.0;
        lr *= 6.0;
        const size_t n = (size_t)k * kp.plane + R.node;
        bool fluid;
        if constexpr (MASK)
            fluid = !(nbr[n] & kSelfBit);
        else
            fluid = k >= kp.z0 && k < kp.z1;
        double out = -kp.kappa * lm;
        if (fluid) {
            const double d = 1.0 - kp.b * r0;
            const double dmu0 = kp.RT / (r0 * d * d) - 2.0 * kp.a;
            out += rhob_local[n] + m0 * dmu0;
            kapc[n] = -m0 * lr;
        } else {
            kapc[n] = 0.0;
        }
        rhobt[n] = out;
    });
}

// Solid nodes: rho_ave_bar = W'(rho_ave) rho_bar(x_s), and the per-node
// dL/d(wet_value) = dW/d(wet) rho_bar(x_s) (active branch of Eq. (38)).
__global__ __launch_bounds__(kBlock) void k_adj_wall_rho_solid(KP kp, const double *rho, const double *rhobt,
                                                               double *raveb, double *wetc) {
    const unsigned idx = blockIdx.x * kBlock + threadIdx.x;
    if (idx >= 2 * kp.plane) return;
    const int side = idx >= kp.plane;
    const unsigned p = idx - (side ? kp.plane : 0u);
    const int y = (int)(p / (unsigned)kp.nx), x = (int)(p - (unsigned)y * kp.nx);
    const int zs = side ? kp.nz - 1 : 0;
    const Nb nb(kp, x, y, zs);
    double num = 0.0, den = 0.0;
    for (int cz = -1; cz <= 1; ++cz) {
        const int zz = zs + cz;
        if (zz < 1 || zz > kp.nz - 2) continue;
        for (int cy = -1; cy <= 1; ++cy)
            for (int cx = -1; cx <= 1; ++cx) {
                num += wq(cx, cy, cz) * rho[nb.at(cx, cy, cz)];
                den += wq(cx, cy, cz);
            }
    }
    const double rave = num / den;
    const size_t n = (size_t)zs * kp.plane + p;
    const double g = rhobt[n];
    double dW = 1.0, dwet = 0.0;
    if (rave >= kp.lo && rave <= kp.hi) {
        if (kp.wet_mode == LBFE_WET_PHI) {
            const double v = kp.wet_value * rave;
            const bool inside = v >= kp.lo && v <= kp.hi;
            dW = inside ? kp.wet_value : 0.0;
            dwet = inside ? rave : 0.0;
        } else if (kp.wet_mode == LBFE_WET_DELTA) {
            const double v = rave - kp.wet_value;
            const bool inside = v >= kp.lo && v <= kp.hi;
            dW = inside ? 1.0 : 0.0;
            dwet = inside ? -1.0 : 0.0;
        }
    }
    raveb[n] = dW * g;
    wetc[idx] = dwet * g;
}

// ---- solid voxel masks ------------------------------------------------------
// The transposes of the mask path's wall averages (Eqs. (36)-(37) at every
// solid node with a fluid neighbour, weights w_i of its fluid neighbours in
// direction order) and of the window of Eq. (38), per node.

// dst = src at fluid nodes, 0 at solid nodes (mu_bar as the Laplacian's
// adjoint sees it)
__global__ __launch_bounds__(kBlock) void k_adj_fluid_copy_m(KP kp, const unsigned *nbr, const double *src,
                                                           double *dst) {
    const unsigned n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    dst[n] = (nbr[n] & kSelfBit) ? 0.0 : src[n];
}

// weight sum of the wall average at solid node n (0: no fluid neighbour)
__device__ inline double mask_den(unsigned w) {
    double den = 0.0;
#pragma unroll
    for (int i = 0; i < 27; ++i)
        if (!(w & (1u << i))) den += wi(i);
    return den;
}

// dst(y) += sum over the solid neighbours s = y + c_i of fluid y of
// w_i / den(s) src(s)
__global__ __launch_bounds__(kBlock) void k_adj_wall_gather_m(KP kp, const unsigned *nbr, const double *src,
                                                            double *dst) {
    const unsigned n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    const unsigned w = nbr[n];
    if ((w & kSelfBit) || w == 0u) return;
    int x, y, z;
    decompose(kp, n, x, y, z);
    const Nb nb(kp, x, y, z);
    double acc = 0.0;
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        if (!(w & (1u << i))) continue;
        const unsigned s = nb.at(cxi(i), cyi(i), czi(i));
        acc += wi(i) / mask_den(nbr[s]) * src[s];
    }
    dst[n] += acc;
}

// Solid nodes: rho_ave_bar = W'(rho_ave) rho_bar(x_s) and the per-node
// dL/d(wet_value) (active branch of Eq. (38)); 0 elsewhere.
__global__ __launch_bounds__(kBlock) void k_adj_wall_rho_solid_m(KP kp, const unsigned *nbr, const double *rho,
                                                               const double *rhobt, double *raveb, double *wetc) {
    const unsigned n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    const unsigned w = nbr[n];
    double rb = 0.0, wc = 0.0;
    if (w & kSelfBit) {
        int x, y, z;
        decompose(kp, n, x, y, z);
        const Nb nb(kp, x, y, z);
        double num = 0.0, den = 0.0;
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            if (w & (1u << i)) continue;
            const double wt = wi(i);
            num += wt * rho[nb.at(cxi(i), cyi(i), czi(i))];
            den += wt;
        }
        if (den > 0.0) {
            const double rave = num / den, g = rhobt[n];
            double dW = 1.0, dwet = 0.0;
            if (rave >= kp.lo && rave <= kp.hi) {
                if (kp.wet_mode == LBFE_WET_PHI) {
                    const double v = kp.wet_value * rave;
                    const bool inside = v >= kp.lo && v <= kp.hi;
                    dW = inside ? kp.wet_value : 0.0;
                    dwet = inside ? rave : 0.0;
                } else if (kp.wet_mode == LBFE_WET_DELTA) {
                    const double v = rave - kp.wet_value;
                    const bool inside = v >= kp.lo && v <= kp.hi;
                    dW = inside ? 1.0 : 0.0;
                    dwet = inside ? -1.0 : 0.0;
                }
            }
            rb = dW * g;
            wc = dwet * g;
        }
    }
    raveb[n] = rb;
    wetc[n] = wc;
}

// lambda_i(t) = direct part + rho_bar_total + c_i . j_bar at fluid nodes.
template <int P> __global__ __launch_bounds__(kBlock) void k_adj_final(KP kp, Bufs b, void *lam) {
    using real = real_t<P>;
    const unsigned idx = tile_id(kp) * kBlock + threadIdx.x;
    if (idx >= kp.nfluid) return;
    const unsigned n = (unsigned)kp.z0 * kp.plane + idx;
    if (kp.masked && (b.nbr[n] & kSelfBit)) return;
    const unsigned row = n / (unsigned)kp.nx, x = n - row * (unsigned)kp.nx;
    const Pack4<real> *pk = (const Pack4<real> *)((const double *)b.abuf + A_PACK * (size_t)kp.N);
    const Lam<real> L(lam, kp);
#pragma unroll
    for (int i = 0; i < 27; ++i) L.st(i, row, x, L.ld(i, row, x) + final_term<real>(pk, i, n));
}

// Deterministic accumulation: per-block sums of three arrays (a0, a2 of n
// entries, a1 of n1), then one block adds them (fixed order) to acc[0..2].
__global__ __launch_bounds__(kBlock) void k_adj_reduce_part(unsigned n, const double *a0, unsigned n1,
                                                            const double *a1, const double *a2, double *part) {
    __shared__ double s[3][kBlock];
    // a fixed grid-stride assignment: the same sums in the same order on
    // every call
    double v0 = 0.0, v1 = 0.0, v2 = 0.0;
    for (unsigned i = blockIdx.x * kBlock + threadIdx.x; i < n; i += gridDim.x * kBlock) {
        if (a0) v0 += a0[i];
        if (a2) v2 += a2[i];
    }
    if (a1)
        for (unsigned i = blockIdx.x * kBlock + threadIdx.x; i < n1; i += gridDim.x * kBlock) v1 += a1[i];
    s[0][threadIdx.x] = v0;
    s[1][threadIdx.x] = v1;
    s[2][threadIdx.x] = v2;
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 3; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x < 3) part[(size_t)blockIdx.x * 3 + threadIdx.x] = s[threadIdx.x][0];
}

__global__ __launch_bounds__(kBlock) void k_adj_reduce_final(unsigned nblk, const double *part, double *acc) {
    __shared__ double s[3][kBlock];
    double v[3] = {0, 0, 0};
    for (unsigned q = threadIdx.x; q < nblk; q += kBlock)
        for (int k = 0; k < 3; ++k) v[k] += part[(size_t)q * 3 + k];
    for (int k = 0; k < 3; ++k) s[k][threadIdx.x] = v[k];
    __syncthreads();
    for (int h = kBlock / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h)
            for (int k = 0; k < 3; ++k) s[k][threadIdx.x] += s[k][threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        acc[0] += s[0][0];  // kappa
        acc[1] += s[1][0];  // wet value
        acc[2] += s[2][0];  // nu
    }
}

// ---- seed and initialiser ---------------------------------------------------
template <int P> __global__ __launch_bounds__(kBlock) void k_adj_seed(KP kp, Bufs b, const double *g, void *lam) {
    using real = real_t<P>;
    const unsigned n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    const unsigned row = n / (unsigned)kp.nx, x = n - row * (unsigned)kp.nx;
    const bool fluid = fluid_node(kp, b, n);
    const real v = fluid ? (real)g[n] : (real)0;
    const Lam<real> L(lam, kp);
#pragma unroll
    for (int i = 0; i < 27; ++i) L.st(i, row, x, v);
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_adj_seed_pop(KP kp, Bufs b, const double *g, void *lam) {
    using real = real_t<P>;
    const unsigned n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    const unsigned row = n / (unsigned)kp.nx, x = n - row * (unsigned)kp.nx;
    const bool fluid = fluid_node(kp, b, n);
    const Lam<real> L(lam, kp);
#pragma unroll
    for (int i = 0; i < 27; ++i) L.st(i, row, x, fluid ? (real)g[(size_t)i * kp.N + n] : (real)0);
}

template <int P>
__global__ __launch_bounds__(kBlock) void k_adj_get(KP kp, Bufs b, const void *lam, double *out) {
    using real = real_t<P>;
    const unsigned n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    const unsigned row = n / (unsigned)kp.nx, x = n - row * (unsigned)kp.nx;
    const bool fluid = fluid_node(kp, b, n);
    const Lam<real> L(const_cast<void *>(lam), kp);
#pragma unroll
    for (int i = 0; i < 27; ++i) out[(size_t)i * kp.N + n] = fluid ? (double)L.ld(i, row, x) : 0.0;
}

// Initialiser f = T(u0)^{-1} k_eq(rho0, p_m): k_eq_bar = T(u0)^{-T} lambda(0);
// rho_bar_local = k_eq_bar_000, mu_bar = p_m_bar / 3 (fluid), 0 at solid.
template <int P>
__global__ __launch_bounds__(kBlock) void k_adj_init_local(KP kp, Bufs b, const void *lam, const double *u0) {
    using real = real_t<P>;
    const unsigned n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    const bool fluid = fluid_node(kp, b, n);
    const size_t N = kp.N;
    double *A = (double *)b.abuf;
    if (!fluid) {
        A[A_RHOB * N + n] = 0.0;
        A[A_MUB * N + n] = 0.0;
        return;
    }
    const unsigned row = n / (unsigned)kp.nx, x = n - row * (unsigned)kp.nx;
    const Lam<real> L(const_cast<void *>(lam), kp);
    real l[27];
#pragma unroll
    for (int i = 0; i < 27; ++i) l[i] = L.ld(i, row, x);
    real ux = 0, uy = 0, uz = 0;
    if (u0) {
        ux = (real)u0[n];
        uy = (real)u0[N + n];
        uz = (real)u0[2 * N + n];
    }
    cm_inverse_T(l, ux, uy, uz);
    const double third = 1.0 / 3.0, ninth = 1.0 / 9.0;
    const double pmb = (double)l[K(2, 0, 0)] + (double)l[K(0, 2, 0)] + (double)l[K(0, 0, 2)] +
                       third * ((double)l[K(2, 2, 0)] + (double)l[K(2, 0, 2)] + (double)l[K(0, 2, 2)]) +
                       ninth * (double)l[K(2, 2, 2)];
    A[A_RHOB * N + n] = (double)l[K(0, 0, 0)];
    A[A_MUB * N + n] = pmb / 3.0;
}

__global__ __launch_bounds__(kBlock) void k_adj_init_out(KP kp, Bufs b, const double *rhobt, double *out) {
    const unsigned n = blockIdx.x * kBlock + threadIdx.x;
    if (n >= kp.N) return;
    out[n] = fluid_node(kp, b, n) ? rhobt[n] : 0.0;
}

template <class Fn> hipError_t dispatch(int prec, Fn &&fn) {
    switch (prec) {
        case LBFE_FP64: return fn(std::integral_constant<int, LBFE_FP64>{});
        case LBFE_FP32: return fn(std::integral_constant<int, LBFE_FP32>{});
        case LBFE_FP16_DEV: return fn(std::integral_constant<int, LBFE_FP16_DEV>{});
        default: return fn(std::integral_constant<int, LBFE_FP16_DEV_F0FP32>{});
    }
}

constexpr unsigned kReduceBlocks = 1024;  // blocks of the gradient reduction

// The chain from mu_bar (A_MUBT after k_adj_phimu; in the initialiser's
// adjoint its local part in A_MUB) to rho_bar_total (A_RHOBT) with walls,
// and the kappa / wet accumulation.
hipError_t chain_tail(hipStream_t s, const KP &kp, const Bufs &b, bool with_gradient_transpose,
                      const double *nuc) {
    const size_t N = kp.N;
    double *A = (double *)b.abuf;
    const unsigned gN = nblocks(N), gw = nblocks(2 * (size_t)kp.plane);
    double *mub_tot = A + (with_gradient_transpose ? A_MUBT : A_MUB) * N;
    const dim3 gall = zgrid(kp, 0, kp.nz);
    const double *wetc = nullptr;
    unsigned nwet = 0;
    if (kp.masked) {
        // mu_bar of the solid nodes back to their fluid neighbours (Eq. (36)),
        // then the Laplacian's adjoint with mu_bar zero at solid nodes
        k_adj_wall_gather_m<<<gN, kBlock, 0, s>>>(kp, b.nbr, mub_tot, mub_tot);
        k_adj_fluid_copy_m<<<gN, kBlock, 0, s>>>(kp, b.nbr, mub_tot, A + A_MUB * N);
        k_adj_rho<true><<<gall, ZCB, 0, s>>>(kp, A + A_MUB * N, A + A_RHOB * N, b.rho, A + A_RHOBT * N,
                                             A + A_KAPC * N, kZChunk, b.nbr);
        k_adj_wall_rho_solid_m<<<gN, kBlock, 0, s>>>(kp, b.nbr, b.rho, A + A_RHOBT * N, A + A_RAVEB * N,
                                                     A + A_WETC * N);
        k_adj_wall_gather_m<<<gN, kBlock, 0, s>>>(kp, b.nbr, A + A_RAVEB * N, A + A_RHOBT * N);
        wetc = A + A_WETC * N;
        nwet = (unsigned)N;
    } else {
        if (kp.walls) k_adj_wall_gather<<<gw, kBlock, 0, s>>>(kp, mub_tot, mub_tot);
        k_adj_rho<false><<<gall, ZCB, 0, s>>>(kp, mub_tot, A + A_RHOB * N, b.rho, A + A_RHOBT * N, A + A_KAPC * N,
                                              kZChunk, nullptr);
        if (kp.walls) {
            k_adj_wall_rho_solid<<<gw, kBlock, 0, s>>>(kp, b.rho, A + A_RHOBT * N, A + A_RAVEB * N, A + A_WETC * N);
            k_adj_wall_gather<<<gw, kBlock, 0, s>>>(kp, A + A_RAVEB * N, A + A_RHOBT * N);
            wetc = A + A_WETC * N;
            nwet = 2u * (unsigned)kp.plane;
        }
    }
    double *part = b.agrad + 8;
    const unsigned gr = gN < kReduceBlocks ? gN : kReduceBlocks;
    k_adj_reduce_part<<<gr, kBlock, 0, s>>>((unsigned)N, A + A_KAPC * N, nwet, wetc, nuc, part);
    k_adj_reduce_final<<<1, kBlock, 0, s>>>(gr, part, b.agrad);
    return hipGetLastError();
}

}  // namespace

size_t adjoint_aux_bytes(int, size_t N) { return (size_t)A_COUNT * 8 * N; }
size_t adjoint_grad_slots() { return 3; }

hipError_t launch_adj_seed(hipStream_t s, int prec, const KP &kp, const Bufs &b, int lcur, const double *g) {
    hipError_t e = launch_fill(s, b.agrad, 64);
    if (e != hipSuccess) return e;
    // solid-node entries of the adjoint arrays must read as zero
    e = launch_fill(s, b.abuf, adjoint_aux_bytes(prec, kp.N));
    if (e != hipSuccess) return e;
    return dispatch(prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        k_adj_seed<P><<<nblocks(kp.N), kBlock, 0, s>>>(kp, b, g, b.lam[lcur]);
        return hipGetLastError();
    });
}

hipError_t launch_adj_seed_pop(hipStream_t s, int prec, const KP &kp, const Bufs &b, int lcur, const double *g) {
    hipError_t e = launch_fill(s, b.agrad, 64);
    if (e != hipSuccess) return e;
    e = launch_fill(s, b.abuf, adjoint_aux_bytes(prec, kp.N));
    if (e != hipSuccess) return e;
    return dispatch(prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        k_adj_seed_pop<P><<<nblocks(kp.N), kBlock, 0, s>>>(kp, b, g, b.lam[lcur]);
        return hipGetLastError();
    });
}

hipError_t launch_adj_get(hipStream_t s, int prec, const KP &kp, const Bufs &b, int lcur, double *out) {
    return dispatch(prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        k_adj_get<P><<<nblocks(kp.N), kBlock, 0, s>>>(kp, b, b.lam[lcur], out);
        return hipGetLastError();
    });
}

hipError_t launch_adj_step(hipStream_t s, int prec, const KP &kp, const Bufs &b, int lcur, const void *ft,
                           bool recompute, bool pending) {
    if (recompute) {
        Bufs fb = b;
        fb.f[0] = const_cast<void *>(ft);
        hipError_t e = launch_aux(s, prec, kp, fb, 0);
        if (e != hipSuccess) return e;
    }
    const unsigned gf = nblocks(kp.nfluid);
    double *A = (double *)b.abuf;
    return dispatch(prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        if (kp.masked) {
            if (pending)
                k_adj_collide<P, true, true><<<gf, kBlock, 0, s>>>(kp, b, ft, b.lam[lcur], b.lam[1 - lcur]);
            else
                k_adj_collide<P, false, true><<<gf, kBlock, 0, s>>>(kp, b, ft, b.lam[lcur], b.lam[1 - lcur]);
            k_adj_phimu<P, true><<<zgrid(kp, 0, kp.nz), PCB, 0, s>>>(kp, b, kZChunk);
        } else {
            if (pending)
                k_adj_collide<P, true, false><<<gf, kBlock, 0, s>>>(kp, b, ft, b.lam[lcur], b.lam[1 - lcur]);
            else
                k_adj_collide<P, false, false><<<gf, kBlock, 0, s>>>(kp, b, ft, b.lam[lcur], b.lam[1 - lcur]);
            if (kp.moving) {
                const unsigned gw = nblocks(2 * (size_t)kp.plane);
                if (pending)
                    k_adj_wall_move<P, true><<<gw, kBlock, 0, s>>>(kp, b, b.lam[lcur]);
                else
                    k_adj_wall_move<P, false><<<gw, kBlock, 0, s>>>(kp, b, b.lam[lcur]);
            }
            k_adj_phimu<P, false><<<zgrid(kp, 0, kp.nz), PCB, 0, s>>>(kp, b, kZChunk);
        }
        hipError_t r = chain_tail(s, kp, b, true, A + A_NUC * (size_t)kp.N);
        if (r != hipSuccess) return r;
        k_adj_pack<P><<<gf, kBlock, 0, s>>>(kp, b);
        return hipGetLastError();  // lambda(t) = direct part; its last term is pending
    });
}

hipError_t launch_adj_finalize(hipStream_t s, int prec, const KP &kp, const Bufs &b, int lcur) {
    return dispatch(prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        k_adj_final<P><<<nblocks(kp.nfluid), kBlock, 0, s>>>(kp, b, b.lam[lcur]);
        return hipGetLastError();
    });
}

hipError_t launch_adj_init(hipStream_t s, int prec, const KP &kp, const Bufs &b, int lcur, const double *rho0,
                           const double *u0, double *out) {
    // forward initialiser quantities: rho (with wall densities) and mu
    const unsigned gN = nblocks(kp.N);
    hipError_t e = launch_init_aux(s, kp, b, rho0);
    if (e != hipSuccess) return e;
    return dispatch(prec, [&](auto pc) {
        constexpr int P = decltype(pc)::value;
        k_adj_init_local<P><<<gN, kBlock, 0, s>>>(kp, b, b.lam[lcur], u0);
        hipError_t r = chain_tail(s, kp, b, false, nullptr);
        if (r != hipSuccess) return r;
        k_adj_init_out<<<gN, kBlock, 0, s>>>(kp, b, (const double *)b.abuf + A_RHOBT * (size_t)kp.N, out);
        return hipGetLastError();
    });
}

}  // namespace lbfe
