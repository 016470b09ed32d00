// Device-side building blocks of the D3Q27 free-energy LB step (gfx950):
// precision policies, population storage codecs, neighbour indexing, the
// factorised central-moment transform, the collision of Eqs. (21)-(26) and
// the discrete operators.  Included by the forward and adjoint kernel files.
#pragma once

#include "lbfe_internal.h"

namespace lbfe {

// ---------------------------------------------------------------------------
// Lattice.  Direction i = 9 (cx+1) + 3 (cy+1) + (cz+1).  The D3Q27 weights of
// Eq. (17) are products of the D1Q3 weights 1/6, 2/3, 1/6.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr double w1(int c) { return c == 0 ? 2.0 / 3.0 : 1.0 / 6.0; }
__host__ __device__ constexpr double wq(int cx, int cy, int cz) { return w1(cx) * w1(cy) * w1(cz); }
__host__ __device__ constexpr int cxi(int i) { return i / 9 - 1; }
__host__ __device__ constexpr int cyi(int i) { return (i / 3) % 3 - 1; }
__host__ __device__ constexpr int czi(int i) { return i % 3 - 1; }
__host__ __device__ constexpr double wi(int i) { return wq(cxi(i), cyi(i), czi(i)); }
constexpr int kRest = 13;

// Central-moment slot of k_{abg} after the factorised transform.
__host__ __device__ constexpr int K(int a, int b, int g) { return 9 * a + 3 * b + g; }

// ---------------------------------------------------------------------------
// Precision policies and population storage
// ---------------------------------------------------------------------------
template <int P> struct Pol { using real = float; };
template <> struct Pol<LBFE_FP64> { using real = double; };

template <int P> struct Pops;

// Population storage is row-blocked: for every x-row (z, y) the 27
// populations are stored one after another, each as nx contiguous values,
// i.e. element (i, z, y, x) sits at ((z ny + y) 27 + i) nx + x.  A wave of
// 64 x-consecutive threads touches one contiguous run per population, and
// the 27 runs of a row share DRAM pages.
//
// Population loads are non-temporal: every kernel reads a population once
// per pass, and a lattice of a few hundred MB would otherwise push the
// reused data (aux fields, stencil halos, the freshly written lattice) out
// of the last-level cache.  Stores stay ordinary (non-temporal stores of the
// shifted push-stream rows were measured slower).
__device__ inline double ldnt(const double *p) { return __builtin_nontemporal_load(p); }
__device__ inline float ldnt(const float *p) { return __builtin_nontemporal_load(p); }
__device__ inline __half ldnt(const __half *p) {
    return __builtin_bit_cast(__half, __builtin_nontemporal_load((const unsigned short *)p));
}
template <> struct Pops<LBFE_FP64> {
    double *p;
    unsigned nx;
    __device__ Pops(const void *q, const KP &kp) : p((double *)q), nx((unsigned)kp.nx) {}
    __device__ size_t off(int i, unsigned row, unsigned x) const { return ((size_t)row * 27 + i) * nx + x; }
    __device__ double ld(int i, unsigned row, unsigned x) const { return ldnt(p + off(i, row, x)); }
    __device__ void st(int i, unsigned row, unsigned x, double v) const { p[off(i, row, x)] = v; }
    __device__ static double quant(int, double v) { return v; }  // value a store then load returns
};

template <> struct Pops<LBFE_FP32> {
    float *p;
    unsigned nx;
    __device__ Pops(const void *q, const KP &kp) : p((float *)q), nx((unsigned)kp.nx) {}
    __device__ size_t off(int i, unsigned row, unsigned x) const { return ((size_t)row * 27 + i) * nx + x; }
    __device__ float ld(int i, unsigned row, unsigned x) const { return ldnt(p + off(i, row, x)); }
    __device__ void st(int i, unsigned row, unsigned x, float v) const { p[off(i, row, x)] = v; }
    __device__ static float quant(int, float v) { return v; }
};

// Half-precision deviation from the rest-state weight, scaled by the weight:
// stored h_i = (f_i - w_i) / w_i, decoded f_i = w_i (1 + h_i).  The scale
// keeps the small deviations of the moving populations away from the half
// subnormal range.
__device__ inline float dec16(int i, __half h) {
    const float w = (float)wi(i);
    return fmaf(w, __half2float(h), w);
}
__device__ inline __half enc16(int i, float f) {
    const float iw = (float)(1.0 / wi(i));
    float t = fmaf(f, iw, -1.0f);
    // t is rounded to float before the conversion (no fused
    // multiply-add-convert instruction), so every kernel encodes a value to
    // the same half
    __asm__ volatile("" : "+v"(t));
    return __float2half_rn(t);
}

template <> struct Pops<LBFE_FP16_DEV> {
    __half *p;
    unsigned nx;
    __device__ Pops(const void *q, const KP &kp) : p((__half *)q), nx((unsigned)kp.nx) {}
    __device__ size_t off(int i, unsigned row, unsigned x) const { return ((size_t)row * 27 + i) * nx + x; }
    __device__ float ld(int i, unsigned row, unsigned x) const { return dec16(i, ldnt(p + off(i, row, x))); }
    __device__ void st(int i, unsigned row, unsigned x, float v) const { p[off(i, row, x)] = enc16(i, v); }
    __device__ static float quant(int i, float v) { return dec16(i, enc16(i, v)); }
};

// Rest population in float ([z][y][x] plane after the half rows), the 26
// moving ones as half deviations, row-blocked 26 per row.
template <> struct Pops<LBFE_FP16_DEV_F0FP32> {
    __half *p;
    float *p0;
    unsigned nx;
    __device__ Pops(const void *q, const KP &kp)
        : p((__half *)q), p0((float *)((char *)q + ((26 * 2 * (size_t)kp.N + 255) & ~size_t(255)))),
          nx((unsigned)kp.nx) {}
    __device__ static int slot(int i) { return i < kRest ? i : i - 1; }
    __device__ size_t off(int i, unsigned row, unsigned x) const { return ((size_t)row * 26 + slot(i)) * nx + x; }
    __device__ float ld(int i, unsigned row, unsigned x) const {
        return i == kRest ? ldnt(p0 + (size_t)row * nx + x) : dec16(i, ldnt(p + off(i, row, x)));
    }
    __device__ void st(int i, unsigned row, unsigned x, float v) const {
        if (i == kRest)
            p0[(size_t)row * nx + x] = v;
        else
            p[off(i, row, x)] = enc16(i, v);
    }
    __device__ static float quant(int i, float v) { return i == kRest ? v : dec16(i, enc16(i, v)); }
};

// ---------------------------------------------------------------------------
// Work mapping.  Workgroups are handed to the 8 XCDs round-robin; with
// xcd_remap the tile index is permuted so that every XCD owns one
// contiguous range of tiles (neighbouring rows share that XCD's L2).
// ---------------------------------------------------------------------------
__device__ inline unsigned tile_id(const KP &kp) {
    const unsigned b = blockIdx.x, nb = gridDim.x;
    if (!kp.xcd_remap) return b;
    const unsigned q = nb >> 3, r = nb & 7u, k = b & 7u;
    return k * q + (k < r ? k : r) + (b >> 3);
}

// Neighbour offsets of node (x, y, z) with periodic wrap: X, Y, Z give node
// indices (Y in units of nx, Z of nx ny); RY, RZ give x-row indices.
struct Nb {
    unsigned X[3], Y[3], Z[3], RY[3], RZ[3];
    __device__ Nb(const KP &kp, int x, int y, int z) {
        X[0] = x == 0 ? kp.nx - 1 : x - 1;
        X[1] = x;
        X[2] = x == kp.nx - 1 ? 0 : x + 1;
        RY[0] = y == 0 ? kp.ny - 1 : y - 1;
        RY[1] = y;
        RY[2] = y == kp.ny - 1 ? 0 : y + 1;
        RZ[0] = (z == 0 ? kp.nz - 1 : z - 1) * (unsigned)kp.ny;
        RZ[1] = z * (unsigned)kp.ny;
        RZ[2] = (z == kp.nz - 1 ? 0 : z + 1) * (unsigned)kp.ny;
        for (int k = 0; k < 3; ++k) {
            Y[k] = RY[k] * (unsigned)kp.nx;
            Z[k] = RZ[k] * (unsigned)kp.nx;
        }
    }
    __device__ unsigned at(int cx, int cy, int cz) const { return X[cx + 1] + Y[cy + 1] + Z[cz + 1]; }
    __device__ unsigned row(int cy, int cz) const { return RY[cy + 1] + RZ[cz + 1]; }
    __device__ unsigned xo(int cx) const { return X[cx + 1]; }
};

__device__ inline void decompose(const KP &kp, unsigned n, int &x, int &y, int &z) {
    z = (int)(n / kp.plane);
    const unsigned r = n - (unsigned)z * kp.plane;
    y = (int)(r / (unsigned)kp.nx);
    x = (int)(r - (unsigned)y * (unsigned)kp.nx);
}

// ---------------------------------------------------------------------------
// Macroscopic moments, Eq. (11): rho = sum f, j = sum f c, of the 27
// populations arriving at a node, summed in one fixed order in double:
// per z-layer cz and row cy the x-partials
//   R = (f(0,cy,cz) + f(+1,cy,cz)) + f(-1,cy,cz),  X = f(+1,cy,cz) - f(-1,cy,cz),
// per layer L = (R(0) + R(+1)) + R(-1), JX = (X(0) + X(+1)) + X(-1),
// JY = R(+1) - R(-1), and over the layers
//   rho = (L(+1) + L(0)) + L(-1),  jx, jy likewise,  jz = L(+1) - L(-1).
// The fused step kernel forms the same partial sums from values exchanged
// between neighbouring nodes, so the density and momentum it writes are bit
// for bit those of this function applied to the stored populations.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int dir(int cx, int cy, int cz) { return 9 * (cx + 1) + 3 * (cy + 1) + (cz + 1); }

struct Layer {
    double L, JX, JY;
};

// x-partials of row (cy, cz) from the centre value and the values arriving
// from x-1 (fp, direction +1) and x+1 (fm, direction -1)
__device__ inline void xpartial(double f0, double fp, double fm, double &R, double &X) {
    R = (f0 + fp) + fm;
    X = fp - fm;
}
__device__ inline Layer layer_of(const double (&R)[3], const double (&X)[3]) {  // index cy + 1
    return Layer{(R[1] + R[2]) + R[0], (X[1] + X[2]) + X[0], R[2] - R[0]};
}

template <class real> __device__ inline Layer layer_sum(const real (&f)[27], int cz) {
    double R[3], X[3];
#pragma unroll
    for (int cy = -1; cy <= 1; ++cy)
        xpartial((double)f[dir(0, cy, cz)], (double)f[dir(1, cy, cz)], (double)f[dir(-1, cy, cz)], R[cy + 1],
                 X[cy + 1]);
    return layer_of(R, X);
}

template <class real>
__device__ inline void moments(const real (&f)[27], double &rho, real &jx, real &jy, real &jz) {
    const Layer P = layer_sum(f, 1), Z = layer_sum(f, 0), M = layer_sum(f, -1);
    rho = (P.L + Z.L) + M.L;
    jx = (real)((P.JX + Z.JX) + M.JX);
    jy = (real)((P.JY + Z.JY) + M.JY);
    jz = (real)(P.L - M.L);
}

// Bulk chemical potential of the vdW fluid, Eq. (32) without the kappa term.
__device__ inline double mu_bulk(const KP &kp, double r) {
    const double id = 1.0 / (1.0 - kp.b * r);
    return kp.RT * (log(r * id) + id) - 2.0 * kp.a * r;
}

// ---------------------------------------------------------------------------
// Factorised central-moment transform (Eq. (19)).  Along one axis with
// velocity component u, the triple (f-, f0, f+) maps to the 1-D central
// moments (k0, k1, k2) = sum f (c - u)^n; the 3-D transform is three such
// passes (z, y, x).  After the passes slot K(a,b,g) holds k_{abg}.
// ---------------------------------------------------------------------------
template <class real> __device__ inline void fwd3(real &fm, real &f0, real &fp, real u) {
    const real s = fp + fm, d = fp - fm;
    const real k0 = s + f0;
    const real k1 = d - u * k0;
    const real k2 = s - (real)2 * u * d + u * u * k0;
    fm = k0;
    f0 = k1;
    fp = k2;
}
template <class real> __device__ inline void inv3(real &a, real &b, real &c, real u) {
    const real k0 = a, k1 = b, k2 = c;
    const real m1 = k1 + u * k0;
    const real m2 = k2 + (real)2 * u * k1 + u * u * k0;
    a = (real)0.5 * (m2 - m1);
    b = k0 - m2;
    c = (real)0.5 * (m2 + m1);
}

template <class real> __device__ inline void cm_forward(real (&f)[27], real ux, real uy, real uz) {
#pragma unroll
    for (int p = 0; p < 9; ++p) fwd3(f[3 * p], f[3 * p + 1], f[3 * p + 2], uz);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int g = 0; g < 3; ++g) fwd3(f[9 * a + g], f[9 * a + 3 + g], f[9 * a + 6 + g], uy);
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int g = 0; g < 3; ++g) fwd3(f[3 * b + g], f[9 + 3 * b + g], f[18 + 3 * b + g], ux);
}

template <class real> __device__ inline void cm_inverse(real (&f)[27], real ux, real uy, real uz) {
#pragma unroll
    for (int b = 0; b < 3; ++b)
#pragma unroll
        for (int g = 0; g < 3; ++g) inv3(f[3 * b + g], f[9 + 3 * b + g], f[18 + 3 * b + g], ux);
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int g = 0; g < 3; ++g) inv3(f[9 * a + g], f[9 * a + 3 + g], f[9 * a + 6 + g], uy);
#pragma unroll
    for (int p = 0; p < 9; ++p) inv3(f[3 * p], f[3 * p + 1], f[3 * p + 2], uz);
}

// ---------------------------------------------------------------------------
// Collision in central-moment space, Eqs. (21)-(26), toward the equilibria of
// Eq. (20).  The combination equations of each order are solved in closed
// form.  om: the 11 rates with om[1] replaced by the local omega_1.
// ---------------------------------------------------------------------------
template <class real> struct Rates {
    real w[11];
};

// The two deviatoric combinations of the normal second-order moments after
// relaxation with omega_1 (Eq. (22)): A for k200 - k020, B for k200 - k002.
template <class real> struct Dev2 {
    real A, B;
};
template <class real>
__device__ inline Dev2<real> dev2(const real (&k)[27], real w1, real q200, real q020, real q002) {
    const real one = 1, half = 0.5;
    const real k200 = k[K(2, 0, 0)], k020 = k[K(0, 2, 0)], k002 = k[K(0, 0, 2)];
    return Dev2<real>{(one - w1) * (k200 - k020) + (one - half * w1) * (q200 - q020),
                      (one - w1) * (k200 - k002) + (one - half * w1) * (q200 - q002)};
}

// The relaxation of Eqs. (21)-(26) with the normal second-order deviators D
// given (dev2 of the same moments, for collide).
template <class real>
__device__ inline void collide_dev(real (&k)[27], const Rates<real> &R, const Dev2<real> &D, real Fx, real Fy,
                                   real Fz, real pm, real q200, real q020, real q002, real q220, real q202,
                                   real q022) {
    const real one = 1, half = 0.5, third = (real)(1.0 / 3.0), ninth = (real)(1.0 / 9.0);
    const real *w = R.w;
    // first order, Eq. (21)
    k[K(1, 0, 0)] = (one - w[0]) * k[K(1, 0, 0)] + (one - half * w[0]) * Fx;
    k[K(0, 1, 0)] = (one - w[0]) * k[K(0, 1, 0)] + (one - half * w[0]) * Fy;
    k[K(0, 0, 1)] = (one - w[0]) * k[K(0, 0, 1)] + (one - half * w[0]) * Fz;
    // second order, Eq. (22)
    k[K(1, 1, 0)] *= (one - w[1]);
    k[K(0, 1, 1)] *= (one - w[1]);
    k[K(1, 0, 1)] *= (one - w[1]);
    {
        const real k200 = k[K(2, 0, 0)], k020 = k[K(0, 2, 0)], k002 = k[K(0, 0, 2)];
        const real S = (one - w[2]) * (k200 + k020 + k002) + (real)3 * w[2] * pm +
                       (one - half * w[2]) * (q200 + q020 + q002);
        k[K(2, 0, 0)] = third * (S + D.A + D.B);
        k[K(0, 2, 0)] = third * (S - (real)2 * D.A + D.B);
        k[K(0, 0, 2)] = third * (S + D.A - (real)2 * D.B);
    }
    // third order, Eq. (23)
    {
        const real c3 = (one - half * w[3]) * (real)(2.0 / 3.0), r4 = one - w[4], r3 = one - w[3];
        real P, M;
        P = r3 * (k[K(1, 2, 0)] + k[K(1, 0, 2)]) + c3 * Fx;
        M = r4 * (k[K(1, 2, 0)] - k[K(1, 0, 2)]);
        k[K(1, 2, 0)] = half * (P + M);
        k[K(1, 0, 2)] = half * (P - M);
        P = r3 * (k[K(2, 1, 0)] + k[K(0, 1, 2)]) + c3 * Fy;
        M = r4 * (k[K(2, 1, 0)] - k[K(0, 1, 2)]);
        k[K(2, 1, 0)] = half * (P + M);
        k[K(0, 1, 2)] = half * (P - M);
        P = r3 * (k[K(2, 0, 1)] + k[K(0, 2, 1)]) + c3 * Fz;
        M = r4 * (k[K(2, 0, 1)] - k[K(0, 2, 1)]);
        k[K(2, 0, 1)] = half * (P + M);
        k[K(0, 2, 1)] = half * (P - M);
        k[K(1, 1, 1)] *= (one - w[5]);
    }
    // fourth order, Eq. (24)
    {
        const real k220 = k[K(2, 2, 0)], k202 = k[K(2, 0, 2)], k022 = k[K(0, 2, 2)];
        const real D1 = (one - w[6]) * (k220 - (real)2 * k202 + k022) + (one - half * w[6]) * (q220 - (real)2 * q202 + q022);
        const real D2 = (one - w[6]) * (k220 + k202 - (real)2 * k022) + (one - half * w[6]) * (q220 + q202 - (real)2 * q022);
        const real S4 = (one - w[7]) * (k220 + k202 + k022) + w[7] * pm + (one - half * w[7]) * (q220 + q202 + q022);
        k[K(2, 2, 0)] = third * (S4 + D1 + D2);
        k[K(2, 0, 2)] = third * (S4 - D1);
        k[K(0, 2, 2)] = third * (S4 - D2);
        k[K(2, 1, 1)] *= (one - w[8]);
        k[K(1, 2, 1)] *= (one - w[8]);
        k[K(1, 1, 2)] *= (one - w[8]);
    }
    // fifth order, Eq. (25)
    {
        const real c9 = (one - half * w[9]) * ninth, r9 = one - w[9];
        k[K(1, 2, 2)] = r9 * k[K(1, 2, 2)] + c9 * Fx;
        k[K(2, 1, 2)] = r9 * k[K(2, 1, 2)] + c9 * Fy;
        k[K(2, 2, 1)] = r9 * k[K(2, 2, 1)] + c9 * Fz;
    }
    // sixth order, Eq. (26)
    k[K(2, 2, 2)] = (one - w[10]) * k[K(2, 2, 2)] + w[10] * pm * ninth;
}

template <class real>
__device__ inline void collide(real (&k)[27], const Rates<real> &R, real Fx, real Fy, real Fz, real pm, real q200,
                               real q020, real q002, real q220, real q202, real q022) {
    collide_dev(k, R, dev2(k, R.w[1], q200, q020, q002), Fx, Fy, Fz, pm, q200, q020, q002, q220, q202, q022);
}

// Fourth-order corrections of Eq. (28) from the second-order ones (0 without corr4).
template <class real> __device__ inline void q4_of(const KP &kp, real q200, real q020, real q002, real &q220,
                                                   real &q202, real &q022) {
    q220 = q202 = q022 = 0;
    if (kp.corr4) {  // Eq. (28)
        const real third = (real)(1.0 / 3.0);
        q220 = (q200 + q020) * third;
        q202 = (q200 + q002) * third;
        q022 = (q020 + q002) * third;
    }
}

// Node kinematics of Eqs. (11)-(12) and the rate after Eq. (26): u = (j +
// F/2)/rho (as a product with 1/rho), p_m = (1 + mu)/3 and omega_1 =
// 1/(rho nu/p_m + 1/2) in the form p_m/(rho nu + p_m/2).  Shared by the
// collision and the adjoint's recomputation, so both see the same roundings.
template <class real> struct Kin {
    real rho, ux, uy, uz, pm, om1;
};
template <class real>
__device__ inline Kin<real> kinematics(const KP &kp, double rd, real jx, real jy, real jz, real Fx, real Fy, real Fz,
                                       double mu) {
    Kin<real> q;
    q.rho = (real)rd;
    const real irho = (real)1 / q.rho;
    q.ux = (jx + (real)0.5 * Fx) * irho;
    q.uy = (jy + (real)0.5 * Fy) * irho;
    q.uz = (jz + (real)0.5 * Fz) * irho;
    q.pm = (real)((1.0 + mu) * (1.0 / 3.0));
    q.om1 = q.pm / (q.rho * (real)kp.nu + (real)0.5 * q.pm);
    return q;
}

// ---------------------------------------------------------------------------
// Collision of one fluid node: moments, u = (j + F/2)/rho, the local
// omega_1 = 1/(rho nu/p_m + 1/2), CM transform, Eqs. (21)-(26), inverse
// transform.  f: the arriving populations in, post-collision out.
// ---------------------------------------------------------------------------
template <class real>
__device__ inline double collide_node(const KP &kp, real (&f)[27], double mu, real Fx, real Fy, real Fz, real q200,
                                      real q020, real q002) {
    double rd;
    real jx, jy, jz;
    moments(f, rd, jx, jy, jz);
    const Kin<real> kin = kinematics(kp, rd, jx, jy, jz, Fx, Fy, Fz, mu);
    const real ux = kin.ux, uy = kin.uy, uz = kin.uz, pm = kin.pm;
    real q220, q202, q022;
    q4_of(kp, q200, q020, q002, q220, q202, q022);
    Rates<real> R;
#pragma unroll
    for (int k = 0; k < 11; ++k) R.w[k] = (real)kp.om[k];
    R.w[1] = kin.om1;

    cm_forward(f, ux, uy, uz);
    collide(f, R, Fx, Fy, Fz, pm, q200, q020, q002, q220, q202, q022);
    cm_inverse(f, ux, uy, uz);
    return rd;
}

// ---------------------------------------------------------------------------
// Moment representation of the post-collision state.  With every rate but
// omega_1 at 1 (the paper's setting, stated after Eq. (26)) the collision
// leaves 16 numbers per node that fix all 27 post-collision central moments:
//   m[0] k000 (the transform's zeroth moment, which the collision keeps),
//   m[1..3] u, m[4..6] F, m[7] p_m, m[8..10] Q200, Q020, Q002,
//   m[11..13] k*110, k*101, k*011 (relaxed with omega_1),
//   m[14..15] the deviatoric pair A, B of dev2;
// every other k* follows from Eqs. (21)-(26) at unit rates: k*100 = F_x/2,
// the normal second-order moments from A, B and their trace 3 p_m + (Q200 +
// Q020 + Q002)/2, k*120 = k*102 = F_x/6, k*111 = 0, the fourth-order triple
// from p_m and the Q terms of Eq. (28), k*211 = 0, k*122 = F_x/18 and k*222 =
// p_m/9.  state_populations rebuilds them with the collision's own code, so
// its populations are those of collide_node (zero signs aside).
// ---------------------------------------------------------------------------
constexpr int kMState = 16;

// The collision of collide_node, ending at the moment state: f, the
// arriving populations, is consumed; m receives the node's state.  Returns
// the density of the arriving populations.
template <class real>
__device__ inline double collide_to_state(const KP &kp, real (&f)[27], double mu, real Fx, real Fy, real Fz,
                                          real q200, real q020, real q002, real (&m)[kMState]) {
    double rd;
    real jx, jy, jz;
    moments(f, rd, jx, jy, jz);
    const Kin<real> kin = kinematics(kp, rd, jx, jy, jz, Fx, Fy, Fz, mu);
    cm_forward(f, kin.ux, kin.uy, kin.uz);
    const Dev2<real> D = dev2(f, kin.om1, q200, q020, q002);
    const real one = 1;
    m[0] = f[K(0, 0, 0)];
    m[1] = kin.ux;
    m[2] = kin.uy;
    m[3] = kin.uz;
    m[4] = Fx;
    m[5] = Fy;
    m[6] = Fz;
    m[7] = kin.pm;
    m[8] = q200;
    m[9] = q020;
    m[10] = q002;
    m[11] = (one - kin.om1) * f[K(1, 1, 0)];
    m[12] = (one - kin.om1) * f[K(1, 0, 1)];
    m[13] = (one - kin.om1) * f[K(0, 1, 1)];
    m[14] = D.A;
    m[15] = D.B;
    return rd;
}

// The 27 post-collision populations of a node from its moment state: the
// relaxation of collide_dev, with the node's rates, applied to central
// moments that are zero but for k000 and the omega_1-relaxed ones (those
// with omega_1 taken as 0, the deviators given).  At unit rates every other
// pre-collision moment enters multiplied by 0, so the moments and their
// roundings are those of the collision that made the state.
template <class real> __device__ inline void state_populations(const KP &kp, const real (&m)[kMState], real (&f)[27]) {
    const real Fx = m[4], Fy = m[5], Fz = m[6], pm = m[7], q200 = m[8], q020 = m[9], q002 = m[10];
    real q220, q202, q022;
    q4_of(kp, q200, q020, q002, q220, q202, q022);
#pragma unroll
    for (int i = 0; i < 27; ++i) f[i] = 0;
    f[K(0, 0, 0)] = m[0];
    f[K(1, 1, 0)] = m[11];
    f[K(1, 0, 1)] = m[12];
    f[K(0, 1, 1)] = m[13];
    Rates<real> R;
#pragma unroll
    for (int k = 0; k < 11; ++k) R.w[k] = (real)kp.om[k];
    R.w[1] = 0;
    collide_dev(f, R, Dev2<real>{m[14], m[15]}, Fx, Fy, Fz, pm, q200, q020, q002, q220, q202, q022);
    cm_inverse(f, m[1], m[2], m[3]);
}

// Populations of the generalized equilibrium of Eq. (20) at (rho, p_m) and
// the tangential wall velocity (ux, uy, 0): the moving-wall bounce-back
// gives the population reflected from direction i the correction
// -(feq_i - feq_opp(i)), so that a fluid moving with the wall is unchanged.
template <class real>
__device__ inline void wall_equilibrium(real rho, real pm, real ux, real uy, real (&feq)[27]) {
#pragma unroll
    for (int i = 0; i < 27; ++i) feq[i] = 0;
    feq[K(0, 0, 0)] = rho;
    feq[K(2, 0, 0)] = feq[K(0, 2, 0)] = feq[K(0, 0, 2)] = pm;
    feq[K(2, 2, 0)] = feq[K(2, 0, 2)] = feq[K(0, 2, 2)] = pm * (real)(1.0 / 3.0);
    feq[K(2, 2, 2)] = pm * (real)(1.0 / 9.0);
    cm_inverse(feq, ux, uy, (real)0);
}

}  // namespace lbfe
