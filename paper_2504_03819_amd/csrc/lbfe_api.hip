// C ABI of the D3Q27 free-energy LB library: parameter validation, derived
// constants, workspace layout, call ordering and error reporting.  All
// device work is delegated to the launchers in lbfe_kernels.hip and
// lbfe_adjoint.hip.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>

#include "lbfe_internal.h"

using namespace lbfe;

struct lbfe_ctx {
    lbfe_params p{};
    KP kp{};
    hipStream_t stream = nullptr;
    int device = 0;
    char *ws = nullptr;
    size_t ws_bytes = 0;
    Bufs b{};
    int cur = 0;   // index of the current population lattice
    int lcur = 0;  // index of the current adjoint lattice
    int64_t step = 0;
    bool bound = false, initialised = false, adj_seeded = false;
    bool fused = false;   // fused collide-stream-moments step (LBFE_PATH_FUSED)
    bool state = false;   // moment-representation state (LBFE_PATH_STATE)
    bool aux_ok = false;  // rho, j, mu0 hold the moments of f[cur]
    bool mask_set = false;  // a solid mask has been given (solid_mask = 1)
    bool lam_pending = false;  // lam[lcur] lacks its last term (see the adjoint kernels)
    std::string err;
};

namespace {

const char *kNoCtx = "null context";

int fail(lbfe_ctx *c, int code, const std::string &msg) {
    if (c) c->err = msg;
    return code;
}

int hip_fail(lbfe_ctx *c, hipError_t e, const char *where) {
    return fail(c, LBFE_E_DEVICE, std::string(where) + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------------------
// Maxwell coexistence of the vdW EOS (Sec. III): solve
//   mu0(rl) = mu0(rv),  p0(rl) = p0(rv)
// by Newton's method on the pair (host, double).
// ---------------------------------------------------------------------------
struct Vdw {
    double a, b, R, T;
    double mu0(double r) const { return R * T * (std::log(r / (1 - b * r)) + 1 / (1 - b * r)) - 2 * a * r; }
    double dmu0(double r) const { return R * T / (r * (1 - b * r) * (1 - b * r)) - 2 * a; }
    double p0(double r) const { return r * R * T / (1 - b * r) - a * r * r; }
};

bool maxwell_pair(const Vdw &v, double &rl, double &rv) {
    rl = 0.75 / v.b;
    rv = 0.03 / v.b;
    for (int it = 0; it < 200; ++it) {
        const double f1 = v.mu0(rl) - v.mu0(rv), f2 = v.p0(rl) - v.p0(rv);
        const double a11 = v.dmu0(rl), a12 = -v.dmu0(rv);
        const double a21 = rl * v.dmu0(rl), a22 = -rv * v.dmu0(rv);  // dp0/drho = rho dmu0/drho
        const double det = a11 * a22 - a12 * a21;
        if (!(std::fabs(det) > 0)) return false;
        const double dl = (f1 * a22 - f2 * a12) / det, dv = (a11 * f2 - a21 * f1) / det;
        double s = 1.0, nl, nv;
        for (;;) {
            nl = rl - s * dl;
            nv = rv - s * dv;
            if (nv > 0 && nv < nl && nl * v.b < 1) break;
            s *= 0.5;
            if (s < 1e-12) return false;
        }
        rl = nl;
        rv = nv;
        if (std::fabs(dl) + std::fabs(dv) < 1e-14 * rl) return std::isfinite(rl) && std::isfinite(rv) && rl - rv > 1e-8;
    }
    return false;
}

bool finite(double x) { return std::isfinite(x); }

// Validation that needs no device.  Returns an empty string when valid.
std::string validate(const lbfe_params &p) {
    if (p.nx < 1 || p.ny < 1 || p.nz < 1) return "nx, ny, nz must be >= 1";
    if (p.walls_z != 0 && p.walls_z != 1) return "walls_z must be 0 or 1";
    if (p.walls_z && p.nz < 3) return "walls_z needs nz >= 3";
    const double N = (double)p.nx * (double)p.ny * (double)p.nz;
    if (N > 2147483647.0) return "nx*ny*nz must be < 2^31";
    if ((double)p.nx * (double)p.ny > 268435456.0) return "nx*ny must be <= 2^28";
    if (p.precision < LBFE_FP64 || p.precision > LBFE_FP16_DEV_F0FP32) return "unknown precision";
    if (!(p.a > 0 && p.b > 0 && p.R > 0 && p.T > 0) || !finite(p.a) || !finite(p.b) || !finite(p.R) || !finite(p.T))
        return "a, b, R, T must be finite and > 0";
    if (!(p.kappa >= 0) || !finite(p.kappa)) return "kappa must be finite and >= 0";
    if (!(p.nu > 0) || !finite(p.nu)) return "nu must be finite and > 0";
    for (int k = 0; k < 11; ++k) {
        if (k == 1) continue;
        if (!(p.omega[k] >= 0 && p.omega[k] <= 2)) return "omega_k must lie in [0, 2]";
    }
    if (p.corr4 != 0 && p.corr4 != 1) return "corr4 must be 0 or 1";
    if (p.wet_mode < LBFE_WET_NEUTRAL || p.wet_mode > LBFE_WET_DELTA) return "unknown wet_mode";
    if (!finite(p.wet_value)) return "wet_value must be finite";
    if (p.wet_mode == LBFE_WET_PHI && !(p.wet_value > 0)) return "phi must be > 0";
    if (p.wet_mode == LBFE_WET_DELTA && !(p.wet_value >= 0)) return "drho must be >= 0";
    if (!finite(p.rho_l) || !finite(p.rho_v) || p.rho_l < 0 || p.rho_v < 0) return "rho_l, rho_v must be >= 0";
    if ((p.rho_l > 0) != (p.rho_v > 0)) return "give both rho_l and rho_v, or neither";
    if (p.rho_l > 0 && !(p.rho_l > p.rho_v)) return "rho_l must exceed rho_v";
    if (p.check_every < 1) return "check_every must be >= 1";
    if (p.adjoint != 0 && p.adjoint != 1) return "adjoint must be 0 or 1";
    bool moving = false;
    for (int k = 0; k < 4; ++k) {
        if (!finite(p.wall_u[k]) || std::fabs(p.wall_u[k]) > 0.3) return "wall_u must be finite with |u| <= 0.3";
        moving = moving || p.wall_u[k] != 0.0;
    }
    if (moving && !p.walls_z) return "moving walls need walls_z = 1";
    if (p.solid_mask != 0 && p.solid_mask != 1) return "solid_mask must be 0 or 1";
    if (p.solid_mask && p.walls_z) return "solid_mask replaces walls_z (put the planes into the mask)";
    if (p.step_path < LBFE_AUTO || p.step_path > LBFE_PATH_STATE) return "unknown step_path";
    if (p.step_path == LBFE_PATH_STATE) {  // the moment state: the paper's rates, storage and boundaries
        if (p.precision != LBFE_FP64 && p.precision != LBFE_FP32) return "the moment-state path stores FP64 or FP32 only";
        for (int k = 0; k < 11; ++k)
            if (k != 1 && p.omega[k] != 1.0) return "the moment-state path needs every omega_k but omega_1 equal to 1";
        if (moving) return "the moment-state path has resting walls only";
        if (p.solid_mask) return "the moment-state path has no solid mask";
        if (!state_plane_ok(p.precision, (size_t)p.nx * p.ny)) return "the moment-state path needs a z-plane below 2 GiB";
    }
    if (p.tile_order < LBFE_AUTO || p.tile_order > LBFE_ORDER_XCD) return "unknown tile_order";
    if (p.chain_chunk < 0 || p.chain_chunk > 64) return "chain_chunk must be 0 (chosen per grid) or 1..64";
    return "";
}

// Workspace layout: every sub-buffer 256-byte aligned.
struct Layout {
    size_t f0, f1, rho, j, mu, mu0, F, Q, nbr, phi, flag, part, red, lam0, lam1, abuf, agrad, total;
};

bool moving_walls(const lbfe_params &p) {
    return p.wall_u[0] != 0.0 || p.wall_u[1] != 0.0 || p.wall_u[2] != 0.0 || p.wall_u[3] != 0.0;
}

// the fused step path is possible: no mask, 32-bit plane offsets
bool fused_possible(const lbfe_params &p) {
    return !p.solid_mask && fused_plane_ok(p.precision, (size_t)p.nx * p.ny);
}

size_t al(size_t x) { return (x + 255) & ~size_t(255); }

Layout layout(const lbfe_params &p) {
    const size_t N = (size_t)p.nx * p.ny * p.nz;
    const size_t nf = p.walls_z ? (size_t)p.nx * p.ny * (p.nz - 2) : N;
    const size_t rb = real_bytes(p.precision);
    Layout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += al(bytes); return r; };
    L.f0 = take(pop_bytes(p.precision, N));
    L.f1 = take(pop_bytes(p.precision, N));
    L.rho = take(8 * N);
    L.j = take(3 * rb * N);
    L.mu = take(8 * N);
    L.mu0 = take(8 * N);
    L.F = take(3 * rb * N);
    L.Q = take(3 * rb * N);
    if (p.solid_mask) {
        L.nbr = take(4 * N);
        L.phi = take(3 * rb * N);
    }
    L.flag = take(256);
    L.part = take(8 * 8 * (size_t)nblocks(nf) + 8 * 8 * (size_t)nblocks(N));
    L.red = take(64);
    if (p.adjoint) {
        L.lam0 = take(lambda_bytes(p.precision, N));
        L.lam1 = take(lambda_bytes(p.precision, N));
        L.abuf = take(adjoint_aux_bytes(p.precision, N));
        L.agrad = take(8 * (8 + adjoint_grad_slots() * (size_t)nblocks(N)));
    }
    L.total = o;
    return L;
}

int need_bound(lbfe_ctx *c) {
    if (!c) return LBFE_E_INVAL;
    if (!c->bound) return fail(c, LBFE_E_STATE, "no workspace bound (lbfe_bind_workspace)");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, LBFE_E_DEVICE, "hipSetDevice failed");
    return LBFE_OK;
}

// a context with solid_mask = 1 needs its mask before any state
int need_mask(lbfe_ctx *c) {
    int r = need_bound(c);
    if (r) return r;
    if (c->p.solid_mask && !c->mask_set) return fail(c, LBFE_E_STATE, "no solid mask (lbfe_set_solid)");
    return LBFE_OK;
}

int need_init(lbfe_ctx *c) {
    int r = need_bound(c);
    if (r) return r;
    if (!c->initialised) return fail(c, LBFE_E_STATE, "no state (lbfe_init_density or lbfe_set_state)");
    return LBFE_OK;
}

int read_flag(lbfe_ctx *c, int &flag) {
    hipError_t e = hipMemcpyAsync(&flag, c->b.flag, sizeof(int), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "flag readback");
    return LBFE_OK;
}

// Completes lambda(t) in place when its last term is still pending (before
// lambda is read out or the auxiliary planes are reused).
int finalize_lambda(lbfe_ctx *c) {
    if (!c->lam_pending) return LBFE_OK;
    hipError_t e = launch_adj_finalize(c->stream, c->p.precision, c->kp, c->b, c->lcur);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint finalize");
    c->lam_pending = false;
    return LBFE_OK;
}

// One record of forward auxiliary fields: rho, mu (double, N each), then
// j, F, Q (3 N each, compute precision), sub-buffers 256-byte aligned.
struct AuxLayout {
    size_t rho, mu, j, F, Q, total;
};

AuxLayout aux_layout(const lbfe_params &p) {
    const size_t N = (size_t)p.nx * p.ny * p.nz, rb = real_bytes(p.precision);
    AuxLayout L{};
    size_t o = 0;
    auto take = [&](size_t bytes) { size_t r = o; o += al(bytes); return r; };
    L.rho = take(8 * N);
    L.mu = take(8 * N);
    L.j = take(3 * rb * N);
    L.F = take(3 * rb * N);
    L.Q = take(3 * rb * N);
    L.total = o;
    return L;
}

// the context's buffers with the aux fields redirected into a record
Bufs with_aux(const lbfe_ctx *c, const void *aux) {
    const AuxLayout L = aux_layout(c->p);
    char *a = (char *)const_cast<void *>(aux);
    Bufs b = c->b;
    b.rho = (double *)(a + L.rho);
    b.mu = (double *)(a + L.mu);
    b.j = a + L.j;
    b.F = a + L.F;
    b.Q = a + L.Q;
    return b;
}

// Steps through the moment state: the populations f[cur] enter the state
// form with the first collision and leave it with the last streaming, so
// between calls the context holds populations.  The state lattices are the
// two population buffers in turn.  With kernel_ms, accumulates the launch
// groups' times as lbfe_step_timed describes.
int step_state(lbfe_ctx *c, int64_t nsteps, double *kernel_ms) {
    if (nsteps == 0) return LBFE_OK;
    const int prec = c->p.precision;
    hipEvent_t ev[3] = {nullptr, nullptr, nullptr};
    hipEvent_t *evp = nullptr;
    if (kernel_ms) {
        for (int k = 0; k < 3; ++k)
            if (hipEventCreate(&ev[k]) != hipSuccess) {
                for (int q = 0; q < k; ++q) (void)hipEventDestroy(ev[q]);
                return fail(c, LBFE_E_DEVICE, "hipEventCreate failed");
            }
        evp = ev;
    }
    // events ev[0..n-1] of the last launch group: interval 0 to slot a, 1 to b
    auto account = [&](int n, int a, int b) -> hipError_t {
        if (!evp) return hipSuccess;
        hipError_t e = hipEventSynchronize(ev[n - 1]);
        float ms = 0.f;
        if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
        kernel_ms[a] += ms;
        if (e == hipSuccess && n == 3) {
            e = hipEventElapsedTime(&ms, ev[1], ev[2]);
            kernel_ms[b] += ms;
        }
        return e;
    };
    int rc = LBFE_OK;
    int a = 1 - c->cur;  // the lattice holding the state
    hipError_t e = launch_state_enter(c->stream, prec, c->kp, c->b, c->cur, !c->aux_ok, evp);
    if (e == hipSuccess) e = account(3, 1, 2);
    for (int64_t s = 0; s < nsteps && e == hipSuccess && rc == LBFE_OK; ++s) {
        const bool last = s + 1 == nsteps;
        // completes step s: the moments of the streamed state (populations too
        // at the end)
        e = launch_state_moments(c->stream, prec, c->kp, c->b, a, last, evp);
        if (e == hipSuccess) e = account(2, 0, 0);
        if (e != hipSuccess) break;
        c->step++;
        if (last) c->cur = 1 - a;
        if ((s + 1) % c->p.check_every == 0 || last) {
            int flag = 0;
            if ((rc = read_flag(c, flag))) break;
            if (flag) {
                if (!last) {  // leave the state form
                    e = launch_state_moments(c->stream, prec, c->kp, c->b, a, true, nullptr);
                    c->cur = 1 - a;
                    if (e != hipSuccess) break;
                }
                char buf[160];
                std::snprintf(buf, sizeof buf, "diverged: NaN/Inf or density outside (0, 1/b) by step %lld",
                              (long long)c->step);
                rc = fail(c, LBFE_E_DIVERGED, buf);
                break;
            }
        }
        if (!last) {  // the collision of step s + 1
            e = launch_state_collide(c->stream, prec, c->kp, c->b, a, evp);
            if (e == hipSuccess) e = account(3, 1, 2);
            a ^= 1;
        }
    }
    for (int k = 0; k < 3; ++k)
        if (ev[k]) (void)hipEventDestroy(ev[k]);
    if (e != hipSuccess) return hip_fail(c, e, "step (moment state)");
    c->aux_ok = true;
    return rc;
}

}  // namespace

extern "C" {

int lbfe_params_default(lbfe_params *p) {
    if (!p) return LBFE_E_INVAL;
    std::memset(p, 0, sizeof(*p));
    p->nx = p->ny = p->nz = 32;
    p->walls_z = 0;
    p->precision = LBFE_FP64;
    p->a = 9.0 / 392.0;
    p->b = 2.0 / 21.0;
    p->R = 1.0;
    p->T = 0.7 * 8.0 * p->a / (27.0 * p->R * p->b);
    p->kappa = 0.02;
    p->nu = 0.15;
    for (int k = 0; k < 11; ++k) p->omega[k] = 1.0;
    p->corr4 = 1;
    p->wet_mode = LBFE_WET_NEUTRAL;
    p->wet_value = 1.0;
    p->rho_l = p->rho_v = 0.0;
    p->check_every = 100;
    p->adjoint = 0;
    return LBFE_OK;
}

int lbfe_coexistence(double a, double b, double R, double T, double *rho_l, double *rho_v) {
    if (!rho_l || !rho_v || !(a > 0 && b > 0 && R > 0)) return LBFE_E_INVAL;
    const double Tc = 8 * a / (27 * R * b);
    if (!(T > 0.3 * Tc && T < Tc)) return LBFE_E_INVAL;
    double rl, rv;
    if (!maxwell_pair(Vdw{a, b, R, T}, rl, rv)) return LBFE_E_INVAL;
    *rho_l = rl;
    *rho_v = rv;
    return LBFE_OK;
}

int lbfe_workspace_bytes(const lbfe_params *p, size_t *bytes) {
    if (!p || !bytes) return LBFE_E_INVAL;
    if (!validate(*p).empty()) return LBFE_E_INVAL;
    *bytes = layout(*p).total;
    return LBFE_OK;
}

int lbfe_create(const lbfe_params *p, void *hip_stream, lbfe_ctx **out) {
    if (!p || !out) return LBFE_E_INVAL;
    *out = nullptr;
    const std::string why = validate(*p);
    if (!why.empty()) {
        std::fprintf(stderr, "lbfe_create: %s\n", why.c_str());
        return LBFE_E_INVAL;
    }
    lbfe_params q = *p;
    const double Tc = 8 * q.a / (27 * q.R * q.b);
    if (q.rho_l == 0.0) {
        double rl = 0, rv = 0;
        if (q.T > 0.3 * Tc && q.T < Tc && maxwell_pair(Vdw{q.a, q.b, q.R, q.T}, rl, rv)) {
            q.rho_l = rl;
            q.rho_v = rv;
        } else if ((q.walls_z || q.solid_mask) && q.wet_mode != LBFE_WET_NEUTRAL) {
            std::fprintf(stderr, "lbfe_create: no coexistence pair at this T; give rho_l, rho_v\n");
            return LBFE_E_INVAL;
        }
    }
    int ndev = 0;
    if (hipGetDeviceCount(&ndev) != hipSuccess || ndev < 1) return LBFE_E_DEVICE;
    lbfe_ctx *c = new (std::nothrow) lbfe_ctx();
    if (!c) return LBFE_E_NOMEM;
    if (hipGetDevice(&c->device) != hipSuccess) {
        delete c;
        return LBFE_E_DEVICE;
    }
    c->p = q;
    c->stream = (hipStream_t)hip_stream;
    KP &k = c->kp;
    k.nx = (int)q.nx;
    k.ny = (int)q.ny;
    k.nz = (int)q.nz;
    k.plane = (unsigned)(q.nx * q.ny);
    k.N = (unsigned)(q.nx * q.ny * q.nz);
    k.walls = q.walls_z;
    k.z0 = q.walls_z ? 1 : 0;
    k.z1 = q.walls_z ? (int)q.nz - 1 : (int)q.nz;
    k.nfluid = (unsigned)(k.z1 - k.z0) * k.plane;
    k.a = q.a;
    k.b = q.b;
    k.RT = q.R * q.T;
    k.kappa = q.kappa;
    k.nu = q.nu;
    for (int i = 0; i < 11; ++i) k.om[i] = q.omega[i];
    k.corr4 = q.corr4;
    for (int i = 0; i < 4; ++i) k.wall_u[i] = q.wall_u[i];
    k.moving = q.wall_u[0] != 0.0 || q.wall_u[1] != 0.0 || q.wall_u[2] != 0.0 || q.wall_u[3] != 0.0;
    k.masked = q.solid_mask;
    k.wet_mode = q.wet_mode;
    k.wet_value = q.wet_value;
    k.lo = 0.05 * q.rho_l + 0.95 * q.rho_v;
    k.hi = 0.95 * q.rho_l + 0.05 * q.rho_v;
    // Schedule (none of it changes a result bit).  Tile order of the
    // streaming kernels: with the hardware's round-robin dealing every XCD
    // works on every eighth tile, and on large grids the push-stream writes
    // then span the whole active z-window on every XCD; one contiguous range
    // of tiles per XCD is 18-27 % faster at 512^3, and on smaller grids also
    // faster whenever nx or ny is not a power of two (160^3, 200^3,
    // 192x192x96: +8-10 %; 320^3 and 384x384x128 in FP32: +16-20 %), neutral
    // at 128^3 and 256^3, and slower on the solid-mask path (its stencil
    // gathers read neighbour rows that the round-robin order keeps in every
    // XCD's L2).
    auto pow2 = [](unsigned v) { return (v & (v - 1)) == 0; };
    const bool irregular = !pow2((unsigned)k.nx) || !pow2((unsigned)k.ny);
    if (q.tile_order == LBFE_AUTO)
        q.tile_order = (k.N >= (1u << 26) || (irregular && !k.masked)) ? LBFE_ORDER_XCD : LBFE_ORDER_ROUND_ROBIN;
    k.xcd_remap = q.tile_order == LBFE_ORDER_XCD;
    // Planes per workgroup of the stencil chain: chosen per grid unless given.
    k.chain_cz = q.chain_chunk;
    q.chain_chunk = k.chain_cz = chain_chunk_for(k);
    // Step path: the fused collide-stream-moments kernel reads the
    // populations once per step; it has no solid mask, and addresses one
    // z-plane of the lattice with 32-bit offsets.  Measured on
    // gfx950 it is faster in FP64 on large grids (256^3: 2.44 against
    // 2.76 ms per step; 512^3: 19.0 against 22.1 ms) and slower in the FP32
    // and FP16 forms, whose collide-stream pass alone runs closer to the
    // bandwidth than the fused kernel with its ring of recollided nodes
    // (512^3 FP32: 12.6 against 11.6 ms per step).
    const bool fused_ok = fused_possible(q);
    if (q.step_path == LBFE_AUTO)
        q.step_path = fused_ok && q.precision == LBFE_FP64 && k.N >= (1u << 24) ? LBFE_PATH_FUSED : LBFE_PATH_TWO_PASS;
    if (q.step_path == LBFE_PATH_FUSED && !fused_ok) {
        std::fprintf(stderr, "lbfe_create: the fused step path needs no solid mask and a lattice z-plane below "
                             "2 GiB\n");
        delete c;
        return LBFE_E_INVAL;
    }
    c->fused = q.step_path == LBFE_PATH_FUSED;
    c->state = q.step_path == LBFE_PATH_STATE;
    c->p = q;
    *out = c;
    return LBFE_OK;
}

int lbfe_bind_workspace(lbfe_ctx *c, void *ws, size_t bytes) {
    if (!c) return LBFE_E_INVAL;
    if (!ws) return fail(c, LBFE_E_INVAL, "null workspace");
    if (((uintptr_t)ws & 255u) != 0) return fail(c, LBFE_E_INVAL, "workspace must be 256-byte aligned");
    const Layout L = layout(c->p);
    if (bytes < L.total) return fail(c, LBFE_E_NOMEM, "workspace smaller than lbfe_workspace_bytes");
    if (hipSetDevice(c->device) != hipSuccess) return fail(c, LBFE_E_DEVICE, "hipSetDevice failed");
    char *w = (char *)ws;
    c->ws = w;
    c->ws_bytes = bytes;
    c->b.f[0] = w + L.f0;
    c->b.f[1] = w + L.f1;
    c->b.rho = (double *)(w + L.rho);
    c->b.j = w + L.j;
    c->b.mu = (double *)(w + L.mu);
    c->b.mu0 = (double *)(w + L.mu0);
    c->b.F = w + L.F;
    c->b.Q = w + L.Q;
    if (c->p.solid_mask) {
        c->b.nbr = (unsigned *)(w + L.nbr);
        c->b.phi = w + L.phi;
    }
    c->b.flag = (int *)(w + L.flag);
    c->b.part = (double *)(w + L.part);
    c->b.red = (double *)(w + L.red);
    if (c->p.adjoint) {
        c->b.lam[0] = w + L.lam0;
        c->b.lam[1] = w + L.lam1;
        c->b.abuf = w + L.abuf;
        c->b.agrad = (double *)(w + L.agrad);
    }
    hipError_t e = launch_fill(c->stream, ws, L.total);
    if (e != hipSuccess) return hip_fail(c, e, "workspace clear");
    c->bound = true;
    c->initialised = false;
    c->aux_ok = false;
    c->mask_set = false;
    c->adj_seeded = false;
    c->cur = 0;
    c->step = 0;
    return LBFE_OK;
}

int lbfe_get_params(const lbfe_ctx *c, lbfe_params *out) {
    if (!c || !out) return LBFE_E_INVAL;
    *out = c->p;
    return LBFE_OK;
}

int lbfe_set_solid(lbfe_ctx *c, const uint8_t *mask) {
    int r = need_bound(c);
    if (r) return r;
    if (!c->p.solid_mask) return fail(c, LBFE_E_STATE, "created with solid_mask = 0");
    if (!mask) return fail(c, LBFE_E_INVAL, "null mask");
    hipError_t e = launch_mask_prep(c->stream, c->kp, c->b, mask);
    if (e != hipSuccess) return hip_fail(c, e, "set_solid");
    c->mask_set = true;
    c->initialised = false;
    c->aux_ok = false;
    return LBFE_OK;
}

int lbfe_init_density(lbfe_ctx *c, const double *rho0, const double *u0) {
    int r = need_mask(c);
    if (r) return r;
    if (!rho0) return fail(c, LBFE_E_INVAL, "rho0 is null");
    hipError_t e = launch_fill(c->stream, c->b.flag, 256);
    if (e == hipSuccess)
        e = c->kp.masked ? launch_check_rho0_mask(c->stream, c->kp, c->b, rho0, c->b.flag)
                         : launch_check_rho0(c->stream, c->kp, rho0, c->b.flag);
    if (e != hipSuccess) return hip_fail(c, e, "init check");
    int flag = 0;
    if ((r = read_flag(c, flag))) return r;
    if (flag) return fail(c, LBFE_E_INVAL, "rho0 not finite or outside 0 < rho < 1/b at a fluid node");
    c->cur = 0;
    c->aux_ok = false;
    e = launch_init(c->stream, c->p.precision, c->kp, c->b, c->cur, rho0, u0);
    if (e != hipSuccess) return hip_fail(c, e, "init");
    c->step = 0;
    c->initialised = true;
    return LBFE_OK;
}

int lbfe_step(lbfe_ctx *c, int64_t nsteps) {
    int r = need_init(c);
    if (r) return r;
    if (nsteps < 0) return fail(c, LBFE_E_INVAL, "nsteps < 0");
    if (c->state) return step_state(c, nsteps, nullptr);
    for (int64_t s = 0; s < nsteps; ++s) {
        hipError_t e = launch_step(c->stream, c->p.precision, c->kp, c->b, c->cur, c->fused, !c->aux_ok, nullptr);
        if (e != hipSuccess) return hip_fail(c, e, "step");
        c->cur ^= 1;
        c->step++;
        c->aux_ok = c->fused;
        if ((s + 1) % c->p.check_every == 0 || s + 1 == nsteps) {
            int flag = 0;
            if ((r = read_flag(c, flag))) return r;
            if (flag) {
                char buf[160];
                std::snprintf(buf, sizeof buf, "diverged: NaN/Inf or density outside (0, 1/b) by step %lld",
                              (long long)c->step);
                return fail(c, LBFE_E_DIVERGED, buf);
            }
        }
    }
    return LBFE_OK;
}

int lbfe_step_timed(lbfe_ctx *c, int64_t nsteps, double kernel_ms[4]) {
    int r = need_init(c);
    if (r) return r;
    if (nsteps < 0 || !kernel_ms) return fail(c, LBFE_E_INVAL, "nsteps < 0 or null kernel_ms");
    hipEvent_t ev[5];
    for (int k = 0; k < 5; ++k)
        if (hipEventCreate(&ev[k]) != hipSuccess) {
            for (int q = 0; q < k; ++q) (void)hipEventDestroy(ev[q]);
            return fail(c, LBFE_E_DEVICE, "hipEventCreate failed");
        }
    for (int k = 0; k < 4; ++k) kernel_ms[k] = 0.0;
    if (c->state) {
        for (int k = 0; k < 5; ++k) (void)hipEventDestroy(ev[k]);
        return step_state(c, nsteps, kernel_ms);
    }
    int rc = LBFE_OK;
    for (int64_t s = 0; s < nsteps && rc == LBFE_OK; ++s) {
        hipError_t e = launch_step(c->stream, c->p.precision, c->kp, c->b, c->cur, c->fused, !c->aux_ok, ev);
        if (e == hipSuccess) e = hipEventSynchronize(ev[4]);
        if (e != hipSuccess) {
            rc = hip_fail(c, e, "step_timed");
            break;
        }
        for (int k = 0; k < 4; ++k) {
            float ms = 0.f;
            (void)hipEventElapsedTime(&ms, ev[k], ev[k + 1]);
            kernel_ms[k] += ms;
        }
        c->cur ^= 1;
        c->step++;
        c->aux_ok = c->fused;
    }
    for (int k = 0; k < 5; ++k) (void)hipEventDestroy(ev[k]);
    if (rc == LBFE_OK) {
        int flag = 0;
        if ((rc = read_flag(c, flag))) return rc;
        if (flag) return fail(c, LBFE_E_DIVERGED, "diverged during timed steps");
    }
    return rc;
}

int lbfe_step_count(const lbfe_ctx *c, int64_t *step) {
    if (!c || !step) return LBFE_E_INVAL;
    *step = c->step;
    return LBFE_OK;
}

int lbfe_field(lbfe_ctx *c, int which, double *out) {
    int r = need_init(c);
    if (r) return r;
    if (!out) return fail(c, LBFE_E_INVAL, "null output");
    if (which < LBFE_FIELD_RHO || which > LBFE_FIELD_PM) return fail(c, LBFE_E_INVAL, "unknown field");
    hipError_t e = launch_aux(c->stream, c->p.precision, c->kp, c->b, c->cur);
    if (e == hipSuccess) e = launch_export(c->stream, c->p.precision, c->kp, c->b, which, out);
    if (e != hipSuccess) return hip_fail(c, e, "field export");
    return LBFE_OK;
}

int lbfe_fields(lbfe_ctx *c, double *rho, double *u, double *mu, double *F) {
    int r = need_init(c);
    if (r) return r;
    hipError_t e = launch_aux(c->stream, c->p.precision, c->kp, c->b, c->cur);
    if (e == hipSuccess && rho) e = launch_export(c->stream, c->p.precision, c->kp, c->b, LBFE_FIELD_RHO, rho);
    if (e == hipSuccess && u) e = launch_export(c->stream, c->p.precision, c->kp, c->b, LBFE_FIELD_U, u);
    if (e == hipSuccess && mu) e = launch_export(c->stream, c->p.precision, c->kp, c->b, LBFE_FIELD_MU, mu);
    if (e == hipSuccess && F) e = launch_export(c->stream, c->p.precision, c->kp, c->b, LBFE_FIELD_F, F);
    if (e != hipSuccess) return hip_fail(c, e, "fields");
    return LBFE_OK;
}

int lbfe_state_bytes(const lbfe_ctx *c, size_t *bytes) {
    if (!c || !bytes) return LBFE_E_INVAL;
    *bytes = pop_bytes(c->p.precision, c->kp.N);
    return LBFE_OK;
}

int lbfe_get_state(lbfe_ctx *c, void *dst) {
    int r = need_init(c);
    if (r) return r;
    if (!dst) return fail(c, LBFE_E_INVAL, "null destination");
    hipError_t e = hipMemcpyAsync(dst, c->b.f[c->cur], pop_bytes(c->p.precision, c->kp.N), hipMemcpyDeviceToDevice,
                                  c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "get_state");
    return LBFE_OK;
}

int lbfe_set_state(lbfe_ctx *c, const void *src, int64_t step) {
    int r = need_mask(c);
    if (r) return r;
    if (!src) return fail(c, LBFE_E_INVAL, "null source");
    if (step < 0) return fail(c, LBFE_E_INVAL, "step < 0");
    hipError_t e = hipMemcpyAsync(c->b.f[c->cur], src, pop_bytes(c->p.precision, c->kp.N), hipMemcpyDeviceToDevice,
                                  c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "set_state");
    c->aux_ok = false;
    c->step = step;
    c->initialised = true;
    return LBFE_OK;
}

int lbfe_get_populations(lbfe_ctx *c, double *f) {
    int r = need_init(c);
    if (r) return r;
    if (!f) return fail(c, LBFE_E_INVAL, "null destination");
    hipError_t e = launch_get_pop(c->stream, c->p.precision, c->kp, c->b, c->b.f[c->cur], f);
    if (e != hipSuccess) return hip_fail(c, e, "get_populations");
    return LBFE_OK;
}

int lbfe_set_populations(lbfe_ctx *c, const double *f) {
    int r = need_mask(c);
    if (r) return r;
    if (!f) return fail(c, LBFE_E_INVAL, "null source");
    hipError_t e = launch_set_pop(c->stream, c->p.precision, c->kp, c->b, c->b.f[c->cur], f);
    if (e != hipSuccess) return hip_fail(c, e, "set_populations");
    c->aux_ok = false;
    c->initialised = true;
    return LBFE_OK;
}

int lbfe_reduce(lbfe_ctx *c, double out[8]) {
    int r = need_init(c);
    if (r) return r;
    if (!out) return fail(c, LBFE_E_INVAL, "null output");
    hipError_t e = launch_aux(c->stream, c->p.precision, c->kp, c->b, c->cur);
    if (e == hipSuccess) e = launch_reduce(c->stream, c->p.precision, c->kp, c->b);
    if (e == hipSuccess) e = hipMemcpyAsync(out, c->b.red, 8 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "reduce");
    return LBFE_OK;
}

int lbfe_reduce_into(lbfe_ctx *c, double *out_dev) {
    if (!c) return LBFE_E_INVAL;
    if (nblocks(c->kp.nfluid) > kScratchPartials) {
        char buf[160];
        std::snprintf(buf, sizeof buf, "lbfe_reduce_into serves up to %u fluid nodes (static scratch); use lbfe_reduce",
                      kScratchPartials * (unsigned)kBlock);
        return fail(c, LBFE_E_INVAL, buf);
    }
    int r = need_init(c);
    if (r) return r;
    if (!out_dev) return fail(c, LBFE_E_INVAL, "null output");
    double *part = nullptr;
    hipError_t e = scratch_partials(c->device, &part);
    if (e != hipSuccess) return hip_fail(c, e, "reduce_into: scratch address");
    e = launch_aux(c->stream, c->p.precision, c->kp, c->b, c->cur);
    if (e == hipSuccess) e = launch_reduce_into(c->stream, c->p.precision, c->kp, c->b, part, out_dev);
    if (e != hipSuccess) return hip_fail(c, e, "reduce_into");
    return LBFE_OK;
}

int lbfe_adjoint_seed(lbfe_ctx *c, const double *dLdrho) {
    int r = need_bound(c);
    if (r) return r;
    if (!c->p.adjoint) return fail(c, LBFE_E_STATE, "created without params.adjoint = 1");
    if (!dLdrho) return fail(c, LBFE_E_INVAL, "null dL/drho");
    c->lcur = 0;
    c->lam_pending = false;
    hipError_t e = launch_adj_seed(c->stream, c->p.precision, c->kp, c->b, c->lcur, dLdrho);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint_seed");
    c->adj_seeded = true;
    return LBFE_OK;
}

int lbfe_adjoint_seed_populations(lbfe_ctx *c, const double *g) {
    int r = need_bound(c);
    if (r) return r;
    if (!c->p.adjoint) return fail(c, LBFE_E_STATE, "created without params.adjoint = 1");
    if (!g) return fail(c, LBFE_E_INVAL, "null dL/df");
    c->lcur = 0;
    c->lam_pending = false;
    hipError_t e = launch_adj_seed_pop(c->stream, c->p.precision, c->kp, c->b, c->lcur, g);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint_seed_populations");
    c->adj_seeded = true;
    return LBFE_OK;
}

int lbfe_adjoint_get(lbfe_ctx *c, double *out) {
    int r = need_bound(c);
    if (r) return r;
    if (!c->p.adjoint) return fail(c, LBFE_E_STATE, "created without params.adjoint = 1");
    if (!c->adj_seeded) return fail(c, LBFE_E_STATE, "adjoint not seeded");
    if (!out) return fail(c, LBFE_E_INVAL, "null output");
    if ((r = finalize_lambda(c))) return r;
    hipError_t e = launch_adj_get(c->stream, c->p.precision, c->kp, c->b, c->lcur, out);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint_get");
    return LBFE_OK;
}

int lbfe_adjoint_step(lbfe_ctx *c, const void *ft) {
    int r = need_bound(c);
    if (r) return r;
    if (!c->p.adjoint) return fail(c, LBFE_E_STATE, "created without params.adjoint = 1");
    if (!c->adj_seeded) return fail(c, LBFE_E_STATE, "adjoint not seeded");
    if (!ft) {  // the context's current state (read only: the step writes lambda and fields)
        if (!c->initialised) return fail(c, LBFE_E_STATE, "no current state");
        ft = c->b.f[c->cur];
    }
    c->aux_ok = false;  // the recomputation below overwrites rho, j, mu0
    hipError_t e = launch_adj_step(c->stream, c->p.precision, c->kp, c->b, c->lcur, ft, true, c->lam_pending);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint_step");
    c->lcur ^= 1;
    c->lam_pending = true;
    return LBFE_OK;
}

int lbfe_aux_bytes(const lbfe_ctx *c, size_t *bytes) {
    if (!c || !bytes) return LBFE_E_INVAL;
    *bytes = aux_layout(c->p).total;
    return LBFE_OK;
}

int lbfe_step_aux(lbfe_ctx *c, void *aux) {
    int r = need_init(c);
    if (r) return r;
    if (!aux || ((uintptr_t)aux & 255u)) return fail(c, LBFE_E_INVAL, "aux record null or not 256-byte aligned");
    hipError_t e = launch_step(c->stream, c->p.precision, c->kp, with_aux(c, aux), c->cur, false, true, nullptr);
    if (e != hipSuccess) return hip_fail(c, e, "step_aux");
    c->cur ^= 1;
    c->step++;
    c->aux_ok = false;  // the workspace fields do not describe the new state
    return LBFE_OK;
}

int lbfe_adjoint_step_aux(lbfe_ctx *c, const void *ft, const void *aux) {
    int r = need_bound(c);
    if (r) return r;
    if (!c->p.adjoint) return fail(c, LBFE_E_STATE, "created without params.adjoint = 1");
    if (!c->adj_seeded) return fail(c, LBFE_E_STATE, "adjoint not seeded");
    if (!ft) return fail(c, LBFE_E_INVAL, "null state");
    if (!aux || ((uintptr_t)aux & 255u)) return fail(c, LBFE_E_INVAL, "aux record null or not 256-byte aligned");
    hipError_t e =
        launch_adj_step(c->stream, c->p.precision, c->kp, with_aux(c, aux), c->lcur, ft, false, c->lam_pending);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint_step_aux");
    c->lcur ^= 1;
    c->lam_pending = true;
    return LBFE_OK;
}

int lbfe_adjoint_init_density(lbfe_ctx *c, const double *rho0, const double *u0, double *out) {
    int r = need_bound(c);
    if (r) return r;
    if (!c->p.adjoint) return fail(c, LBFE_E_STATE, "created without params.adjoint = 1");
    if (!c->adj_seeded) return fail(c, LBFE_E_STATE, "adjoint not seeded");
    if (!rho0 || !out) return fail(c, LBFE_E_INVAL, "null rho0 or output");
    if ((r = finalize_lambda(c))) return r;
    c->aux_ok = false;
    hipError_t e = launch_adj_init(c->stream, c->p.precision, c->kp, c->b, c->lcur, rho0, u0, out);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint_init_density");
    return LBFE_OK;
}

int lbfe_adjoint_grads(lbfe_ctx *c, double out[4]) {
    int r = need_bound(c);
    if (r) return r;
    if (!c->p.adjoint) return fail(c, LBFE_E_STATE, "created without params.adjoint = 1");
    if (!out) return fail(c, LBFE_E_INVAL, "null output");
    hipError_t e = hipMemcpyAsync(out, c->b.agrad, 4 * sizeof(double), hipMemcpyDeviceToHost, c->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(c->stream);
    if (e != hipSuccess) return hip_fail(c, e, "adjoint_grads");
    return LBFE_OK;
}

const char *lbfe_last_error(const lbfe_ctx *c) {
    if (!c) return kNoCtx;
    return c->err.c_str();
}

int lbfe_destroy(lbfe_ctx *c) {
    delete c;
    return LBFE_OK;
}

}  // extern "C"
