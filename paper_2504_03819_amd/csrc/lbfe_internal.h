// Internal declarations shared by the HIP kernels and the C-ABI host code of
// the D3Q27 free-energy LB library.  Not part of the public interface.
#pragma once

#include <hip/hip_fp16.h>
#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>

#include "lbfe.h"

namespace lbfe {

constexpr int kBlock = 256;  // threads per workgroup (4 wave64s)
// allocation-free reduction: block partials the static scratch holds (up to
// kScratchPartials * kBlock = 2^24 fluid nodes), and the devices it serves
constexpr unsigned kScratchPartials = 1u << 16;
constexpr int kMaxDevices = 64;

// Kernel-side copy of the parameters, passed by value to every kernel.
struct KP {
    int nx, ny, nz;
    unsigned plane;   // nx * ny
    unsigned N;       // nx * ny * nz
    int walls;        // solid planes z = 0 and z = nz-1
    int z0, z1;       // fluid planes [z0, z1)
    unsigned nfluid;  // (z1 - z0) * plane
    double a, b, RT, kappa, nu;
    double om[11];
    int corr4, wet_mode;
    double wet_value, lo, hi;  // wetting value and contact-line window
    int xcd_remap;             // map consecutive tiles onto one XCD
    double wall_u[4];          // (ux, uy) of the bottom and top walls
    int moving;                // some wall velocity is nonzero
    int masked;                // solid voxel mask (Bufs::nbr) instead of planes
    int chain_cz;              // planes per stencil-chain workgroup
};

// Device pointers of one context (all inside the caller's workspace).
struct Bufs {
    void *f[2];          // population lattices (current = f[cur])
    double *rho;         // [N] density (solid planes: Eqs. (37)-(38))
    void *j;             // [3][N] sum_i f_i c_i, compute precision
    double *mu;          // [N] chemical potential (solid: Eq. (36))
    double *mu0;         // [N] bulk part mu0(rho) of mu at fluid nodes
    void *F;             // [3][N] force, compute precision
    void *Q;             // [3][N] Q200, Q020, Q002 of Eq. (27), compute precision, 0 at solid
    unsigned *nbr;       // [N] with a solid mask: bit i set when x + c_i is solid
    void *phi;           // [3][N] phi of Eq. (27) (mask path), compute precision
    int *flag;           // divergence / domain flag
    double *part;        // reduction partials [nblk][8]
    double *red;         // final reductions [8]
    // adjoint
    void *lam[2];        // adjoint populations
    void *abuf;          // adjoint auxiliary fields (see adjoint kernels)
    double *agrad;       // [4] gradient accumulators, then block partials
};

// Launchers (lbfe_kernels.hip).  All enqueue on `s` and return hipError_t.
hipError_t launch_fill(hipStream_t s, void *p, size_t bytes);
hipError_t launch_init(hipStream_t s, int prec, const KP &kp, const Bufs &b, int cur, const double *rho0,
                       const double *u0);
hipError_t launch_aux(hipStream_t s, int prec, const KP &kp, const Bufs &b, int cur);
// One step f[cur] -> f[1 - cur].  fused: chain + fused collide-stream-moments
// (+ wall density), with a moments pass first if `refresh`; otherwise the
// unfused moments, chain, collide-stream.  ev5: optional timing events.
hipError_t launch_step(hipStream_t s, int prec, const KP &kp, const Bufs &b, int cur, bool fused, bool refresh,
                       hipEvent_t *ev5);
// collide + stream + rho, j, mu0 of the streamed state (lbfe_fused.hip);
// fused_plane_ok: one z-plane of the lattice fits its 32-bit plane offsets
hipError_t launch_fused(hipStream_t s, int prec, const KP &kp, const Bufs &b, int cur);
bool fused_plane_ok(int prec, size_t plane);
// Moment-representation state (lbfe_moment.hip), for unit rates but omega_1:
// passes over a state lattice `sin` (16 values per node): kStateMoments forms
// rho, j, mu0 of the streamed state, kStatePops also writes its populations
// to the lattice `out`, kStateCollide collides the streamed state with the
// current mu, F, Q and writes the new state to `out`; launch_state_first
// collides the populations `fin` into the state lattice `sout`.  FP64 and
// FP32 only (hipErrorInvalidValue otherwise).  state_plane_ok: one z-plane of
// either lattice fits its 32-bit plane offsets.
enum StateMode { kStateMoments = 0, kStatePops = 1, kStateCollide = 2 };
hipError_t launch_state_pass(hipStream_t s, int prec, int mode, const KP &kp, const Bufs &b, const void *sin,
                             void *out);
hipError_t launch_state_first(hipStream_t s, int prec, const KP &kp, const Bufs &b, const void *fin, void *sout);
bool state_plane_ok(int prec, size_t plane);
// The state form's launch groups (lbfe_kernels.hip); ev, when non-null,
// receives events at the start, after the chain (enter, collide) and at the
// end.  enter: [moments of f[cur] if refresh], chain, f[cur] collided into
// the state lattice f[1 - cur].  moments: rho, j, mu0 (and with `pops` the
// populations, into f[1 - a]) of the state f[a], wall densities.  collide:
// chain, then the state f[a] stepped into f[1 - a].
hipError_t launch_state_enter(hipStream_t s, int prec, const KP &kp, const Bufs &b, int cur, bool refresh,
                              hipEvent_t *ev);
hipError_t launch_state_moments(hipStream_t s, int prec, const KP &kp, const Bufs &b, int a, bool pops,
                                hipEvent_t *ev);
hipError_t launch_state_collide(hipStream_t s, int prec, const KP &kp, const Bufs &b, int a, hipEvent_t *ev);
// mu, F and Q of the current rho, j (lbfe_chain.hip); chain_chunk_for: the
// planes per workgroup, kp.chain_cz if set, else chosen for the grid
hipError_t launch_chain(hipStream_t s, int prec, const KP &kp, const Bufs &b);
int chain_chunk_for(const KP &kp);
hipError_t launch_export(hipStream_t s, int prec, const KP &kp, const Bufs &b, int which, double *out);
hipError_t launch_reduce(hipStream_t s, int prec, const KP &kp, const Bufs &b);
// the same reduction with the block partials in `part` (the static scratch
// of lbfe_kernels.hip, from scratch_partials on the current device) and the
// 8 results to `out`; hipErrorInvalidValue beyond kScratchPartials blocks
hipError_t scratch_partials(int device, double **out);
hipError_t launch_reduce_into(hipStream_t s, int prec, const KP &kp, const Bufs &b, double *part, double *out);
hipError_t launch_get_pop(hipStream_t s, int prec, const KP &kp, const Bufs &b, const void *f, double *out);
hipError_t launch_set_pop(hipStream_t s, int prec, const KP &kp, const Bufs &b, void *f, const double *in);
hipError_t launch_check_rho0(hipStream_t s, const KP &kp, const double *rho0, int *flag);
// rho0 (fluid nodes) -> rho with wall densities -> mu, as in the initialiser
hipError_t launch_init_aux(hipStream_t s, const KP &kp, const Bufs &b, const double *rho0);

// solid voxel masks (lbfe_mask.hip): neighbour words from a uint8 mask, and
// the mask path's aux fields, step, initialiser and rho0 check
hipError_t launch_mask_prep(hipStream_t s, const KP &kp, const Bufs &b, const uint8_t *solid);
hipError_t launch_aux_mask(hipStream_t s, int prec, const KP &kp, const Bufs &b, int cur);
hipError_t launch_step_mask(hipStream_t s, int prec, const KP &kp, const Bufs &b, int cur, hipEvent_t *ev5);
hipError_t launch_init_mask(hipStream_t s, int prec, const KP &kp, const Bufs &b, int cur, const double *rho0,
                            const double *u0);
hipError_t launch_check_rho0_mask(hipStream_t s, const KP &kp, const Bufs &b, const double *rho0, int *flag);
hipError_t launch_init_aux_mask(hipStream_t s, const KP &kp, const Bufs &b, const double *rho0);

// adjoint (lbfe_adjoint.hip)
size_t adjoint_aux_bytes(int prec, size_t N);
size_t adjoint_grad_slots();
hipError_t launch_adj_seed(hipStream_t s, int prec, const KP &kp, const Bufs &b, int lcur, const double *dLdrho);
hipError_t launch_adj_seed_pop(hipStream_t s, int prec, const KP &kp, const Bufs &b, int lcur, const double *lam);
hipError_t launch_adj_get(hipStream_t s, int prec, const KP &kp, const Bufs &b, int lcur, double *out);
// recompute: evaluate the forward fields of ft first (else b holds them);
// pending: lam[lcur] holds only the direct part of lambda(t+1).  Leaves
// lam[1 - lcur] as the direct part of lambda(t), its last term pending.
hipError_t launch_adj_step(hipStream_t s, int prec, const KP &kp, const Bufs &b, int lcur, const void *ft,
                           bool recompute, bool pending);
// applies the pending last term to lam[lcur] in place
hipError_t launch_adj_finalize(hipStream_t s, int prec, const KP &kp, const Bufs &b, int lcur);
hipError_t launch_adj_init(hipStream_t s, int prec, const KP &kp, const Bufs &b, int lcur, const double *rho0,
                           const double *u0, double *out);

inline unsigned nblocks(size_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// Byte sizes per precision
inline size_t real_bytes(int prec) { return prec == LBFE_FP64 ? 8 : 4; }
inline size_t pop_bytes(int prec, size_t N) {
    switch (prec) {
        case LBFE_FP64: return 27 * 8 * N;
        case LBFE_FP32: return 27 * 4 * N;
        case LBFE_FP16_DEV: return 27 * 2 * N;
        default: {  // 26 half planes, then one float plane (256-byte aligned)
            size_t h = (26 * 2 * N + 255) & ~size_t(255);
            return h + 4 * N;
        }
    }
}
inline size_t lambda_bytes(int prec, size_t N) { return 27 * real_bytes(prec) * N; }

}  // namespace lbfe
