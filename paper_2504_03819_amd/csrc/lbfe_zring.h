// z-marching LDS ring for 27-point stencils over a few scalar fields: the
// adjoint's transposed stencils and the solid-mask path's FP64 Q stencil.
#pragma once

#include "lbfe_internal.h"

namespace lbfe {
namespace {

// ---------------------------------------------------------------------------
// z-marching stencil tiles.  A workgroup owns a 32 x 16 column tile of one
// z-chunk.  The stencil inputs of four consecutive planes (tile + one-node
// halo) sit in an LDS ring; plane k+2 is loaded into
// registers while plane k is evaluated, so one barrier per plane suffices
// (the slot written at plane k+1 was last read at plane k-2).  Plane indices
// wrap periodically, as in the forward kernels; in a walled box the
// wrapped planes are solid and the fields read there are zero or unused.
// ---------------------------------------------------------------------------
constexpr int ZTX = 32, ZTY = 16, ZWX = ZTX + 2, ZNR = ZWX * (ZTY + 2), ZCB = ZTX * ZTY;
constexpr int ZM = (ZNR + ZCB - 1) / ZCB;  // halo-region points per thread

__device__ inline int zwrap(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

template <int NF> struct ZRing {
    double (*lds)[NF][ZNR];  // [4][NF][ZNR]
    const double *src[NF];
    const float *srcf[NF];  // field f is read from here instead when bit f of fmask is set
    unsigned fmask;
    int a, b, tid, nz;
    bool own;       // the tile point is inside the grid
    unsigned node;  // its in-plane index
    unsigned plane;
    unsigned off[ZM];
    bool has[ZM];
    double pre[NF][ZM];
    unsigned zmask;  // fields zeroed on non-fluid planes (bit f)
    const KP *kp;

    __device__ void init(const KP &k, double (*l)[NF][ZNR], int x0, int y0) {
        kp = &k;
        lds = l;
        tid = threadIdx.x;
        a = tid % ZTX;
        b = tid / ZTX;
        nz = k.nz;
        plane = k.plane;
        own = x0 + a < k.nx && y0 + b < k.ny;
        node = own ? (unsigned)(y0 + b) * k.nx + (x0 + a) : 0u;
        zmask = 0;
        fmask = 0;
#pragma unroll
        for (int m = 0; m < ZM; ++m) {
            const int r = tid + m * ZCB;
            has[m] = r < ZNR;
            const int rr = has[m] ? r : 0;
            off[m] = (unsigned)zwrap(y0 + rr / ZWX - 1, k.ny) * k.nx + zwrap(x0 + rr % ZWX - 1, k.nx);
        }
    }
    __device__ void load(int p) {
        const int zz = zwrap(p, nz);
        const size_t base = (size_t)zz * plane;
        const bool fl = zz >= kp->z0 && zz < kp->z1;
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int m = 0; m < ZM; ++m)
                if (has[m])
                    pre[f][m] = ((zmask >> f) & 1) && !fl ? 0.0
                                : ((fmask >> f) & 1)     ? (double)srcf[f][base + off[m]]
                                                         : src[f][base + off[m]];
    }
    __device__ void commit(int p) {
#pragma unroll
        for (int f = 0; f < NF; ++f)
#pragma unroll
            for (int m = 0; m < ZM; ++m)
                if (has[m]) lds[p & 3][f][tid + m * ZCB] = pre[f][m];
    }
    // field f at (x + dx, y + dy, plane p)
    __device__ double at(int f, int p, int dx, int dy) const { return lds[p & 3][f][(b + 1 + dy) * ZWX + a + 1 + dx]; }
    // planes [zs, ze) of the chunk, body(k) once per plane after the barrier
    template <class Body> __device__ void march(int zs, int ze, Body body) {
        load(zs - 1);
        commit(zs - 1);
        load(zs);
        commit(zs);
        load(zs + 1);
        for (int k = zs; k < ze; ++k) {
            commit(k + 1);
            __syncthreads();
            if (k + 1 < ze) load(k + 2);
            body(k);
        }
    }
};

__device__ inline void ztile(const KP &kp, int cz, int zlo, int zhi, int &x0, int &y0, int &zs, int &ze) {
    const int ntx = (kp.nx + ZTX - 1) / ZTX;
    x0 = (int)(blockIdx.x % ntx) * ZTX;
    y0 = (int)(blockIdx.x / ntx) * ZTY;
    zs = zlo + (int)blockIdx.y * cz;
    ze = min(zs + cz, zhi);
}

// Grid of z-marching kernels over planes [zlo, zhi).
constexpr int kZChunk = 16;
dim3 zgrid(const KP &kp, int zlo, int zhi) {
    const unsigned ntx = (kp.nx + ZTX - 1) / ZTX, nty = (kp.ny + ZTY - 1) / ZTY;
    return dim3(ntx * nty, (unsigned)((zhi - zlo + kZChunk - 1) / kZChunk));
}

}  // namespace
}  // namespace lbfe
