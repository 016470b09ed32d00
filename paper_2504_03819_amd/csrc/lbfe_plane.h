// Plane-wise buffer access and LDS planes shared by the z-marching
// collide-stream kernels (lbfe_fused.hip, lbfe_moment.hip): raw buffer
// descriptors for one z-plane of a row-blocked lattice or of a [z][y][x]
// field, the storage encoding of a population value, one LDS plane of
// post-collision populations, and the tile geometry.
#pragma once

#include "lbfe_device.h"

namespace lbfe {
namespace plane {

// Raw buffer access to one z-plane of a row-blocked lattice or of a [z][y][x]
// field: the plane's base goes into a buffer descriptor (scalar registers),
// every access takes a 32-bit per-lane byte offset plus a uniform slot
// offset, so the 27 population addresses of a node cost no vector
// registers.  A lane with offset kOOB (past the plane) reads 0 and stores
// nothing.
typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
constexpr unsigned kOOB = 0x80000000u;
constexpr int kPopStore = 2;  // population stores non-temporal (read only by the next step)
__device__ inline __amdgpu_buffer_rsrc_t rsrc(const void *base, unsigned bytes) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void *>(base), 0, (int)bytes, 0x00020000);
}
__device__ inline double bld(double *, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, v, s, 0));
}
__device__ inline float bld(float *, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, v, s, 0));
}
__device__ inline __half bld(__half *, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    return __builtin_bit_cast(__half, __builtin_amdgcn_raw_buffer_load_b16(r, v, s, 0));
}
template <int POL = 0> __device__ inline void bst(double x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b64(__builtin_bit_cast(u32x2, x), r, v, s, POL);
}
template <int POL = 0> __device__ inline void bst(float x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b32(__builtin_bit_cast(unsigned, x), r, v, s, POL);
}
template <int POL = 0> __device__ inline void bst(__half x, __amdgpu_buffer_rsrc_t r, unsigned v, unsigned s) {
    __builtin_amdgcn_raw_buffer_store_b16(__builtin_bit_cast(unsigned short, x), r, v, s, POL);
}

// Storage encoding of one population value (a store then a load of the
// lattice returns dec(enc(v))) and the plane geometry of the row-blocked
// lattice: NS slots of nx values per x-row, S bytes each; with f0 in FP32 the
// rest population lives in a float [z][y][x] array after the half rows.
template <int P> struct Code {
    using st = float;
    static constexpr unsigned S = 4, NS = 27;
    __device__ static st enc(int, float v) { return v; }
    __device__ static float dec(int, st v) { return v; }
    __device__ static int slot(int i) { return i; }
};
template <> struct Code<LBFE_FP64> {
    using st = double;
    static constexpr unsigned S = 8, NS = 27;
    __device__ static st enc(int, double v) { return v; }
    __device__ static double dec(int, st v) { return v; }
    __device__ static int slot(int i) { return i; }
};
template <> struct Code<LBFE_FP16_DEV> {
    using st = __half;
    static constexpr unsigned S = 2, NS = 27;
    __device__ static st enc(int i, float v) { return enc16(i, v); }
    __device__ static float dec(int i, st v) { return dec16(i, v); }
    __device__ static int slot(int i) { return i; }
};
template <> struct Code<LBFE_FP16_DEV_F0FP32> {
    using st = __half;
    static constexpr unsigned S = 2, NS = 26;
    __device__ static st enc(int i, float v) { return enc16(i, v); }
    __device__ static float dec(int i, st v) { return dec16(i, v); }
    __device__ static int slot(int i) { return i < kRest ? i : i - 1; }
};

// One z-plane of a lattice: the half / real rows and, with f0 in FP32, the
// rest-population plane.
template <int P> struct LatPlane {
    using C = Code<P>;
    __amdgpu_buffer_rsrc_t r, r0;
    unsigned nxS;  // bytes per slot run
    __device__ LatPlane(const void *base, const KP &kp, int z) {
        const size_t rows = (size_t)C::NS * C::S * kp.plane;  // bytes of one plane's rows
        nxS = (unsigned)kp.nx * C::S;
        r = rsrc((const char *)base + (size_t)z * rows, (unsigned)rows);
        if constexpr (P == LBFE_FP16_DEV_F0FP32) {
            const size_t h = (26 * 2 * (size_t)kp.N + 255) & ~size_t(255);
            r0 = rsrc((const char *)base + h + (size_t)z * 4 * kp.plane, 4u * kp.plane);
        } else {
            r0 = r;
        }
    }
    // vo: byte offset of the node's row position, (y NS nx + x) S; vo0: of
    // the node in the rest-population plane, (y nx + x) 4
    __device__ typename Pol<P>::real ld(int i, unsigned vo, unsigned vo0) const {
        if constexpr (P == LBFE_FP16_DEV_F0FP32) {
            if (i == kRest) return bld((float *)nullptr, r0, vo0, 0);
        }
        return C::dec(i, bld((typename C::st *)nullptr, r, vo, (unsigned)C::slot(i) * nxS));
    }
};

// One LDS plane of post-collision values in their storage encoding.  With
// f0 in FP32 the rest population sits in a float array of its own.
template <int P, int NR> struct Plane {
    using C = Code<P>;
    using real = typename Pol<P>::real;
    typename C::st v[27][NR];
    __device__ void put(int i, int k, real x) { v[i][k] = C::enc(i, x); }
    __device__ real get(int i, int k) const { return C::dec(i, v[i][k]); }
    // raw encoded value i of LDS node k to slot `slot` of the lattice node
    // at byte offsets (vo, vo0) of plane L
    __device__ void store(const LatPlane<P> &L, int slot, int i, int k, unsigned vo, unsigned) const {
        bst<kPopStore>(v[i][k], L.r, vo, (unsigned)slot * L.nxS);
    }
};
template <int NR> struct Plane<LBFE_FP16_DEV_F0FP32, NR> {
    using C = Code<LBFE_FP16_DEV_F0FP32>;
    __half v[27][NR];  // slot kRest unused
    float r0[NR];
    __device__ void put(int i, int k, float x) {
        if (i == kRest)
            r0[k] = x;
        else
            v[i][k] = enc16(i, x);
    }
    __device__ float get(int i, int k) const { return i == kRest ? r0[k] : dec16(i, v[i][k]); }
    __device__ void store(const LatPlane<LBFE_FP16_DEV_F0FP32> &L, int slot, int i, int k, unsigned vo,
                          unsigned vo0) const {
        if (i == kRest)  // the rest population never changes slot
            bst<kPopStore>(r0[k], L.r0, vo0, 0);
        else
            bst<kPopStore>(v[i][k], L.r, vo, (unsigned)C::slot(slot) * L.nxS);
    }
};

__device__ inline int wrapi(int v, int n) {
    v %= n;
    return v < 0 ? v + n : v;
}

struct Acc {  // partial moments of one destination plane
    double r, jx, jy, lp;
};

// Tile origin and z-range [zs, ze) of this workgroup.  The grid is (tiles,
// chunks); tiles are dealt to the XCDs in contiguous ranges (consecutive
// tiles, which share ring columns, on one XCD), all tiles of a chunk
// together.
struct Chunk {
    int x0, y0, zs, ze;
};
template <int TX, int TY> __device__ inline Chunk chunk_of(const KP &kp, int cz) {
    const int ntx = (kp.nx + TX - 1) / TX;
    const unsigned ntiles = gridDim.x, nb = gridDim.x * gridDim.y;
    const unsigned hw = blockIdx.y * gridDim.x + blockIdx.x;
    const unsigned qq = nb >> 3, rem = nb & 7u, xcd = hw & 7u;
    const unsigned lid = xcd * qq + (xcd < rem ? xcd : rem) + (hw >> 3);
    const int tile = (int)(lid % ntiles), chunk = (int)(lid / ntiles);
    Chunk c;
    c.x0 = (tile % ntx) * TX;
    c.y0 = (tile / ntx) * TY;
    c.zs = kp.z0 + chunk * cz;
    c.ze = min(c.zs + cz, kp.z1);
    return c;
}

// Planes per workgroup: long chunks amortise the two ring planes; enough
// workgroups to give every CU one.
inline int chunk_planes(const KP &kp, unsigned tiles) {
    const int nzf = kp.z1 - kp.z0;
    int cz = 64;
    while (cz > 8 && (size_t)tiles * ((nzf + cz - 1) / cz) < 256) cz /= 2;
    return cz;
}

template <int TX, int TY, int NT> struct Geo {
    static constexpr int WX = TX + 2, WY = TY + 2, NR = WX * WY;
    static_assert(NR <= NT, "one lane per ring-inclusive node");
    static_assert(TX * TY % 64 == 0, "owned columns fill whole waves");
};

}  // namespace plane
}  // namespace lbfe
