// Device-side access to the AA-pattern population store: natural and swapped
// layout readers with the boundary rules, odd-step writers, the per-cell
// force and the macroscopic fields of one cell. Shared by the lattice and
// actuator-line kernels.
#pragma once
#include "lbm_device.h"
#include "lbm_internal.h"

namespace lbm {

__device__ __forceinline__ int wrapi(int v, int n) { return v < 0 ? v + n : (v >= n ? v - n : v); }

__device__ __forceinline__ size_t cidx(const Geo &g, int x, int y, int z) {
    return ((size_t)z * g.ny + y) * g.nx + x;
}

// Blocked population layout: the x rows are cut into blocks of W cells, and
// a block keeps its 27 directions one after the other, W values each:
// store[z][y][x / W][i][x % W] (rows padded to g.nbx whole blocks), W =
// blk_width(element size). A wave of 64 cells of one row then reads and
// writes one or two contiguous 27 W regions in an even step, instead of 27
// streams spread over the whole store.
template <typename T>
struct Blk {
    static constexpr int W = blk_width((int)sizeof(T));
    static constexpr int LOG = W == 32 ? 5 : (W == 64 ? 6 : 7);
    static constexpr int SLOTS = 27 * W;
    static_assert((1 << LOG) == W, "power-of-two block width");
};
template <typename T>
__device__ __forceinline__ size_t slot_idx(const Geo &g, int i, int x, int y, int z) {
    return (((size_t)z * g.ny + y) * g.nbx + (size_t)(x >> Blk<T>::LOG)) * Blk<T>::SLOTS +
           (size_t)(i * Blk<T>::W + (x & (Blk<T>::W - 1)));
}
// element offset of cell x's slot 0 within its row of blocks
template <typename T>
__device__ __forceinline__ uint32_t row_xpart(int x) {
    return (uint32_t)(x >> Blk<T>::LOG) * (uint32_t)Blk<T>::SLOTS + (uint32_t)(x & (Blk<T>::W - 1));
}

__device__ __forceinline__ float phi1(int c, float u) {
    return c == 0 ? (2.0f / 3.0f - u * u) : 0.5f * (1.0f / 3.0f + u * u + c * u);
}

// f_eq_i(1, u_in(y,z)) - w_i for the inlet, from the given inlet plane
__device__ __forceinline__ float inlet_dev(const Geo &g, const float *uin, int i, int y, int z) {
    const int q = y + g.ny * z, pl = g.ny * g.nz;
    const float ux = uin[q], uy = uin[pl + q], uz = uin[2 * pl + q];
    return phi1(cx_of(i), ux) * phi1(cy_of(i), uy) * phi1(cz_of(i), uz) - wgt(i);
}

// Pre-collision deviation of direction I at (x,y,z) from the swapped layout.
template <typename T, int I>
__device__ __forceinline__ float read_swapped(const Geo &g, int x, int y, int z) {
    constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I), RI = refl_z(I);
    const T *pops = (const T *)g.pops;
    int sx = x - cx, sy = y - cy, sz = z - cz;
    bool refl = false;
    if (cz != 0 && (sz < 0 || sz >= g.nz)) {
        const int bc = sz < 0 ? g.bc_zlo : g.bc_zhi;
        if (bc == BC_NOSLIP) return Store<T>::ld(pops + slot_idx<T>(g, I, x, y, z));
        if (bc == BC_FREESLIP) {
            refl = true;
            sz = z;
        } else {
            sz = wrapi(sz, g.nz);
        }
    }
    sy = wrapi(sy, g.ny);
    const int ii = refl ? RI : I;
    if (cx != 0 && (sx < 0 || sx >= g.nx)) {
        if (g.bc_x == BC_PERIODIC) {
            sx = wrapi(sx, g.nx);
        } else if (sx < 0) {
            return inlet_dev(g, g.uin_rd, ii, sy, sz);
        } else {
            const T *G = (const T *)g.ghost;
            return Store<T>::ld(G + (size_t)(ii / 3) * g.ny * g.nz + sy + (size_t)g.ny * sz);
        }
    }
    return Store<T>::ld(pops + slot_idx<T>(g, 26 - ii, sx, sy, sz));
}

// Odd-step push of the post-collision deviation of direction I.
template <typename T, int I>
__device__ __forceinline__ void write_odd(const Geo &g, int x, int y, int z, float v) {
    constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I), RI = refl_z(I);
    T *pops = (T *)g.pops;
    int tx = x + cx, ty = y + cy, tz = z + cz;
    bool refl = false;
    if (cz != 0 && (tz < 0 || tz >= g.nz)) {
        const int bc = tz < 0 ? g.bc_zlo : g.bc_zhi;
        if (bc == BC_NOSLIP) {
            Store<T>::st(pops + slot_idx<T>(g, 26 - I, x, y, z), v);
            return;
        }
        if (bc == BC_FREESLIP) {
            refl = true;
            tz = z;
        } else {
            tz = wrapi(tz, g.nz);
        }
    }
    ty = wrapi(ty, g.ny);
    if (cx != 0 && (tx < 0 || tx >= g.nx)) {
        if (g.bc_x != BC_PERIODIC) return;
        tx = wrapi(tx, g.nx);
    }
    Store<T>::st(pops + slot_idx<T>(g, refl ? RI : I, tx, ty, tz), v);
}

// Force on a cell: uniform part + optional dense field + rotor boxes.
__device__ __forceinline__ void cell_force(const Physics &ph, size_t n, size_t cell, int x, int y, int z,
                                           float &Fx, float &Fy, float &Fz) {
    Fx = ph.bf[0];
    Fy = ph.bf[1];
    Fz = ph.bf[2];
    if (ph.ffield) {
        Fx += ph.ffield[cell];
        Fy += ph.ffield[n + cell];
        Fz += ph.ffield[2 * n + cell];
    }
    for (int b = 0; b < ph.nbox; ++b) {
        const ForceBox &B = ph.box[b];
        const int lx = x - B.x0, ly = y - B.y0, lz = z - B.z0;
        if ((unsigned)lx < (unsigned)B.bnx && (unsigned)ly < (unsigned)B.bny && (unsigned)lz < (unsigned)B.bnz) {
            const size_t nb = (size_t)B.bnx * B.bny * B.bnz;
            const size_t q = (size_t)lx + (size_t)B.bnx * ((size_t)ly + (size_t)B.bny * lz);
            Fx += B.F[q];
            Fy += B.F[nb + q];
            Fz += B.F[2 * nb + q];
        }
    }
}

template <int CL>
__device__ __forceinline__ float omega1_of(const CellMoments &m, const Physics &ph) {
    if (CL == CL_SMAG) return smag_omega(q_norm(m), ph.tau0, ph.smag_c);
    return ph.omega;
}

template <typename T, int I>
struct Unroll {
    // load/store helpers unrolled over the 27 directions at compile time;
    // s0 is the element index of the cell's slot 0 (slot_idx<T>(g, 0, x, y, z))
    static __device__ __forceinline__ void read_natural(const Geo &g, size_t s0, float *d) {
        d[I] = Store<T>::ld((const T *)g.pops + s0 + I * Blk<T>::W);
        Unroll<T, I + 1>::read_natural(g, s0, d);
    }
    static __device__ __forceinline__ void read_sw(const Geo &g, int x, int y, int z, float *d) {
        d[I] = read_swapped<T, I>(g, x, y, z);
        Unroll<T, I + 1>::read_sw(g, x, y, z, d);
    }
    static __device__ __forceinline__ void write_swap_local(const Geo &g, size_t s0, const float *o) {
        Store<T>::st((T *)g.pops + s0 + (26 - I) * Blk<T>::W, o[I]);
        Unroll<T, I + 1>::write_swap_local(g, s0, o);
    }
    static __device__ __forceinline__ void write_push(const Geo &g, int x, int y, int z, const float *o) {
        write_odd<T, I>(g, x, y, z, o[I]);
        Unroll<T, I + 1>::write_push(g, x, y, z, o);
    }
};
template <typename T>
struct Unroll<T, 27> {
    static __device__ __forceinline__ void read_natural(const Geo &, size_t, float *) {}
    static __device__ __forceinline__ void read_sw(const Geo &, int, int, int, float *) {}
    static __device__ __forceinline__ void write_swap_local(const Geo &, size_t, const float *) {}
    static __device__ __forceinline__ void write_push(const Geo &, int, int, int, const float *) {}
};

// Fast path (no boundary rules in the addressing): a tile lies in one z
// plane, so the bases of the z planes z - 1, z, z + 1 are uniform across the
// workgroup (scalar registers) and every access is one global load or store
// with that base, a 32-bit lane offset and the direction's slot as the
// constant offset. Nbr holds, for cell (x, y, z), the element offsets within
// a z plane of the rows y - 1, y, y + 1 (ys) and of the cells x - 1, x, x + 1
// within a row (xo), wrapped periodically, and the element bases of the z
// planes z - 1, z, z + 1 (zb), wrapped. Valid while a z plane of blocks has
// fewer than 2^32 bytes (checked on the host).
struct Nbr {
    uint32_t ys[3], xo[3];
    size_t zb[3];
};
template <typename T>
__device__ __forceinline__ void fast_nbr(const Geo &g, int x, int y, int z, Nbr &n) {
    const int xm = x == 0 ? g.nx - 1 : x - 1, xp = x == g.nx - 1 ? 0 : x + 1;
    n.xo[0] = row_xpart<T>(xm);
    n.xo[1] = row_xpart<T>(x);
    n.xo[2] = row_xpart<T>(xp);
    const uint32_t rowlen = (uint32_t)g.nbx * (uint32_t)Blk<T>::SLOTS, yr = (uint32_t)y * rowlen;
    n.ys[0] = y == 0 ? (uint32_t)(g.ny - 1) * rowlen : yr - rowlen;
    n.ys[1] = yr;
    n.ys[2] = y == g.ny - 1 ? 0u : yr + rowlen;
    const size_t zplane = (size_t)g.ny * rowlen;
    n.zb[0] = (size_t)(z == 0 ? g.nz - 1 : z - 1) * zplane;
    n.zb[1] = (size_t)z * zplane;
    n.zb[2] = (size_t)(z == g.nz - 1 ? 0 : z + 1) * zplane;
}
// FP32 storage addresses every fast-path access with a per-lane 64-bit
// address (global_load v, v[a:b], off) instead of the scalar base + 32-bit
// offset form, which 16-bit storage keeps.
typedef __attribute__((address_space(1))) float global_f32;
__device__ __forceinline__ global_f32 *lane_f32(const void *p) {
    uint64_t a = (uint64_t)p;
    asm volatile("" : "+v"(a));  // keep the sum per lane (the compiler would fold it back to a scalar base)
    return (global_f32 *)a;
}
// slot i of the cell at (x + dx, y + dy, z + dz), dx, dy, dz in {-1, 0, 1}
template <typename T>
__device__ __forceinline__ float ld_nbr(const Geo &g, const Nbr &n, int dx, int dy, int dz, int i) {
    const char *plane = (const char *)g.pops + n.zb[dz + 1] * sizeof(T) + (size_t)i * Blk<T>::W * sizeof(T);
    const char *p = plane + (n.ys[dy + 1] + n.xo[dx + 1]) * (uint32_t)sizeof(T);
    if constexpr (sizeof(T) == 4) return *lane_f32(p);
    else return Store<T>::ld((const T *)p);
}
template <typename T>
__device__ __forceinline__ void st_nbr(const Geo &g, const Nbr &n, int dx, int dy, int dz, int i, float v) {
    char *plane = (char *)g.pops + n.zb[dz + 1] * sizeof(T) + (size_t)i * Blk<T>::W * sizeof(T);
    char *p = plane + (n.ys[dy + 1] + n.xo[dx + 1]) * (uint32_t)sizeof(T);
    if constexpr (sizeof(T) == 4) *lane_f32(p) = v;
    else Store<T>::st((T *)p, v);
}
// slot i of the cell itself (the even step), every storage type in the
// scalar-base form: one scalar base per direction and the lane's 32-bit
// offset. For FP32 the base is made opaque (empty asm on a scalar register
// pair), so that each direction keeps a scalar base of its own: left alone the
// compiler shares one base and puts the directions' distances (i * 128 bytes)
// in the instructions' immediate offsets, which measured 0.6 % slower per
// step at 512^3.
// The cell's z, and so the base, must be the same across the wave (one z
// plane per workgroup, as in the stream-collide tiles).
template <typename T>
__device__ __forceinline__ const char *own_plane(const Geo &g, const Nbr &n, int i) {
    return (const char *)g.pops + n.zb[1] * sizeof(T) + (size_t)i * Blk<T>::W * sizeof(T);
}
template <typename T>
__device__ __forceinline__ float ld_own(const Geo &g, const Nbr &n, int i) {
    const uint32_t off = (n.ys[1] + n.xo[1]) * (uint32_t)sizeof(T);
    if constexpr (sizeof(T) == 4) {
        uint64_t b = (uint64_t)own_plane<T>(g, n, i);
        asm volatile("" : "+s"(b));
        return *(const global_f32 *)((b + off));
    } else {
        return Store<T>::ld((const T *)(own_plane<T>(g, n, i) + off));
    }
}
template <typename T>
__device__ __forceinline__ void st_own(const Geo &g, const Nbr &n, int i, float v) {
    const uint32_t off = (n.ys[1] + n.xo[1]) * (uint32_t)sizeof(T);
    if constexpr (sizeof(T) == 4) {
        uint64_t b = (uint64_t)own_plane<T>(g, n, i);
        asm volatile("" : "+s"(b));
        *(global_f32 *)(b + off) = v;
    } else {
        Store<T>::st((T *)(own_plane<T>(g, n, i) + off), v);
    }
}

template <typename T, int I>
struct Unroll32 {
    // even step: the cell's own slots
    static __device__ __forceinline__ void read_natural(const Geo &g, const Nbr &n, float *d) {
        d[I] = ld_own<T>(g, n, I);
        Unroll32<T, I + 1>::read_natural(g, n, d);
    }
    static __device__ __forceinline__ void write_swap_local(const Geo &g, const Nbr &n, const float *o) {
        st_own<T>(g, n, 26 - I, o[I]);
        Unroll32<T, I + 1>::write_swap_local(g, n, o);
    }
    // odd step: slot 26 - I of x - c_I, and the push into slot I of x + c_I
    static __device__ __forceinline__ void read_periodic(const Geo &g, const Nbr &n, float *d) {
        d[I] = ld_nbr<T>(g, n, -cx_of(I), -cy_of(I), -cz_of(I), 26 - I);
        Unroll32<T, I + 1>::read_periodic(g, n, d);
    }
    static __device__ __forceinline__ void write_periodic(const Geo &g, const Nbr &n, const float *o) {
        st_nbr<T>(g, n, cx_of(I), cy_of(I), cz_of(I), I, o[I]);
        Unroll32<T, I + 1>::write_periodic(g, n, o);
    }
    // the nine directions with c_x = CX only
    template <int CX>
    static __device__ __forceinline__ void write_periodic_cx(const Geo &g, const Nbr &n, const float *o) {
        if constexpr (cx_of(I) == CX) st_nbr<T>(g, n, cx_of(I), cy_of(I), cz_of(I), I, o[I]);
        Unroll32<T, I + 1>::template write_periodic_cx<CX>(g, n, o);
    }
};
template <typename T>
struct Unroll32<T, 27> {
    static __device__ __forceinline__ void read_natural(const Geo &, const Nbr &, float *) {}
    static __device__ __forceinline__ void write_swap_local(const Geo &, const Nbr &, const float *) {}
    static __device__ __forceinline__ void read_periodic(const Geo &, const Nbr &, float *) {}
    static __device__ __forceinline__ void write_periodic(const Geo &, const Nbr &, const float *) {}
    template <int CX>
    static __device__ __forceinline__ void write_periodic_cx(const Geo &, const Nbr &, const float *) {}
};

// ------------------------------------------------------------ readers
// A swapped-layout read of cell (x, y, z) needs no boundary rule when none of
// its 26 neighbours lies across an open x face or a z wall; it is then the
// fast path's periodic-wrap read (valid while a z plane of blocks has fewer
// than 2^32 bytes), whose 27 loads are independent of each other.
template <typename T>
__device__ __forceinline__ bool swapped_read_is_plain(const Geo &g, int x, int z) {
    const bool fits = (size_t)g.ny * (size_t)g.nbx * Blk<T>::SLOTS * sizeof(T) < ((size_t)1 << 32);
    const bool xin = g.bc_x == BC_PERIODIC || (x > 0 && x < g.nx - 1);
    const bool zlo = g.bc_zlo == BC_NOSLIP || g.bc_zlo == BC_FREESLIP;
    const bool zhi = g.bc_zhi == BC_NOSLIP || g.bc_zhi == BC_FREESLIP;
    return fits && xin && (!zlo || z > 0) && (!zhi || z < g.nz - 1);
}

template <typename T, int PAR>
__device__ __forceinline__ void read_cell(const Geo &g, size_t cell, int x, int y, int z, float *d) {
    if (PAR == 0) {
        Unroll<T, 0>::read_natural(g, slot_idx<T>(g, 0, x, y, z), d);
    } else if (swapped_read_is_plain<T>(g, x, z)) {
        Nbr n;
        fast_nbr<T>(g, x, y, z, n);
        Unroll32<T, 0>::read_periodic(g, n, d);
    } else {
        Unroll<T, 0>::read_sw(g, x, y, z, d);
    }
}

// rho, j (FP64 sums of the stored deviations) and u with half the force
template <typename T, int PAR>
__device__ __forceinline__ void cell_macro(const Geo &g, const Physics &ph, size_t cell, int x, int y, int z,
                                           double &rho, double &ux, double &uy, double &uz) {
    float d[27];
    read_cell<T, PAR>(g, cell, x, y, z, d);
    double r = 0, jx = 0, jy = 0, jz = 0;
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        r += d[i];
        jx += cx_of(i) * (double)d[i];
        jy += cy_of(i) * (double)d[i];
        jz += cz_of(i) * (double)d[i];
    }
    float Fx, Fy, Fz;
    cell_force(ph, (size_t)g.nx * g.ny * g.nz, cell, x, y, z, Fx, Fy, Fz);
    rho = 1.0 + r;
    ux = (jx + 0.5 * Fx) / rho;
    uy = (jy + 0.5 * Fy) / rho;
    uz = (jz + 0.5 * Fz) / rho;
}

}  // namespace lbm
