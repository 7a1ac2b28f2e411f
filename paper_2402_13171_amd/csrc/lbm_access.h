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
        if (bc == BC_NOSLIP) return Store<T>::ld(pops + (size_t)I * g.P + cidx(g, x, y, z));
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
    return Store<T>::ld(pops + (size_t)(26 - ii) * g.P + cidx(g, sx, sy, sz));
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
            Store<T>::st(pops + (size_t)(26 - I) * g.P + cidx(g, x, y, z), v);
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
    Store<T>::st(pops + (size_t)(refl ? RI : I) * g.P + cidx(g, tx, ty, tz), v);
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
    // load/store helpers unrolled over the 27 directions at compile time
    static __device__ __forceinline__ void read_natural(const Geo &g, size_t cell, float *d) {
        d[I] = Store<T>::ld((const T *)g.pops + (size_t)I * g.P + cell);
        Unroll<T, I + 1>::read_natural(g, cell, d);
    }
    static __device__ __forceinline__ void read_sw(const Geo &g, int x, int y, int z, float *d) {
        d[I] = read_swapped<T, I>(g, x, y, z);
        Unroll<T, I + 1>::read_sw(g, x, y, z, d);
    }
    static __device__ __forceinline__ void write_swap_local(const Geo &g, size_t cell, const float *o) {
        Store<T>::st((T *)g.pops + (size_t)(26 - I) * g.P + cell, o[I]);
        Unroll<T, I + 1>::write_swap_local(g, cell, o);
    }
    static __device__ __forceinline__ void write_push(const Geo &g, int x, int y, int z, const float *o) {
        write_odd<T, I>(g, x, y, z, o[I]);
        Unroll<T, I + 1>::write_push(g, x, y, z, o);
    }
    // periodic fast paths: row offsets for dy,dz in {-1,0,1}
    static __device__ __forceinline__ void read_periodic(const Geo &g, const int *xs, const size_t *rows, float *d) {
        constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I);
        // source x - c: xs[1 - cx], rows[(1 - cy) + 3 (1 - cz)]
        d[I] = Store<T>::ld((const T *)g.pops + (size_t)(26 - I) * g.P + rows[(1 - cy) + 3 * (1 - cz)] + xs[1 - cx]);
        Unroll<T, I + 1>::read_periodic(g, xs, rows, d);
    }
    static __device__ __forceinline__ void write_periodic(const Geo &g, const int *xs, const size_t *rows, const float *o) {
        constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I);
        Store<T>::st((T *)g.pops + (size_t)I * g.P + rows[(1 + cy) + 3 * (1 + cz)] + xs[1 + cx], o[I]);
        Unroll<T, I + 1>::write_periodic(g, xs, rows, o);
    }
};
// Fast-path variants with 32-bit byte offsets from per-plane base pointers:
// the plane base is uniform across the wave (scalar registers), so each access
// is one global load/store with a 32-bit vector offset. Valid while
// n * sizeof(T) < 2^32 (checked on the host, which otherwise uses the
// 64-bit general path).
// FP32 storage addresses every access with a per-lane 64-bit address instead
// (global_load v, v[a:b], off): on MI355X the 27-plane pattern of a 512^3
// step moved about 2 % more bytes per second that way, for the stream-collide
// kernel and a bare copy of its accesses alike; with 16-bit storage the
// scalar-base form was the faster one (by about 1.5 %) and stays.
typedef __attribute__((address_space(1))) float global_f32;
__device__ __forceinline__ global_f32 *lane_addr_f32(const Geo &g, int i, uint32_t boff) {
    uint64_t a = (uint64_t)((float *)g.pops + ((size_t)i * g.P + (size_t)(boff / 4u)));
    asm volatile("" : "+v"(a));  // keep the sum per lane (the compiler would fold it back to a scalar base)
    return (global_f32 *)a;
}
template <typename T>
__device__ __forceinline__ float ld_plane(const Geo &g, int i, uint32_t boff) {
    if constexpr (sizeof(T) == 4) return *lane_addr_f32(g, i, boff);
    else return Store<T>::ld((const T *)((const char *)g.pops + (size_t)i * g.P * sizeof(T) + boff));
}
template <typename T>
__device__ __forceinline__ void st_plane(const Geo &g, int i, uint32_t boff, float v) {
    if constexpr (sizeof(T) == 4) *lane_addr_f32(g, i, boff) = v;
    else Store<T>::st((T *)((char *)g.pops + (size_t)i * g.P * sizeof(T) + boff), v);
}

template <typename T, int I>
struct Unroll32 {
    static __device__ __forceinline__ void read_natural(const Geo &g, uint32_t boff, float *d) {
        d[I] = ld_plane<T>(g, I, boff);
        Unroll32<T, I + 1>::read_natural(g, boff, d);
    }
    static __device__ __forceinline__ void write_swap_local(const Geo &g, uint32_t boff, const float *o) {
        st_plane<T>(g, 26 - I, boff, o[I]);
        Unroll32<T, I + 1>::write_swap_local(g, boff, o);
    }
    // rows[(dy+1) + 3 (dz+1)] and xs[dx+1] are element offsets of the wrapped neighbours
    static __device__ __forceinline__ void read_periodic(const Geo &g, const uint32_t *xs, const uint32_t *rows,
                                                         float *d) {
        constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I);
        const uint32_t boff = (rows[(1 - cy) + 3 * (1 - cz)] + xs[1 - cx]) * (uint32_t)sizeof(T);
        d[I] = ld_plane<T>(g, 26 - I, boff);
        Unroll32<T, I + 1>::read_periodic(g, xs, rows, d);
    }
    static __device__ __forceinline__ void write_periodic(const Geo &g, const uint32_t *xs, const uint32_t *rows,
                                                          const float *o) {
        constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I);
        const uint32_t boff = (rows[(1 + cy) + 3 * (1 + cz)] + xs[1 + cx]) * (uint32_t)sizeof(T);
        st_plane<T>(g, I, boff, o[I]);
        Unroll32<T, I + 1>::write_periodic(g, xs, rows, o);
    }
    // the nine directions with c_x = CX only
    template <int CX>
    static __device__ __forceinline__ void write_periodic_cx(const Geo &g, const uint32_t *xs, const uint32_t *rows,
                                                             const float *o) {
        constexpr int cx = cx_of(I), cy = cy_of(I), cz = cz_of(I);
        if constexpr (cx == CX) {
            const uint32_t boff = (rows[(1 + cy) + 3 * (1 + cz)] + xs[1 + cx]) * (uint32_t)sizeof(T);
            st_plane<T>(g, I, boff, o[I]);
        }
        Unroll32<T, I + 1>::template write_periodic_cx<CX>(g, xs, rows, o);
    }
};
template <typename T>
struct Unroll32<T, 27> {
    static __device__ __forceinline__ void read_natural(const Geo &, uint32_t, float *) {}
    static __device__ __forceinline__ void write_swap_local(const Geo &, uint32_t, const float *) {}
    static __device__ __forceinline__ void read_periodic(const Geo &, const uint32_t *, const uint32_t *, float *) {}
    static __device__ __forceinline__ void write_periodic(const Geo &, const uint32_t *, const uint32_t *, const float *) {}
    template <int CX>
    static __device__ __forceinline__ void write_periodic_cx(const Geo &, const uint32_t *, const uint32_t *,
                                                             const float *) {}
};

template <typename T>
struct Unroll<T, 27> {
    static __device__ __forceinline__ void read_natural(const Geo &, size_t, float *) {}
    static __device__ __forceinline__ void read_sw(const Geo &, int, int, int, float *) {}
    static __device__ __forceinline__ void write_swap_local(const Geo &, size_t, const float *) {}
    static __device__ __forceinline__ void write_push(const Geo &, int, int, int, const float *) {}
    static __device__ __forceinline__ void read_periodic(const Geo &, const int *, const size_t *, float *) {}
    static __device__ __forceinline__ void write_periodic(const Geo &, const int *, const size_t *, const float *) {}
};

// ------------------------------------------------------------ readers
template <typename T, int PAR>
__device__ __forceinline__ void read_cell(const Geo &g, size_t cell, int x, int y, int z, float *d) {
    if (PAR == 0) Unroll<T, 0>::read_natural(g, cell, d);
    else Unroll<T, 0>::read_sw(g, x, y, z, d);
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
