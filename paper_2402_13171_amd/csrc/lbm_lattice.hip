// Lattice kernels: fused AA-pattern stream-collide, initialisation, field
// extraction and FP64 reductions.
//
// AA pattern (in place, one read and one write per population and step):
//   even step: read slot i of the own cell, collide, write f*_i to slot 26-i
//              of the own cell (no neighbour access);
//   odd step:  read the pre-collision f_i from slot 26-i of x - c_i, collide,
//              write f*_i to slot i of x + c_i.
// After an even step the store is in "swapped" layout: the value f_i(x) that
// the two-array scheme would hold after streaming is found in slot 26-i at
// x - c_i (or given by a boundary rule). Every reader of the swapped layout
// (odd steps, field extraction, sampling, checkpoints) uses read_swapped.
//
// Non-periodic boundaries (x inflow/outflow, z bounce-back or free-slip) only
// change where an odd step reads and writes:
//   read, source outside in z:  bounce-back -> slot i of the own cell (the
//       even step left f*_{26-i} there); free-slip -> reflect c_z and read
//       from the same z layer;
//   read, source outside in x:  x = -1 -> inlet equilibrium; x = nx -> the
//       ghost plane G written by the previous even step (reading slot 26-i at
//       nx-1 directly would race with the cell at nx-2);
//   write, target outside in z: bounce-back -> slot 26-i of the own cell;
//       free-slip -> reflected slot in the same z layer;
//   write, target outside in x: dropped;
//   plus the slots no fluid cell pushes: at x = 0 the inlet equilibrium, at
//   x = nx-1 a copy of the outgoing population (zero gradient).
// Each rule mirrors the two-array pull with the same boundary readings, and
// every slot keeps exactly one reader and one writer per step.
#include "lbm_access.h"
#include "lbm_mlp_dev.h"

namespace lbm {

// Slots that no fluid cell pushes in an odd step (x inflow/outflow only).
template <typename T>
__device__ __forceinline__ void odd_boundary_extras(const Geo &g, int x, int y, int z, const float *o) {
    T *pops = (T *)g.pops;
    if (x == 0) {
        // directions entering through the inlet: f_eq(1, u_in) at the source
#pragma unroll
        for (int I = 2; I < 27; I += 3) {  // c_x = +1
            const int cy = cy_of(I), cz = cz_of(I);
            int sz = z - cz;
            int ii = I;
            if (cz != 0 && (sz < 0 || sz >= g.nz)) {
                const int bc = sz < 0 ? g.bc_zlo : g.bc_zhi;
                if (bc == BC_NOSLIP) continue;  // filled by the bounce-back push
                if (bc == BC_FREESLIP) {
                    ii = refl_z(I);
                    sz = z;
                } else {
                    sz = wrapi(sz, g.nz);
                }
            }
            const int sy = wrapi(y - cy, g.ny);
            Store<T>::st(pops + slot_idx<T>(g, I, 0, y, z), inlet_dev(g, g.uin_wr, ii, sy, sz));
        }
    }
    if (x == g.nx - 1) {
        // directions entering through the outlet: copy of the outgoing value
#pragma unroll
        for (int J = 0; J < 27; J += 3) {  // c_x = -1
            const int cy = cy_of(J), cz = cz_of(J);
            const int ty = wrapi(y + cy, g.ny);
            int tz = z + cz;
            if (cz != 0 && (tz < 0 || tz >= g.nz)) {
                const int bc = tz < 0 ? g.bc_zlo : g.bc_zhi;
                if (bc == BC_NOSLIP) continue;
                if (bc == BC_FREESLIP) {
                    Store<T>::st(pops + slot_idx<T>(g, refl_z(J), x, ty, z), o[J]);
                    continue;
                }
                tz = wrapi(tz, g.nz);
            }
            Store<T>::st(pops + slot_idx<T>(g, J, x, ty, tz), o[J]);
        }
    }
}

// Workgroups are dealt round-robin to the 8 XCDs (each with its own L2).
// Renumber them so that XCD j works through chunks of XCD_CHUNK consecutive
// tiles (chunks j, j+8, j+16, ...): tiles adjacent in x, whose odd-step reads
// share cache lines at the tile edge, land on the same L2, while the eight
// XCDs' current chunks stay adjacent, so that the chip as a whole streams one
// contiguous window of every plane. (Handing each XCD one contiguous eighth
// of the tiles instead, eight windows far apart in every plane, measured up
// to 7% slower for 16-bit storage and about 2% for FP32.) Tiles past the last
// whole group of 8 chunks keep their own number. Bijective for any count.
constexpr unsigned XCD_CHUNK = 1024;
__device__ __forceinline__ unsigned xcd_tile(unsigned b, unsigned total) {
    constexpr unsigned NX = 8;
    const unsigned full = total - total % (NX * XCD_CHUNK);
    if (b >= full) return b;
    const unsigned xcd = b % NX, local = b / NX;
    return ((local / XCD_CHUNK) * NX + xcd) * XCD_CHUNK + local % XCD_CHUNK;
}

// One workgroup of 256 threads = one tile of tw (x) by 256/tw (y) cells in one
// z plane, tw in {64, 128, 256}; a wave is a 64-cell row segment. Wide tiles
// keep the cache lines that odd-step shifted accesses split between
// neighbouring row segments inside one workgroup.
// Empty asm statements that claim to rewrite a value (a vector or a scalar
// register), so that addresses built from it are recomputed where they are
// used rather than kept live from an earlier use.
__device__ __forceinline__ void opaque_v(uint32_t &v) { asm volatile("" : "+v"(v)); }
__device__ __forceinline__ void opaque_s(int &v) { asm volatile("" : "+s"(v)); }

// Odd-step sources outside the box in x for a cell off the z walls (z wraps
// if periodic): x = -1 gives the inlet equilibrium, x = nx the ghost plane.
// The fast path has already loaded in-box values from the wrapped positions;
// the lanes at x = 0 and x = nx-1 overwrite those nine values.
template <typename T>
__device__ __forceinline__ void open_x_sources(const Geo &g, int x, int y, int z, float *d) {
    if (x == 0) {
#pragma unroll
        for (int I = 2; I < 27; I += 3) {  // c_x = +1: source at x = -1
            const int sy = wrapi(y - cy_of(I), g.ny), sz = wrapi(z - cz_of(I), g.nz);
            d[I] = inlet_dev(g, g.uin_rd, I, sy, sz);
        }
    }
    if (x == g.nx - 1) {
        const T *G = (const T *)g.ghost;
#pragma unroll
        for (int I = 0; I < 27; I += 3) {  // c_x = -1: source at x = nx
            const int sy = wrapi(y - cy_of(I), g.ny), sz = wrapi(z - cz_of(I), g.nz);
            d[I] = Store<T>::ld(G + (size_t)(I / 3) * g.ny * g.nz + sy + (size_t)g.ny * sz);
        }
    }
}

// Update of one cell (x, y, z) given by the launch: read, collide, write.
// valid = false: a lane without a cell of its own; it returns at once, except
// in the learned-closure variant, whose matrix-core instructions need every
// lane of the wave: there it computes on (x, y, z) (a valid neighbour cell)
// and stores nothing. mlp_lds: the workgroup's LDS copy of the network, its
// DMA started by the caller (mlp_stage_lds).
// XO (fast path): x inflow/outflow rules per lane. Even steps: the x = nx-1
// lanes also write the outflow ghost plane. Odd steps: the reads of the x = 0
// and x = nx-1 lanes from outside the box are replaced by the inlet
// equilibrium and the ghost plane, their pushes out of the box dropped, and
// the slots no fluid cell pushes filled (odd_boundary_extras).
// Odd-step stores of the 18 x-shifted directions through LDS. Pushed
// directly, every wave's store of direction i (c_x = +-1) starts one element
// off a cache line, so each line is written by two waves, and a part of the
// lines reaches HBM twice (3-8 % more write traffic than the algorithmic
// bytes). Here each lane first puts its value in LDS, then lane t stores the
// value aimed at its own x (aligned whole lines per wave): for c_x = -1
// lanes 0..254 take the pushes of lanes 1..255 and lane 255 stores lane 0's
// push to x0 - 1; for c_x = +1 lanes 1..255 take lanes 0..254 and lane 0
// stores lane 255's push to x0 + 256 (x0: the tile's first x, wrapped
// periodically). The same slots and values as the direct pushes, one store
// per lane and direction. In an open domain the pushes out of the box at x = 0
// and x = nx-1 are dropped. Needs one x-row tile of 256 valid lanes (tw = 256,
// nx a multiple of 256). stage: [18][258] of T.
constexpr int STAGE_W = 258;
// the launch chooses the staged kernels when the tiles allow it
static bool odd_staged_ok(const Geo &g, unsigned tw_log2) { return tw_log2 == 8u && (g.nx % 256) == 0; }
template <typename T, bool XO>
__device__ __forceinline__ void write_odd_staged(const Geo &g, int x, const Nbr &n, const float *o, T *stage) {
    const uint32_t t = threadIdx.x;
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        Store<T>::st(stage + j * STAGE_W + t, o[3 * j]);                // c_x = -1, source lane t
        Store<T>::st(stage + (9 + j) * STAGE_W + t + 2, o[3 * j + 2]);  // c_x = +1, source lane t
    }
    Unroll32<T, 0>::template write_periodic_cx<0>(g, n, o);
    __syncthreads();
    const int x0 = x - (int)t;
    const int x_lo = x0 == 0 ? g.nx - 1 : x0 - 1;      // x0 - 1, wrapped
    const int x_hi = x0 + 256 == g.nx ? 0 : x0 + 256;  // x0 + 256, wrapped
    const bool last = t == 255u, first = t == 0u;
    const uint32_t xm = last ? row_xpart<T>(x_lo) : n.xo[1], im = last ? 0u : t + 1u;   // c_x = -1
    const uint32_t xp = first ? row_xpart<T>(x_hi) : n.xo[1], ip = first ? 257u : t + 1u;  // c_x = +1
    const bool keep_m = !(XO && last && x0 == 0), keep_p = !(XO && first && x0 + 256 == g.nx);
#pragma unroll
    for (int j = 0; j < 9; ++j) {
        // directions 3j (c_x = -1) and 3j + 2 (c_x = +1) share c_y, c_z: the
        // row y + c_y of the z plane z + c_z
        const int cy = cy_of(3 * j), cz = cz_of(3 * j);
        const uint32_t r = n.ys[1 + cy];
        const char *pm = (const char *)g.pops + (n.zb[1 + cz] + (size_t)(3 * j) * Blk<T>::W) * sizeof(T);
        const char *pp = (const char *)g.pops + (n.zb[1 + cz] + (size_t)(3 * j + 2) * Blk<T>::W) * sizeof(T);
        const T vm = stage[j * STAGE_W + im], vp = stage[(9 + j) * STAGE_W + ip];
        if (keep_m) *(T *)(pm + (r + xm) * (uint32_t)sizeof(T)) = vm;
        if (keep_p) *(T *)(pp + (r + xp) * (uint32_t)sizeof(T)) = vp;
    }
}

template <typename T, int PAR, int CL, bool BCG, bool FRC, bool GR, bool XO = false, bool LS = false>
__device__ __forceinline__ void cell_update(const Geo &g, const Physics &ph, int x, int y, int z, bool valid,
                                            MlpLds &mlp_lds, T *stage = nullptr) {
    if (CL != CL_MLP && !valid) return;
    const size_t cell = cidx(g, x, y, z);
    float d[27];
    Nbr n;  // fast path (no boundary rules in the addressing), see Unroll32
    if (PAR == 0) {
        if (BCG) {
            Unroll<T, 0>::read_natural(g, slot_idx<T>(g, 0, x, y, z), d);
        } else {
            fast_nbr<T>(g, x, y, z, n);
            Unroll32<T, 0>::read_natural(g, n, d);
        }
    } else if (!BCG) {
        fast_nbr<T>(g, x, y, z, n);
        Unroll32<T, 0>::read_periodic(g, n, d);
        if (XO) open_x_sources<T>(g, x, y, z, d);
    } else {
        Unroll<T, 0>::read_sw(g, x, y, z, d);
    }

    float Fx = 0.f, Fy = 0.f, Fz = 0.f;
    if (FRC) cell_force(ph, (size_t)g.nx * g.ny * g.nz, cell, x, y, z, Fx, Fy, Fz);
    const CellMoments m = moments_of<FRC>(d, Fx, Fy, Fz);
    float om1;
    if (CL == CL_MLP) {
        float f[6];
        closure_features(m, ph.tau0, f);
        mlp_stage_wait();
        const float nut = mlp_nu_t_wave(*ph.mlp, mlp_lds, f);
        om1 = frcp(3.0f * (ph.nu0 + nut) + 0.5f);
    } else {
        om1 = omega1_of<CL>(m, ph);
    }
    float o[27];
    if (GR) collide_general(d, m, om1, ph.omega2, ph.omega_hi, Fx, Fy, Fz, o);
    else collide_unit_rates(m, om1, ph.omega2, Fx, Fy, Fz, o);
    if (CL == CL_MLP && !valid) return;
    sr_round_cell<T>(o, (uint32_t)cell, ph.sr_seed);
    // the closure variant needs its registers for the network: the store
    // offsets and z-plane bases are rebuilt here from opaque copies of x, y
    // and z instead of being held from the loads on through the network (the
    // store base itself stays the kernel argument, so the stores keep the
    // global scalar-base form)
    if (CL == CL_MLP && !BCG) {
        uint32_t xo = (uint32_t)x, yo = (uint32_t)y;
        int zo = z;
        opaque_v(xo);
        opaque_v(yo);
        opaque_s(zo);
        fast_nbr<T>(g, (int)xo, (int)yo, zo, n);
    }
    const Geo &gw = g;

    if (PAR == 0) {
        if (BCG) Unroll<T, 0>::write_swap_local(g, slot_idx<T>(g, 0, x, y, z), o);
        else Unroll32<T, 0>::write_swap_local(gw, n, o);
        if ((BCG || XO) && g.bc_x == BC_INOUT && x == g.nx - 1) {
            T *G = (T *)g.ghost;
#pragma unroll
            for (int J = 0; J < 27; J += 3)
                Store<T>::st(G + (size_t)(J / 3) * g.ny * g.nz + y + (size_t)g.ny * z, o[J]);
        }
    } else if (!BCG) {
        if constexpr (LS) {
            write_odd_staged<T, XO>(gw, x, n, o, stage);
            if (XO) odd_boundary_extras<T>(g, x, y, z, o);
        } else if (XO) {
            // pushes out of the box through x are dropped
            if (x != 0) Unroll32<T, 0>::template write_periodic_cx<-1>(gw, n, o);
            Unroll32<T, 0>::template write_periodic_cx<0>(gw, n, o);
            if (x != g.nx - 1) Unroll32<T, 0>::template write_periodic_cx<1>(gw, n, o);
            odd_boundary_extras<T>(g, x, y, z, o);
        } else {
            Unroll32<T, 0>::write_periodic(gw, n, o);
        }
    } else {
        Unroll<T, 0>::write_push(g, x, y, z, o);
        if (g.bc_x == BC_INOUT) odd_boundary_extras<T>(g, x, y, z, o);
    }
}


// LS: odd-step stores staged through LDS (write_odd_staged); the launch picks
// it for odd steps of 16-bit storage on the fast path without the learned
// closure when the tiles are whole 256-lane rows. (Measured in one process:
// 7 % faster odd steps for FP16 and BF16, 2 % slower for FP32, slower for the
// closure variant, which is bound by its arithmetic.)
template <typename T, int PAR, int CL, bool BCG, bool FRC, bool GR, bool XO = false, bool LS = false>
__global__ __launch_bounds__(256) void k_stream_collide(Geo g, Physics ph, unsigned gx, unsigned gy, unsigned total,
                                                        unsigned tw_log2) {
    const unsigned tile = xcd_tile(blockIdx.x, total);
    const unsigned tw = 1u << tw_log2, th = 256u >> tw_log2;
    const int x0 = (int)((tile % gx) * tw + (threadIdx.x & (tw - 1)));
    const int y0 = (int)(((tile / gx) % gy) * th + (threadIdx.x >> tw_log2));
    const int z = (int)(tile / (gx * gy));
    // z planes left to the boundary-cell kernel: whole workgroups
    if ((g.skip_zlo && z == 0) || (g.skip_zhi && z == g.nz - 1)) return;
    const bool valid = x0 < g.nx && y0 < g.ny;
    if (CL != CL_MLP && !valid) return;
    // closure variant: lanes without a cell recompute the nearest cell of their row
    const int x = CL == CL_MLP ? min(x0, g.nx - 1) : x0;
    const int y = CL == CL_MLP ? min(y0, g.ny - 1) : y0;
    // network operands: DMA into LDS now, in flight with the population loads
    __shared__ MlpLds mlp_lds;
    if (CL == CL_MLP) mlp_stage_lds(ph.mlp, &mlp_lds);
    if constexpr (LS) {
        static_assert(PAR == 1 && !BCG && CL != CL_MLP, "staged stores: fast-path odd steps without the closure");
        __shared__ T stage[18 * STAGE_W];
        cell_update<T, PAR, CL, BCG, FRC, GR, XO, true>(g, ph, x, y, z, valid, mlp_lds, stage);
    } else {
        cell_update<T, PAR, CL, BCG, FRC, GR, XO>(g, ph, x, y, z, valid, mlp_lds);
    }
}

// Odd step on the z wall planes (z = 0 and / or nz-1, all x and y) with the
// general boundary rules; pairs with a fast-path launch that skips them.
template <typename T, int CL, bool FRC>
__global__ __launch_bounds__(256) void k_stream_collide_walls(Geo g, Physics ph, unsigned nlo, unsigned nhi) {
    // nlo / nhi: cells of the z = 0 / z = nz-1 plane to update (nx ny or 0)
    const unsigned nb = nlo + nhi;
    const unsigned b0 = blockIdx.x * 256u + threadIdx.x;
    const bool valid = b0 < nb;
    if (CL != CL_MLP && !valid) return;
    const unsigned b = valid ? b0 : nb - 1;
    const bool lo = b < nlo;
    const unsigned r = lo ? b : b - nlo;
    const int x = (int)(r % (unsigned)g.nx), y = (int)(r / (unsigned)g.nx), z = lo ? 0 : g.nz - 1;
    __shared__ MlpLds mlp_lds;
    if (CL == CL_MLP) mlp_stage_lds(ph.mlp, &mlp_lds);
    cell_update<T, 1, CL, true, FRC, false>(g, ph, x, y, z, valid, mlp_lds);
}

// Pure-memory twin of the periodic fast path: the same tiles, tile order,
// 32-bit offsets and AA access pattern of one step, no collision (each value
// goes back to the slot the collision would write, so the store keeps its
// content up to a permutation). Its rate is the achievable-bandwidth ceiling
// of the stream-collide access pattern.
template <typename T, int PAR, bool LS = false>
__global__ __launch_bounds__(256) void k_pattern_probe(Geo g, unsigned gx, unsigned gy, unsigned total,
                                                       unsigned tw_log2) {
    const unsigned tile = xcd_tile(blockIdx.x, total);
    const unsigned tw = 1u << tw_log2, th = 256u >> tw_log2;
    const int x = (int)((tile % gx) * tw + (threadIdx.x & (tw - 1)));
    const int y = (int)(((tile / gx) % gy) * th + (threadIdx.x >> tw_log2));
    const int z = (int)(tile / (gx * gy));
    if (x >= g.nx || y >= g.ny) return;
    float d[27];
    Nbr n;
    fast_nbr<T>(g, x, y, z, n);
    if (PAR == 0) {
        Unroll32<T, 0>::read_natural(g, n, d);
        Unroll32<T, 0>::write_swap_local(g, n, d);
    } else {
        Unroll32<T, 0>::read_periodic(g, n, d);
        if constexpr (LS) {
            __shared__ T stage[18 * STAGE_W];
            write_odd_staged<T, false>(g, x, n, d, stage);
        } else {
            Unroll32<T, 0>::write_periodic(g, n, d);
        }
    }
}

int launch_pattern_probe(int storage, int parity, const Geo &g, hipStream_t s) {
    const unsigned twl = g.nx >= 256 ? 8u : (g.nx >= 128 ? 7u : 6u);
    const unsigned tw = 1u << twl, th = 256u >> twl;
    const unsigned gx = (g.nx + tw - 1) / tw, gy = (g.ny + th - 1) / th, total = gx * gy * (unsigned)g.nz;
    const dim3 grd(total, 1, 1), blk(256, 1, 1);
    // the odd pass stores like the staged stream-collide kernels where those
    // run (16-bit storage)
    const bool ls = odd_staged_ok(g, twl);
    switch (storage * 2 + parity) {
        case 0: k_pattern_probe<float, 0><<<grd, blk, 0, s>>>(g, gx, gy, total, twl); break;
        case 1: k_pattern_probe<float, 1><<<grd, blk, 0, s>>>(g, gx, gy, total, twl); break;
        case 2: k_pattern_probe<__half, 0><<<grd, blk, 0, s>>>(g, gx, gy, total, twl); break;
        case 3:
            if (ls) k_pattern_probe<__half, 1, true><<<grd, blk, 0, s>>>(g, gx, gy, total, twl);
            else k_pattern_probe<__half, 1><<<grd, blk, 0, s>>>(g, gx, gy, total, twl);
            break;
        case 4: k_pattern_probe<bf16_t, 0><<<grd, blk, 0, s>>>(g, gx, gy, total, twl); break;
        case 5:
            if (ls) k_pattern_probe<bf16_t, 1, true><<<grd, blk, 0, s>>>(g, gx, gy, total, twl);
            else k_pattern_probe<bf16_t, 1><<<grd, blk, 0, s>>>(g, gx, gy, total, twl);
            break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ------------------------------------------------------------ dispatch
// one stream-collide launch; staged odd-step stores where they apply
template <typename T, int PAR, int CL, bool BCG, bool FRC, bool GR, bool XO = false>
static void launch_k1(bool ls, dim3 grd, dim3 blk, hipStream_t s, const Geo &g, const Physics &ph, unsigned gx,
                      unsigned gy, unsigned total, unsigned twl) {
    if constexpr (PAR == 1 && !BCG && CL != CL_MLP && sizeof(T) == 2) {
        if (ls) {
            k_stream_collide<T, PAR, CL, BCG, FRC, GR, XO, true><<<grd, blk, 0, s>>>(g, ph, gx, gy, total, twl);
            return;
        }
    }
    k_stream_collide<T, PAR, CL, BCG, FRC, GR, XO><<<grd, blk, 0, s>>>(g, ph, gx, gy, total, twl);
}

template <typename T, int PAR, int CL>
static void launch_sc(int mode, bool frc, bool gr, const Geo &g, const Physics &ph, hipStream_t s) {
    const unsigned twl = g.nx >= 256 ? 8u : (g.nx >= 128 ? 7u : 6u);
    const unsigned tw = 1u << twl, th = 256u >> twl;
    const unsigned gx = (g.nx + tw - 1) / tw, gy = (g.ny + th - 1) / th, total = gx * gy * (unsigned)g.nz;
    dim3 blk(256, 1, 1), grd(total, 1, 1);
    const bool ls = odd_staged_ok(g, twl);
    // general rates only on the general-boundary path (periodic boxes included)
    if (gr) {
        if (frc) launch_k1<T, PAR, CL, true, true, true>(ls, grd, blk, s, g, ph, gx, gy, total, twl);
        else launch_k1<T, PAR, CL, true, false, true>(ls, grd, blk, s, g, ph, gx, gy, total, twl);
    } else if (mode == SC_GENERAL) {
        if (frc) launch_k1<T, PAR, CL, true, true, false>(ls, grd, blk, s, g, ph, gx, gy, total, twl);
        else launch_k1<T, PAR, CL, true, false, false>(ls, grd, blk, s, g, ph, gx, gy, total, twl);
    } else if (mode == SC_SPLIT && PAR == 0) {
        // even step of an open domain: cell-local, the z walls play no part;
        // only the x = nx-1 lanes add the outflow ghost plane
        const bool xo = g.bc_x == BC_INOUT;
        if (frc) {
            if (xo) launch_k1<T, PAR, CL, false, true, false, true>(ls, grd, blk, s, g, ph, gx, gy, total, twl);
            else launch_k1<T, PAR, CL, false, true, false>(ls, grd, blk, s, g, ph, gx, gy, total, twl);
        } else {
            if (xo) launch_k1<T, PAR, CL, false, false, false, true>(ls, grd, blk, s, g, ph, gx, gy, total, twl);
            else launch_k1<T, PAR, CL, false, false, false>(ls, grd, blk, s, g, ph, gx, gy, total, twl);
        }
    } else if (mode == SC_FAST) {
        if (frc) launch_k1<T, PAR, CL, false, true, false>(ls, grd, blk, s, g, ph, gx, gy, total, twl);
        else launch_k1<T, PAR, CL, false, false, false>(ls, grd, blk, s, g, ph, gx, gy, total, twl);
    } else if constexpr (PAR == 1) {
        // odd step of an open domain: every cell off the z walls on the fast
        // path, the x inflow/outflow rules applied per lane; then the wall
        // planes with the general rules. The two sets own disjoint slots.
        Geo gi = g;
        gi.skip_zlo = g.bc_zlo != BC_PERIODIC;
        gi.skip_zhi = g.bc_zhi != BC_PERIODIC;
        const bool xo = g.bc_x == BC_INOUT;
        if (frc) {
            if (xo) launch_k1<T, PAR, CL, false, true, false, true>(ls, grd, blk, s, gi, ph, gx, gy, total, twl);
            else launch_k1<T, PAR, CL, false, true, false>(ls, grd, blk, s, gi, ph, gx, gy, total, twl);
        } else {
            if (xo) launch_k1<T, PAR, CL, false, false, false, true>(ls, grd, blk, s, gi, ph, gx, gy, total, twl);
            else launch_k1<T, PAR, CL, false, false, false>(ls, grd, blk, s, gi, ph, gx, gy, total, twl);
        }
        const unsigned nxy = (unsigned)g.nx * (unsigned)g.ny;
        const unsigned nlo = gi.skip_zlo ? nxy : 0u, nhi = gi.skip_zhi ? nxy : 0u;
        if (nlo + nhi > 0) {
            const dim3 gw((nlo + nhi + 255u) / 256u, 1, 1);
            if (frc) k_stream_collide_walls<T, CL, true><<<gw, blk, 0, s>>>(gi, ph, nlo, nhi);
            else k_stream_collide_walls<T, CL, false><<<gw, blk, 0, s>>>(gi, ph, nlo, nhi);
        }
    }
}

template <typename T, int PAR>
static int launch_sc_cl(int closure, int mode, bool frc, bool gr, const Geo &g, const Physics &ph, hipStream_t s) {
    switch (closure) {
        case CL_NONE: launch_sc<T, PAR, CL_NONE>(mode, frc, gr, g, ph, s); return 0;
        case CL_SMAG: launch_sc<T, PAR, CL_SMAG>(mode, frc, gr, g, ph, s); return 0;
        case CL_MLP: launch_sc<T, PAR, CL_MLP>(mode, frc, gr, g, ph, s); return 0;
        default: return -1;
    }
}

template <typename T>
static int launch_sc_par(int parity, int closure, int mode, bool frc, bool gr, const Geo &g, const Physics &ph,
                         hipStream_t s) {
    return parity == 0 ? launch_sc_cl<T, 0>(closure, mode, frc, gr, g, ph, s)
                       : launch_sc_cl<T, 1>(closure, mode, frc, gr, g, ph, s);
}

int launch_stream_collide(int storage, int stochastic, int parity, int closure, int mode, bool force,
                          bool general_rates, const Geo &g, const Physics &ph, hipStream_t s) {
    if (mode != SC_FAST && mode != SC_GENERAL && mode != SC_SPLIT) return -1;
    int rc;
    switch (storage * 2 + (stochastic ? 1 : 0)) {
        case 0:
        case 1: rc = launch_sc_par<float>(parity, closure, mode, force, general_rates, g, ph, s); break;
        case 2: rc = launch_sc_par<__half>(parity, closure, mode, force, general_rates, g, ph, s); break;
        case 3: rc = launch_sc_par<f16_sr>(parity, closure, mode, force, general_rates, g, ph, s); break;
        case 4: rc = launch_sc_par<bf16_t>(parity, closure, mode, force, general_rates, g, ph, s); break;
        case 5: rc = launch_sc_par<bf16_sr>(parity, closure, mode, force, general_rates, g, ph, s); break;
        default: return -1;
    }
    if (rc) return rc;
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ------------------------------------------------------------ initialisation
__device__ __forceinline__ double phi1d(int c, double u) {
    return c == 0 ? (2.0 / 3.0 - u * u) : 0.5 * (1.0 / 3.0 + u * u + c * u);
}

template <typename T>
__device__ __forceinline__ void store_eq(const Geo &g, size_t cell, double rho, double ux, double uy, double uz) {
    T *pops = (T *)g.pops;
    const int x = (int)(cell % g.nx), y = (int)((cell / g.nx) % g.ny), z = (int)(cell / ((size_t)g.nx * g.ny));
    const size_t s0 = slot_idx<T>(g, 0, x, y, z);
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const double w = (cx_of(i) == 0 ? 2.0 / 3.0 : 1.0 / 6.0) * (cy_of(i) == 0 ? 2.0 / 3.0 : 1.0 / 6.0) *
                         (cz_of(i) == 0 ? 2.0 / 3.0 : 1.0 / 6.0);
        const double fe = rho * phi1d(cx_of(i), ux) * phi1d(cy_of(i), uy) * phi1d(cz_of(i), uz);
        Store<T>::st(pops + s0 + (size_t)i * Blk<T>::W, (float)(fe - w));
    }
}

template <typename T>
__global__ void k_init_tgv(Geo g, double u0, double k, double rho0) {
    const size_t n = (size_t)g.nx * g.ny * g.nz;
    for (size_t c = blockIdx.x * (size_t)blockDim.x + threadIdx.x; c < n; c += (size_t)gridDim.x * blockDim.x) {
        const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / ((size_t)g.nx * g.ny));
        const double ux = u0 * sin(k * x) * cos(k * y) * cos(k * z);
        const double uy = -u0 * cos(k * x) * sin(k * y) * cos(k * z);
        store_eq<T>(g, c, rho0, ux, uy, 0.0);
    }
}

template <typename T>
__global__ void k_init_eq(Geo g, const double *rho, const double *u, size_t cell0, size_t ncell) {
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < ncell; q += (size_t)gridDim.x * blockDim.x)
        store_eq<T>(g, cell0 + q, rho[q], u[q], u[ncell + q], u[2 * ncell + q]);
}

template <typename T>
static void init_tgv_t(const Geo &g, double u0, double k, double rho0, hipStream_t s) {
    k_init_tgv<T><<<2048, 256, 0, s>>>(g, u0, k, rho0);
}
int launch_init_tgv(int storage, const Geo &g, double u0, double k, double rho0, hipStream_t s) {
    switch (storage) {
        case 0: init_tgv_t<float>(g, u0, k, rho0, s); break;
        case 1: init_tgv_t<__half>(g, u0, k, rho0, s); break;
        case 2: init_tgv_t<bf16_t>(g, u0, k, rho0, s); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}
int launch_init_eq(int storage, const Geo &g, const double *rho, const double *u, size_t cell0, size_t ncell,
                   hipStream_t s) {
    const int nb = (int)((ncell + 255) / 256 < 4096 ? (ncell + 255) / 256 : 4096);
    switch (storage) {
        case 0: k_init_eq<float><<<nb, 256, 0, s>>>(g, rho, u, cell0, ncell); break;
        case 1: k_init_eq<__half><<<nb, 256, 0, s>>>(g, rho, u, cell0, ncell); break;
        case 2: k_init_eq<bf16_t><<<nb, 256, 0, s>>>(g, rho, u, cell0, ncell); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T, int PAR>
__global__ void k_fields(Geo g, Physics ph, double *rho, double *u, size_t cell0, size_t ncell) {
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < ncell; q += (size_t)gridDim.x * blockDim.x) {
        const size_t c = cell0 + q;
        const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / ((size_t)g.nx * g.ny));
        double r, ux, uy, uz;
        cell_macro<T, PAR>(g, ph, c, x, y, z, r, ux, uy, uz);
        rho[q] = r;
        u[q] = ux;
        u[ncell + q] = uy;
        u[2 * ncell + q] = uz;
    }
}

template <typename T, int PAR>
__global__ void k_pops(Geo g, double *f, size_t cell0, size_t ncell) {
    for (size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x; q < ncell; q += (size_t)gridDim.x * blockDim.x) {
        const size_t c = cell0 + q;
        const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / ((size_t)g.nx * g.ny));
        float d[27];
        read_cell<T, PAR>(g, c, x, y, z, d);
#pragma unroll
        for (int i = 0; i < 27; ++i) {
            const double w = (cx_of(i) == 0 ? 2.0 / 3.0 : 1.0 / 6.0) * (cy_of(i) == 0 ? 2.0 / 3.0 : 1.0 / 6.0) *
                             (cz_of(i) == 0 ? 2.0 / 3.0 : 1.0 / 6.0);
            f[(size_t)i * ncell + q] = w + (double)d[i];
        }
    }
}

template <typename T, int PAR>
__global__ void k_sample_pops(Geo g, const size_t *cells, size_t m, double *f) {
    const size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (q >= m) return;
    const size_t c = cells[q];
    const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / ((size_t)g.nx * g.ny));
    float d[27];
    read_cell<T, PAR>(g, c, x, y, z, d);
#pragma unroll
    for (int i = 0; i < 27; ++i) {
        const double w = (cx_of(i) == 0 ? 2.0 / 3.0 : 1.0 / 6.0) * (cy_of(i) == 0 ? 2.0 / 3.0 : 1.0 / 6.0) *
                         (cz_of(i) == 0 ? 2.0 / 3.0 : 1.0 / 6.0);
        f[q * 27 + i] = w + (double)d[i];
    }
}

template <typename T, int PAR>
static void sample_t(const Geo &g, const size_t *cells, size_t m, double *f, hipStream_t s) {
    k_sample_pops<T, PAR><<<(unsigned)((m + 255) / 256), 256, 0, s>>>(g, cells, m, f);
}
int launch_sample_pops(int storage, int parity, const Geo &g, const size_t *cells, size_t m, double *f,
                       hipStream_t s) {
    switch (storage * 2 + parity) {
        case 0: sample_t<float, 0>(g, cells, m, f, s); break;
        case 1: sample_t<float, 1>(g, cells, m, f, s); break;
        case 2: sample_t<__half, 0>(g, cells, m, f, s); break;
        case 3: sample_t<__half, 1>(g, cells, m, f, s); break;
        case 4: sample_t<bf16_t, 0>(g, cells, m, f, s); break;
        case 5: sample_t<bf16_t, 1>(g, cells, m, f, s); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// block means over w^3 cells: rho, u, u u (coarse cells cc0 .. cc0+ncc)
template <typename T, int PAR>
__global__ void k_filtered(Geo g, Physics ph, int w, double *out, size_t cc0, size_t ncc) {
    const size_t q = blockIdx.x * (size_t)blockDim.x + threadIdx.x;
    if (q >= ncc) return;
    const int cnx = g.nx / w, cny = g.ny / w;
    const size_t cc = cc0 + q;
    const int X = (int)(cc % cnx), Y = (int)((cc / cnx) % cny), Z = (int)(cc / ((size_t)cnx * cny));
    double acc[10] = {0, 0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int dz = 0; dz < w; ++dz)
        for (int dy = 0; dy < w; ++dy)
            for (int dx = 0; dx < w; ++dx) {
                const int x = X * w + dx, y = Y * w + dy, z = Z * w + dz;
                double r, ux, uy, uz;
                cell_macro<T, PAR>(g, ph, cidx(g, x, y, z), x, y, z, r, ux, uy, uz);
                acc[0] += r;
                acc[1] += ux;
                acc[2] += uy;
                acc[3] += uz;
                acc[4] += ux * ux;
                acc[5] += uy * uy;
                acc[6] += uz * uz;
                acc[7] += ux * uy;
                acc[8] += ux * uz;
                acc[9] += uy * uz;
            }
    const double inv = 1.0 / ((double)w * w * w);
#pragma unroll
    for (int k = 0; k < 10; ++k) out[(size_t)k * ncc + q] = acc[k] * inv;
}

template <typename T, int PAR>
static void filtered_t(const Geo &g, const Physics &ph, int w, double *out, size_t cc0, size_t ncc, hipStream_t s) {
    k_filtered<T, PAR><<<(unsigned)((ncc + 127) / 128), 128, 0, s>>>(g, ph, w, out, cc0, ncc);
}
int launch_filtered(int storage, int parity, const Geo &g, const Physics &ph, int w, double *out, size_t cc0,
                    size_t ncc, hipStream_t s) {
    switch (storage * 2 + parity) {
        case 0: filtered_t<float, 0>(g, ph, w, out, cc0, ncc, s); break;
        case 1: filtered_t<float, 1>(g, ph, w, out, cc0, ncc, s); break;
        case 2: filtered_t<__half, 0>(g, ph, w, out, cc0, ncc, s); break;
        case 3: filtered_t<__half, 1>(g, ph, w, out, cc0, ncc, s); break;
        case 4: filtered_t<bf16_t, 0>(g, ph, w, out, cc0, ncc, s); break;
        case 5: filtered_t<bf16_t, 1>(g, ph, w, out, cc0, ncc, s); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T, int PAR>
static void fields_t(const Geo &g, const Physics &ph, double *rho, double *u, size_t cell0, size_t ncell,
                     hipStream_t s) {
    const int nb = (int)((ncell + 255) / 256 < 4096 ? (ncell + 255) / 256 : 4096);
    k_fields<T, PAR><<<nb, 256, 0, s>>>(g, ph, rho, u, cell0, ncell);
}
int launch_fields(int storage, int parity, const Geo &g, const Physics &ph, double *rho, double *u, size_t cell0,
                  size_t ncell, hipStream_t s) {
    switch (storage * 2 + parity) {
        case 0: fields_t<float, 0>(g, ph, rho, u, cell0, ncell, s); break;
        case 1: fields_t<float, 1>(g, ph, rho, u, cell0, ncell, s); break;
        case 2: fields_t<__half, 0>(g, ph, rho, u, cell0, ncell, s); break;
        case 3: fields_t<__half, 1>(g, ph, rho, u, cell0, ncell, s); break;
        case 4: fields_t<bf16_t, 0>(g, ph, rho, u, cell0, ncell, s); break;
        case 5: fields_t<bf16_t, 1>(g, ph, rho, u, cell0, ncell, s); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

template <typename T, int PAR>
static void pops_t(const Geo &g, double *f, size_t cell0, size_t ncell, hipStream_t s) {
    const int nb = (int)((ncell + 255) / 256 < 4096 ? (ncell + 255) / 256 : 4096);
    k_pops<T, PAR><<<nb, 256, 0, s>>>(g, f, cell0, ncell);
}
int launch_pops(int storage, int parity, const Geo &g, double *f, size_t cell0, size_t ncell, hipStream_t s) {
    switch (storage * 2 + parity) {
        case 0: pops_t<float, 0>(g, f, cell0, ncell, s); break;
        case 1: pops_t<float, 1>(g, f, cell0, ncell, s); break;
        case 2: pops_t<__half, 0>(g, f, cell0, ncell, s); break;
        case 3: pops_t<__half, 1>(g, f, cell0, ncell, s); break;
        case 4: pops_t<bf16_t, 0>(g, f, cell0, ncell, s); break;
        case 5: pops_t<bf16_t, 1>(g, f, cell0, ncell, s); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ------------------------------------------------------------ FP64 reductions
// Two-stage deterministic sums: a fixed grid of blocks writes per-block
// partials (tree order fixed by the block size), one block adds them in order.
constexpr int RED_BLOCK = 256;
constexpr int NMOM = 6;  // mass, px, py, pz, ke, nan-count

__device__ __forceinline__ double block_sum(double v, double *sh) {
    const int t = threadIdx.x;
    sh[t] = v;
    __syncthreads();
    for (int s = RED_BLOCK / 2; s > 0; s >>= 1) {
        if (t < s) sh[t] += sh[t + s];
        __syncthreads();
    }
    const double r = sh[0];
    __syncthreads();
    return r;
}

template <typename T, int PAR>
__global__ __launch_bounds__(RED_BLOCK) void k_moments_partial(Geo g, Physics ph, double *partials) {
    __shared__ double sh[RED_BLOCK];
    const size_t n = (size_t)g.nx * g.ny * g.nz;
    double acc[NMOM] = {0, 0, 0, 0, 0, 0};
    for (size_t c = blockIdx.x * (size_t)RED_BLOCK + threadIdx.x; c < n; c += (size_t)gridDim.x * RED_BLOCK) {
        const int x = (int)(c % g.nx), y = (int)((c / g.nx) % g.ny), z = (int)(c / ((size_t)g.nx * g.ny));
        double r, ux, uy, uz;
        cell_macro<T, PAR>(g, ph, c, x, y, z, r, ux, uy, uz);
        acc[0] += r;
        acc[1] += r * ux;
        acc[2] += r * uy;
        acc[3] += r * uz;
        acc[4] += 0.5 * r * (ux * ux + uy * uy + uz * uz);
        // cells that are no longer a valid state: NaN, non-positive density, or
        // a speed above one lattice unit per step (far beyond the sound speed)
        const double u2 = ux * ux + uy * uy + uz * uz;
        acc[5] += (!(r > 0.0) || !(u2 <= 1.0)) ? 1.0 : 0.0;
    }
    for (int k = 0; k < NMOM; ++k) {
        const double s = block_sum(acc[k], sh);
        if (threadIdx.x == 0) partials[(size_t)blockIdx.x * NMOM + k] = s;
    }
}

__global__ __launch_bounds__(RED_BLOCK) void k_moments_final(const double *partials, int nblocks, double *out) {
    __shared__ double sh[RED_BLOCK];
    for (int k = 0; k < NMOM; ++k) {
        double a = 0;
        for (int b = threadIdx.x; b < nblocks; b += RED_BLOCK) a += partials[(size_t)b * NMOM + k];
        const double s = block_sum(a, sh);
        if (threadIdx.x == 0) out[k] = s;
    }
}

__global__ void k_check(const double *mom, double mass0, double tol, int *flag) {
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        const double m = mom[0];
        const bool bad = mom[5] > 0.0 || !(fabs(m - mass0) <= tol * fabs(mass0));
        if (bad) *flag = 1;
    }
}

template <typename T, int PAR>
static void moments_t(const Geo &g, const Physics &ph, double *partials, int nblocks, double *out, hipStream_t s) {
    k_moments_partial<T, PAR><<<nblocks, RED_BLOCK, 0, s>>>(g, ph, partials);
    k_moments_final<<<1, RED_BLOCK, 0, s>>>(partials, nblocks, out);
}
int launch_moments(int storage, int parity, const Geo &g, const Physics &ph, double *partials, int nblocks,
                   double *out, hipStream_t s) {
    switch (storage * 2 + parity) {
        case 0: moments_t<float, 0>(g, ph, partials, nblocks, out, s); break;
        case 1: moments_t<float, 1>(g, ph, partials, nblocks, out, s); break;
        case 2: moments_t<__half, 0>(g, ph, partials, nblocks, out, s); break;
        case 3: moments_t<__half, 1>(g, ph, partials, nblocks, out, s); break;
        case 4: moments_t<bf16_t, 0>(g, ph, partials, nblocks, out, s); break;
        case 5: moments_t<bf16_t, 1>(g, ph, partials, nblocks, out, s); break;
        default: return -1;
    }
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

int launch_check(int storage, int parity, const Geo &g, const Physics &ph, double *partials, int nblocks,
                 double mass0, double tol, int *flag, hipStream_t s) {
    double *out = partials + (size_t)nblocks * NMOM;
    const int rc = launch_moments(storage, parity, g, ph, partials, nblocks, out, s);
    if (rc) return rc;
    k_check<<<1, 64, 0, s>>>(out, mass0, tol, flag);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

// ------------------------------------------------------------ inlet plane
// u_in(q) = mean(q) + (1 - f) box[s0](q) + f box[s1](q), s = s_pos mod lt
__global__ __launch_bounds__(256) void k_inflow(float *uin, const float *mean, const float *box, int lt, int plane,
                                                double s_pos) {
    const int q = blockIdx.x * 256 + threadIdx.x;
    if (q >= plane) return;
    double sp = fmod(s_pos, (double)lt);
    if (sp < 0.0) sp += lt;
    int s0 = (int)floor(sp);
    if (s0 >= lt) s0 = lt - 1;
    const int s1 = s0 + 1 == lt ? 0 : s0 + 1;
    const float f = (float)(sp - s0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        float v = mean[(size_t)c * plane + q];
        if (box) {
            const float a = box[((size_t)c * lt + s0) * plane + q], b = box[((size_t)c * lt + s1) * plane + q];
            v += (1.0f - f) * a + f * b;
        }
        uin[(size_t)c * plane + q] = v;
    }
}

int launch_inflow(float *uin, const float *mean, const float *box, int lt, int plane, double s_pos, hipStream_t s) {
    k_inflow<<<(plane + 255) / 256, 256, 0, s>>>(uin, mean, box, lt, plane, s_pos);
    return hipGetLastError() == hipSuccess ? 0 : -2;
}

}  // namespace lbm
