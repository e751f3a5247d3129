// kernels.hpp -- gfx950 kernels of the porous-media lattice Boltzmann step.
//
// One thread per lattice cell, 256 threads (four wave64) per block, blocks
// over the flattened cell index so that every population plane is read and
// written in contiguous, coalesced runs along x.  Populations are
// structure-of-arrays [19][nz][ny][nx] in two copies (A-B): a step pulls from
// the copy holding step n and writes step n+1 into the other one, so each
// population is read once and written once per step and no cell waits for
// another.  In 16-bit storage the miscible model pairs its two lattices:
// plane q holds one 32-bit word (f_q, h_q) per cell.  The hot path is bound by HBM bandwidth, not arithmetic; there is
// no dense contraction, hence no MFMA.
//
// Addressing: every population plane is addressed as a wave-uniform base
// (scalar registers) plus a 32-bit per-lane byte offset, which maps onto the
// global_load/global_store "saddr" form; only waves that hold a cell next to
// a wall take the path with per-lane bounce-back address selects.  The
// collision is refactored into a few fused multiply-adds per direction
// around per-cell constants.
//
// Paper references: Sec. 2.1 (Eqs. macros1, macros, lbe2, coeffforce1,
// forcement, expandV, expandVsub, equilc1, equilc2), Sec. 2.2 (Eqs. equild,
// boltzeqD), Sec. 4 (order of the operations of a step), Eq. nuall (local
// viscosity).
#pragma once

#include "d3q19.hpp"

namespace plbm {

enum { PH_SINGLE = 0, PH_MISCIBLE = 1, PH_IMMISCIBLE = 2, PH_FREESURF = 3 };
enum { CELL_FLUID = 0, CELL_SOLID = 1, CELL_RES = 2 };

#ifndef PLBM_BLOCK
#define PLBM_BLOCK 256
#endif
#ifndef PLBM_XCD
#define PLBM_XCD 0
#endif
#ifndef PLBM_SLAB
#define PLBM_SLAB 0
#endif
#define PLBM_STEP_ATTR __launch_bounds__(PLBM_BLOCK)

constexpr int BLOCK = PLBM_BLOCK;
constexpr int MAXB = 64;     // lattices per batched launch
constexpr int NPART = 9;     // diagnostic partial sums per block

// Per-lattice parameters, resident in the lattice's workspace.
struct LatDev {
    int nx, ny, nz;
    int ncell;
    int nblocks;
    int bpp;                    // blocks per z-plane for the slab mapping (0: identity)
    int physics;
    int forch, eps_grad;
    int uniform_eps, uniform_kinv;
    int full_tensor;            // K^-1 per cell as frame quaternion (4 planes) + eigenvalues (3 planes)
    uint32_t wall_faces, res_faces;   // bit f: face f (-x,+x,-y,+y,-z,+z) is a wall / a reservoir
    double eps_u, kinv_u[3];
    double G[3];
    double k1, k0;              // viscosity law, per-cell factor e^{k1 C + k0}
    double nu1, nu2;            // two-fluid viscosities
    double tau_d, D;            // solute relaxation time and diffusivity
    double A, beta;             // surface tension, recolouring
    double face_rho[6], face_conc[6];
    double face_cw[7];          // wall colour (1 + cos theta)/2 of each face; [6]: obstacles
    void *f[2];                 // hydrodynamic populations (deviations f - w), copies A, B
    void *h[2];                 // second lattice (solute h or fluid-1 g), copies A, B
    void *fm[2], *hm[2];        // split 16-bit codecs: per-cell FP32 mass planes of each copy
    void *eps, *kinv, *mom, *rho1;
    const void *links;          // obstacle mask as link words (bit 0: solid, bit q: x - v_q solid), or null
    const void *fs;             // free-surface state (FsDev), or null
    const void *ms;             // further solutes (MsDev), or null
    double *partials, *diag;
    int *err;
    uint32_t div_nx[3], div_nxy[3];   // magic numbers of the divisions by nx and nx*ny
    uint32_t pstride;           // elements from one population plane to the next (>= ncell)
    uint32_t ppstride;          // paired planes (miscible, 16-bit storage): words from one plane to the next
};

// Solutes beyond the first (miscible mode with several species), in the
// workspace: per solute its two population copies (19 planes of the lattice's
// plane stride) and, for split storage, its two mass planes; its D and tau_d
// (D = (tau_d - 1/2)/3 in double, as for the first solute) and reservoir
// concentrations.  The moments buffer then holds their concentrations as
// planes 5, 6, ...
constexpr int MAXSPX = 3;
struct MsDev {
    int nsx;                    // number of further solutes (1..MAXSPX)
    void *h[MAXSPX][2];
    void *hm[MAXSPX][2];
    double tau_d[MAXSPX], D[MAXSPX];
    double face_conc[MAXSPX][6];
};

// the further-solute block (global memory, read with scalar loads)
__device__ inline const GL MsDev *ms_of(const LatDev *L)
{
    return static_cast<const GL MsDev *>((const GL void *)L->ms);
}

// Arguments of one batched launch: lattice l owns logical blocks
// [blk_start[l], blk_start[l+1]).  flags bit 0: copy holding step n; bit 1:
// write the moments and the FP64 diagnostics of this step.  nuc: the uniform
// factor nu0 * min(a0 + a1 e^{alpha t}, cap) of the step being computed.
struct BatchArgs {
    int n, total_blocks;
    int blk_start[MAXB + 1];
    int flags[MAXB];
    const LatDev *lat[MAXB];
    double nuc[MAXB];
};

// Optional mapping of hardware blocks (dispatched round-robin over the 8
// XCDs) to contiguous logical ranges per XCD.  Off by default: it makes the
// XCDs sweep eight distant regions at once, which measures slower.
__device__ inline int xcd_remap(int b, int nb)
{
    if (!PLBM_XCD) return b;
    const int X = 8;
    int q = nb / X, r = nb - q * X;
    int xcd = b % X, slot = b / X;
    return xcd * q + min(xcd, r) + slot;
}

// Hardware block b (dispatched round-robin, XCD b mod 8) -> logical block of
// its lattice: each XCD takes runs of XCD_ROWS consecutive rows (blocks), so
// that most y-neighbour rows of a block's stencils were fetched into the same
// XCD's L2, while the eight XCDs still work on 8 x XCD_ROWS consecutive rows at
// a time.  b is the block's index within its lattice's range of the launch;
// every range starts at a multiple of 8 x XCD_ROWS and spans a whole number of
// such groups (the library pads it; blocks mapped beyond the lattice's rows
// exit), so b mod 8 is the XCD in batched launches too.  Measured against the
// identity (results bitwise the same): 256^3 FP32 -0.3 to -1.2%, BF16 -1.5%;
// 512^3 FP32 -1.7%, BF16 -4%, FP16 split -9%.  Runs of 2 rows gained less, runs
// of 8 cost the 256^3 FP32 step 1.6%.  Identity unless nb is a multiple of
// 8 x XCD_ROWS.
constexpr int XCD_ROWS = 4;
constexpr int XCD_GROUP = 8 * XCD_ROWS;
__device__ inline int row_group_remap(int b, int nb)
{
    if (nb % XCD_GROUP != 0) return b;
    const int x = b & 7, s = b >> 3;
    return (s / XCD_ROWS) * XCD_GROUP + x * XCD_ROWS + (s % XCD_ROWS);
}

// Slab mapping within one lattice: when a z-plane is a whole number bpp of
// blocks with bpp a multiple of 8, hardware block b (XCD b mod 8) takes the
// (b mod 8)-th eighth of the y-rows of plane b / bpp.  Each XCD then owns one
// y-slab of every plane, so the y+-1 and z+-1 neighbour rows read by the
// porosity gradient and the colour gradient stay in that XCD's L2, while all
// XCDs sweep the same plane together.  It cuts the fetched bytes of the
// 256^3 FP32 miscible step from 1.07x to 1.03x of the algorithmic reads but
// measures 4% slower than the identity, so it is compiled in only with
// PLBM_SLAB=1 (step and colour kernels only).  bpp == 0: identity.
__device__ inline int slab_remap(int b, int bpp)
{
    if (bpp == 0) return b;
    const int z = b / bpp, r = b - z * bpp;
    return z * bpp + (r & 7) * (bpp >> 3) + (r >> 3);
}

// Logical block (row) of the lattice-local hardware block b of a step or
// colour launch whose range for this lattice is nb blocks; -1 for the padding
// beyond the lattice's rows.  The slab mapping, when compiled in, replaces the
// row groups.
__device__ inline int step_block(int b, int nb, const LatDev *L)
{
    if constexpr (PLBM_SLAB) return b < L->nblocks ? slab_remap(b, L->bpp) : -1;
    const int lb = row_group_remap(b, nb);
    return lb < L->nblocks ? lb : -1;
}

__device__ inline int find_lattice(const BatchArgs &a, int gb)
{
    int l = 0;
    while (l + 1 < a.n && gb >= a.blk_start[l + 1]) ++l;
    return l;
}

// link word of a cell: 0 without an obstacle mask
__device__ inline uint32_t link_word(const LatDev *L, uint32_t idx)
{
    return L->links ? static_cast<const GL uint32_t *>((const GL void *)L->links)[idx] : 0u;
}

// Class of a cell: a wall-face cell is solid (face = its face); else an
// obstacle of the mask is solid (face = 6); else a reservoir-face cell
// belongs to that reservoir; else fluid.
// Faces of the box a cell lies on, as bits f = 2 axis + (0: low, 1: high).
__device__ inline uint32_t faces_of(const LatDev *L, int x, int y, int z)
{
    return uint32_t(x == 0) | uint32_t(x == L->nx - 1) << 1 | uint32_t(y == 0) << 2 |
           uint32_t(y == L->ny - 1) << 3 | uint32_t(z == 0) << 4 | uint32_t(z == L->nz - 1) << 5;
}

// Class of a cell: a wall-face cell is solid (face = its face); else an
// obstacle of the mask is solid (face = 6); else a reservoir-face cell
// belongs to that reservoir; else fluid.  The lowest face wins where faces
// meet.  Branch-free: selects on the face bits.
__device__ inline int cell_type(const LatDev *L, int x, int y, int z, uint32_t lw, int &face)
{
    const uint32_t on = faces_of(L, x, y, z);
    const uint32_t wall = on & L->wall_faces, res = on & L->res_faces;
    const bool obst = (lw & 1u) != 0;
    face = wall ? int(__builtin_ctz(wall)) : (obst ? 6 : (res ? int(__builtin_ctz(res)) : -1));
    return (wall || obst) ? CELL_SOLID : (res ? CELL_RES : CELL_FLUID);
}

// Neighbourhood of a fluid cell: wrapped coordinates of x-1 / x+1 etc. as
// flat offsets, and the set of links whose upstream cell x - v_q is solid.
// A fluid cell is never on a wall or reservoir plane, so on non-periodic axes
// x-1 and x+1 are always inside the box.
struct Nbr {
    uint32_t xm, x0, xp;        // x offsets
    uint32_t ym, y0, yp;        // y * nx
    uint32_t zm, z0, zp;        // z * nx * ny
    uint32_t bb;                // bit q (1..18): x - v_q is solid (bounce-back link)
};

// lw: the cell's link word (obstacle mask); without a mask the bounce-back
// links follow from the wall faces: a wall plane at x - 1 cuts every link
// with c_x > 0, and so on.
__device__ inline Nbr neighbours(const LatDev *L, int x, int y, int z, uint32_t lw)
{
    Nbr b;
    const uint32_t nx = L->nx, ny = L->ny, nz = L->nz, nxy = nx * ny;
    b.x0 = x;
    b.xm = x ? x - 1 : nx - 1;
    b.xp = (uint32_t)x + 1 < nx ? x + 1 : 0;
    b.y0 = y * nx;
    b.ym = (y ? y - 1 : ny - 1) * nx;
    b.yp = ((uint32_t)y + 1 < ny ? y + 1 : 0) * nx;
    b.z0 = z * nxy;
    b.zm = (z ? z - 1 : nz - 1) * nxy;
    b.zp = ((uint32_t)z + 1 < nz ? z + 1 : 0) * nxy;
    if (L->links) {
        b.bb = lw & ~1u;
    } else {
        // wall planes one cell away from this cell, as face bits
        const uint32_t w = L->wall_faces &
                           (uint32_t(x == 1) | uint32_t((uint32_t)x + 2 == nx) << 1 | uint32_t(y == 1) << 2 |
                            uint32_t((uint32_t)y + 2 == ny) << 3 | uint32_t(z == 1) << 4 |
                            uint32_t((uint32_t)z + 2 == nz) << 5);
        b.bb = (w & 1u ? XP : 0u) | (w & 2u ? XN : 0u) | (w & 4u ? YP : 0u) | (w & 8u ? YN : 0u) |
               (w & 16u ? ZP : 0u) | (w & 32u ? ZN : 0u);
    }
    return b;
}

// offset of the cell x + s*v_q (s = +1 or -1)
template <int Q, int SIGN>
__device__ inline uint32_t shifted(const Nbr &b)
{
    constexpr int sx = SIGN * cx(Q), sy = SIGN * cy(Q), sz = SIGN * cz(Q);
    const uint32_t ox = sx > 0 ? b.xp : (sx < 0 ? b.xm : b.x0);
    const uint32_t oy = sy > 0 ? b.yp : (sy < 0 ? b.ym : b.y0);
    const uint32_t oz = sz > 0 ? b.zp : (sz < 0 ? b.zm : b.z0);
    return ox + oy + oz;
}

// is the cell x + s*v_q solid?  (x + v_q = x - v_opp(q))
template <int Q, int SIGN>
__device__ inline bool shifted_solid(const Nbr &b)
{
    constexpr int bitq = SIGN < 0 ? Q : opp(Q);
    return ((b.bb >> bitq) & 1u) != 0;
}

// does any cell of the wave have a solid upstream neighbour?  (wave-uniform)
__device__ inline bool wave_near_solid(const Nbr &b)
{
    return __builtin_amdgcn_ballot_w64(b.bb != 0u) != 0;
}

template <class T>
__device__ inline const GL T *plane(const void *base, uint32_t n, int q)
{
    return static_cast<const GL T *>((const GL void *)base) + size_t(q) * n;
}

template <class T>
__device__ inline GL T *plane_w(void *base, uint32_t n, int q)
{
    return static_cast<GL T *>((GL void *)base) + size_t(q) * n;
}

// element i of a plane: uniform base + zero-extended 32-bit byte offset
template <class T>
__device__ inline const GL T *at(const GL T *p, uint32_t i)
{
    return reinterpret_cast<const GL T *>(reinterpret_cast<const GL char *>(p) + i * uint32_t(sizeof(T)));
}

template <class T>
__device__ inline GL T *at(GL T *p, uint32_t i)
{
    return reinterpret_cast<GL T *>(reinterpret_cast<GL char *>(p) + i * uint32_t(sizeof(T)));
}

template <class R>
__device__ inline R ldg(const void *base, uint32_t i)
{
    return *at(static_cast<const GL R *>((const GL void *)base), i);
}

template <class R>
__device__ inline void stg(void *base, uint32_t i, R v)
{
    *at(static_cast<GL R *>((GL void *)base), i) = v;
}

// element i of plane k of a field with n values per plane (64-bit uniform
// plane base, 32-bit offset within the plane)
template <class R>
__device__ inline R ldp(const void *base, uint32_t n, int k, uint32_t i)
{
    return *at(plane<R>(base, n, k), i);
}

template <class R>
__device__ inline void stp(void *base, uint32_t n, int k, uint32_t i, R v)
{
    *at(plane_w<R>(base, n, k), i) = v;
}

// Pull streaming (Eqs. lbe2, boltzeqD): f_q(x) = f~_q(x - v_q), or
// f~_opp(q)(x) when x - v_q is solid (halfway bounce-back).
//
// Source of direction Q in one uniform plane base: the plane pair
// {Q, opp(Q)} is addressed from the lower plane, so the streamed value
// (plane Q at x - v_q) and the bounced one (plane opp(Q) at x itself) are both
// 32-bit offsets from the same base and a bounce-back is one select (n is the
// plane stride; the library keeps 2 n * sizeof(storage) <= 2^32 bytes).
template <int Q>
__device__ inline uint32_t pair_offset(const Nbr &b, uint32_t n, uint32_t idx, bool bb)
{
    const uint32_t src = shifted<Q, -1>(b);
    if constexpr (Q < opp(Q)) return bb ? n + idx : src;
    else return bb ? idx : n + src;
}

template <int Q>
constexpr int pair_lo() { return Q < opp(Q) ? Q : opp(Q); }

// Split codecs: a population is w_q m + r_q, with the per-cell mass m in an
// FP32 plane M and the remainder r_q in the 16-bit planes; a bounced link
// takes both from the cell itself.  BB = false: no cell of the wave has a
// solid upstream neighbour.  XL: the masses of the links with c_x != 0 are
// not loaded here (xl_masses).
template <class S, bool BB, bool XL, int Q = 0>
__device__ inline void split_loads(const void *P, const void *M, uint32_t n, uint32_t idx, const Nbr &b,
                                   typename Codec<S>::R *r, typename Codec<S>::R *m)
{
    using R = typename Codec<S>::R;
    if constexpr (BB && Q != 0) {
        const bool s = shifted_solid<Q, -1>(b);
        r[Q] = Codec<S>::load(at(plane<S>(P, n, pair_lo<Q>()), pair_offset<Q>(b, n, idx, s)));
        m[Q] = ldg<R>(M, s ? idx : shifted<Q, -1>(b));
    } else {
        const uint32_t src = shifted<Q, -1>(b);
        r[Q] = Codec<S>::load(at(plane<S>(P, n, Q), src));
        if constexpr (!XL || cx(Q) == 0) m[Q] = ldg<R>(M, src);
    }
    if constexpr (Q + 1 < NQ) split_loads<S, BB, XL, Q + 1>(P, M, n, idx, b, r, m);
}

// Split codecs, waves without bounce-back: the upstream mass of a link with
// c_x = +1 (-1) is the one that the lane below (above) loads for the link of
// the same row with c_x = 0, when that lane holds the cell x - 1 (x + 1) of
// this cell's row: it is taken across the wave by a DPP shift of one lane
// instead of being loaded again (9 mass loads instead of 19).  A lane whose
// neighbour lane is outside the wave, inactive, holds another cell or lies in
// another row (the row ends or wraps there) needs that mass from memory: every
// lane issues one more load per row, with the others and before the shifts,
// at the outer mass it needs (or its row's own, which it has), and a wave in
// which some lane needs both outer masses of its rows that way takes the
// general path.  Timed at 256^3, the split miscible step ran 4-5% faster
// than with the 19 loads; staging the rows in LDS behind a barrier, or
// loading the outer masses under per-lane branches, ran slower than that.
struct XLanes {
    bool lo, hi;   // the lane loads its mass at x - 1 (lo) or x + 1 (hi)
};

template <int CTRL>
__device__ inline float lane_shift(float v)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}

template <int CTRL>
__device__ inline f32x2_t lane_shift(f32x2_t v)
{
    return f32x2_t{lane_shift<CTRL>(v.x), lane_shift<CTRL>(v.y)};
}

constexpr int DPP_WAVE_SHL1 = 0x130;   // lane i reads lane i + 1
constexpr int DPP_WAVE_SHR1 = 0x138;   // lane i reads lane i - 1

__device__ inline XLanes xlanes(const Nbr &b, uint32_t idx)
{
    const uint64_t act = __builtin_amdgcn_read_exec();
    const int lane = int(__lane_id());
    const uint32_t below = uint32_t(__builtin_amdgcn_update_dpp(0, int(idx), DPP_WAVE_SHR1, 0xf, 0xf, false));
    const uint32_t above = uint32_t(__builtin_amdgcn_update_dpp(0, int(idx), DPP_WAVE_SHL1, 0xf, 0xf, false));
    XLanes x;
    x.lo = lane == 0 || !((act >> ((lane - 1) & 63)) & 1u) || below + 1u != idx || b.xm + 1u != b.x0;
    x.hi = lane == 63 || !((act >> ((lane + 1) & 63)) & 1u) || above != idx + 1u || b.x0 + 1u != b.xp;
    return x;
}

// does a lane of the wave need both outer masses of its rows from memory?
__device__ inline bool xl_general(const XLanes &x) { return __builtin_amdgcn_ballot_w64(x.lo && x.hi) != 0; }

template <int CX, int CY, int CZ>
__host__ __device__ constexpr int link_of()
{
    for (int q = 0; q < NQ; ++q)
        if (cx(q) == CX && cy(q) == CY && cz(q) == CZ) return q;
    return -1;
}

// the one load per row (kept in slot Q of the row's c_x = +1 link)
template <class T, int Q = 1>
__device__ inline void xl_loads(const void *M, const Nbr &b, const XLanes &x, T *e)
{
    if constexpr (cx(Q) > 0) {
        constexpr int qm = link_of<-1, cy(Q), cz(Q)>(), q0 = link_of<0, cy(Q), cz(Q)>();
        const uint32_t lo = shifted<Q, -1>(b), hi = shifted<qm, -1>(b), own = shifted<q0, -1>(b);
        e[Q] = ldg<T>(M, x.lo ? lo : (x.hi ? hi : own));
    }
    if constexpr (Q + 1 < NQ) xl_loads<T, Q + 1>(M, b, x, e);
}

// Both shifts of a row are computed before its selects, where every lane of
// the pull is active.  Written inside a select (x.lo ? e : shift), a shift
// was moved by hipcc into the branch it made of the select, ran there with
// the lanes of x.lo masked off and read them: wrong masses wherever a row
// ends inside a wave (tests/test_gpu_split_rows.py covers such rows).
template <class T, int Q = 1>
__device__ inline void xl_masses(const XLanes &x, const T *e, T *m)
{
    if constexpr (cx(Q) > 0) {
        constexpr int qm = link_of<-1, cy(Q), cz(Q)>(), q0 = link_of<0, cy(Q), cz(Q)>();
        const T lo = lane_shift<DPP_WAVE_SHR1>(m[q0]), hi = lane_shift<DPP_WAVE_SHL1>(m[q0]);
        m[Q] = x.lo ? e[Q] : lo;
        m[qm] = x.hi ? e[Q] : hi;
    }
    if constexpr (Q + 1 < NQ) xl_masses<T, Q + 1>(x, e, m);
}

// The same sharing for a per-cell field read at the 18 neighbours x + v_q of
// a gradient stencil (the porosity gradient of the solute's drift): v[q] =
// E(x + v_q) from 8 row loads (the links with c_x = 0), 5 edge loads and
// the shifts.  The mirror of xl_loads / xl_masses for x + v_q instead of
// x - v_q; the shifts again come before the selects.
template <class R, int Q = 1>
__device__ inline void nb_rows(const void *E, const Nbr &b, R *v)
{
    if constexpr (cx(Q) == 0) v[Q] = ldg<R>(E, shifted<Q, 1>(b));
    if constexpr (Q + 1 < NQ) nb_rows<R, Q + 1>(E, b, v);
}

template <class R, int Q = 1>
__device__ inline void nb_edges(const void *E, const Nbr &b, const XLanes &x, R *e)
{
    if constexpr (cx(Q) > 0) {
        constexpr int qm = link_of<-1, cy(Q), cz(Q)>(), q0 = link_of<0, cy(Q), cz(Q)>();
        // x + v_qm is the cell at x - 1 of the row, x + v_Q the one at x + 1
        const uint32_t lo = shifted<qm, 1>(b), hi = shifted<Q, 1>(b), own = shifted<q0, 1>(b);
        e[Q] = ldg<R>(E, x.lo ? lo : (x.hi ? hi : own));
    }
    if constexpr (Q + 1 < NQ) nb_edges<R, Q + 1>(E, b, x, e);
}

template <class R, int Q = 1>
__device__ inline void nb_shift(const XLanes &x, const R *e, R *v)
{
    if constexpr (cx(Q) > 0) {
        constexpr int qm = link_of<-1, cy(Q), cz(Q)>(), q0 = link_of<0, cy(Q), cz(Q)>();
        const R lo = lane_shift<DPP_WAVE_SHR1>(v[q0]), hi = lane_shift<DPP_WAVE_SHL1>(v[q0]);
        v[qm] = x.lo ? e[Q] : lo;
        v[Q] = x.hi ? e[Q] : hi;
    }
    if constexpr (Q + 1 < NQ) nb_shift<R, Q + 1>(x, e, v);
}

template <class S, bool BB, bool XL = false, int Q = 0>
__device__ inline void pull_each(const void *P, const void *M, uint32_t n, uint32_t idx, const Nbr &b,
                                 typename Codec<S>::R *out, const XLanes &xl = XLanes{})
{
    using R = typename Codec<S>::R;
    if constexpr (Codec<S>::split) {
        // all remainder and mass loads first, then the decode
        R r[NQ], m[NQ];
        split_loads<S, BB, XL>(P, M, n, idx, b, r, m);
        if constexpr (XL) {
            R e[NQ];
            xl_loads<R>(M, b, xl, e);
            xl_masses<R>(xl, e, m);
        }
#pragma unroll
        for (int q = 0; q < NQ; ++q) out[q] = fma(weight<R>(q), m[q], r[q]);
    } else {
        if constexpr (BB && Q != 0) {
            const bool s = shifted_solid<Q, -1>(b);
            out[Q] = Codec<S>::load(at(plane<S>(P, n, pair_lo<Q>()), pair_offset<Q>(b, n, idx, s)));
        } else {
            out[Q] = Codec<S>::load(at(plane<S>(P, n, Q), shifted<Q, -1>(b)));
        }
        if constexpr (Q + 1 < NQ) pull_each<S, BB, false, Q + 1>(P, M, n, idx, b, out);
    }
}

// Pull of one lattice.  Waves without a solid upstream neighbour (all but a
// thin layer next to walls and obstacles) take the path without selects (and
// with the split codecs, XS, the one that shares the x-links' masses).
template <class S, bool XS = true>
__device__ inline void pull_all(const void *P, const void *M, uint32_t n, uint32_t idx, const Nbr &b,
                                typename Codec<S>::R *out)
{
    if constexpr (Codec<S>::split && XS) {
        const XLanes xl = xlanes(b, idx);
        if (wave_near_solid(b) || xl_general(xl)) pull_each<S, true>(P, M, n, idx, b, out);
        else pull_each<S, false, true>(P, M, n, idx, b, out, xl);
    } else {
        if (wave_near_solid(b)) pull_each<S, true>(P, M, n, idx, b, out);
        else pull_each<S, false>(P, M, n, idx, b, out);
    }
}

template <class S, int Q = 0>
__device__ inline void store_each(void *P, uint32_t n, uint32_t idx, const typename Codec<S>::R *v)
{
    Codec<S>::store(at(plane_w<S>(P, n, Q), idx), v[Q]);
    if constexpr (Q + 1 < NQ) store_each<S, Q + 1>(P, n, idx, v);
}

// Store the 19 populations of a cell.  Split codecs: with m = sum_q v_q in
// FP32, the remainders r_q = v_q - w_q m are rounded to 16 bits (r~_q) and
// the mass plane holds m - sum_q r~_q, so that the decoded populations
// w_q (m - sum r~) + r~_q sum to m again (the weights sum to 1): the cell's
// mass survives the rounding.  Storing m itself lost mass steadily: in
// opposite links the remainders are +-a + b, and where b is below the 16-bit
// resolution of a the two roundings drop about 2b with one sign.  The
// correction moves every decoded population by w_q times the rounding sum
// and leaves the momentum as it was (sum_q w_q v_q = 0).
template <class S>
__device__ inline void store_all(void *P, void *M, uint32_t n, uint32_t idx, const typename Codec<S>::R *v)
{
    using R = typename Codec<S>::R;
    if constexpr (Codec<S>::split) {
        R m = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) m += v[q];
        R s = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const uint16_t e = Codec<S>::enc(fma(-weight<R>(q), m, v[q]));
            s += Codec<S>::dec(e);
            Codec<S>::store_bits(at(plane_w<S>(P, n, q), idx), e);
        }
        stg<R>(M, idx, m - s);
    } else {
        store_each<S>(P, n, idx, v);
    }
}

// Paired storage (miscible model, 16-bit codecs): plane q of a copy holds,
// per cell, the PairCodec word of (f_q, h_q); split codecs keep the cell's
// two FP32 masses as one pair (m_f, m_h).  One pull then loads one word per
// link for both lattices.  Rounding and arithmetic are those of the unpaired
// codecs, so results are bitwise the same.
template <int PHYS, class S>
constexpr bool paired_v = PHYS == PH_MISCIBLE && sizeof(S) == 2;

template <class S, bool BB, bool XL, int Q = 0>
__device__ inline void pair_loads(const void *P, const void *M, uint32_t n, uint32_t idx, const Nbr &b,
                                  typename Codec<S>::R *a, typename Codec<S>::R *c, f32x2_t *m)
{
    using W = typename PairCodec<S>::W;
    if constexpr (BB && Q != 0) {
        const bool s = shifted_solid<Q, -1>(b);
        PairCodec<S>::load(at(plane<W>(P, n, pair_lo<Q>()), pair_offset<Q>(b, n, idx, s)), a[Q], c[Q]);
        if constexpr (Codec<S>::split) m[Q] = ldg<f32x2_t>(M, s ? idx : shifted<Q, -1>(b));
    } else {
        const uint32_t src = shifted<Q, -1>(b);
        PairCodec<S>::load(at(plane<W>(P, n, Q), src), a[Q], c[Q]);
        if constexpr (Codec<S>::split && (!XL || cx(Q) == 0)) m[Q] = ldg<f32x2_t>(M, src);
    }
    if constexpr (Q + 1 < NQ) pair_loads<S, BB, XL, Q + 1>(P, M, n, idx, b, a, c, m);
}

// Pull of both lattices from paired planes (a: f, c: h).
template <class S>
__device__ inline void pull_pair(const void *P, const void *M, uint32_t n, uint32_t idx, const Nbr &b,
                                 typename Codec<S>::R *a, typename Codec<S>::R *c)
{
    using R = typename Codec<S>::R;
    f32x2_t m[Codec<S>::split ? NQ : 1];
    if constexpr (Codec<S>::split) {
        const XLanes xl = xlanes(b, idx);
        if (wave_near_solid(b) || xl_general(xl)) {
            pair_loads<S, true, false>(P, M, n, idx, b, a, c, m);
        } else {
            pair_loads<S, false, true>(P, M, n, idx, b, a, c, m);
            f32x2_t e[NQ];
            xl_loads<f32x2_t>(M, b, xl, e);
            xl_masses<f32x2_t>(xl, e, m);
        }
    } else {
        if (wave_near_solid(b)) pair_loads<S, true, false>(P, M, n, idx, b, a, c, m);
        else pair_loads<S, false, false>(P, M, n, idx, b, a, c, m);
    }
    if constexpr (Codec<S>::split) {
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            a[q] = fma(weight<R>(q), m[q].x, a[q]);
            c[q] = fma(weight<R>(q), m[q].y, c[q]);
        }
    }
}

// Store of both lattices' 19 populations into paired planes (split codecs:
// the masses as in store_all, less the sums of the rounded remainders, one
// pair per cell).
template <class S>
__device__ inline void store_pair(void *P, void *M, uint32_t n, uint32_t idx, const typename Codec<S>::R *a,
                                  const typename Codec<S>::R *c)
{
    using R = typename Codec<S>::R;
    using W = typename PairCodec<S>::W;
    if constexpr (Codec<S>::split) {
        R ma = 0, mc = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            ma += a[q];
            mc += c[q];
        }
        R sa = 0, sc = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const W wd = PairCodec<S>::encode(fma(-weight<R>(q), ma, a[q]), fma(-weight<R>(q), mc, c[q]));
            R ta, tc;
            PairCodec<S>::decode(wd, ta, tc);
            sa += ta;
            sc += tc;
            st(at(plane_w<W>(P, n, q), idx), wd);
        }
        stg<f32x2_t>(M, idx, f32x2_t{ma - sa, mc - sc});
    } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) PairCodec<S>::store(at(plane_w<W>(P, n, q), idx), a[q], c[q]);
    }
}

// Reciprocal, division, square root, reciprocal square root and exponential
// in two forms: HW = false the correctly rounded division and square root and
// the libm-accurate exp, HW = true the hardware instructions (about 1 ulp; a
// quotient as a product with the hardware reciprocal).  FP64
// is always the accurate form.  HwMath<S>: FP32 storage computes with the
// accurate forms (free there: the FP32 steps are bound by HBM, 0.945 ms either
// way at 256^3); the 16-bit storage forms, whose rounding of the stored
// populations is 4-5 orders larger than an ulp of the arithmetic, keep the
// hardware forms (the accurate ones cost the BF16 step 4%).
template <class S> struct HwMath { static constexpr bool value = true; };
template <> struct HwMath<float> { static constexpr bool value = false; };
template <> struct HwMath<double> { static constexpr bool value = false; };

template <bool HW>
__device__ inline float rcp(float x)
{
    if constexpr (HW) return __builtin_amdgcn_rcpf(x);
    else return 1.0f / x;
}
template <bool HW>
__device__ inline double rcp(double x) { return 1.0 / x; }
// a / b: the correctly rounded quotient, or (HW) a times the hardware reciprocal
template <bool HW>
__device__ inline float fdiv(float a, float b)
{
    if constexpr (HW) return a * __builtin_amdgcn_rcpf(b);
    else return a / b;
}
template <bool HW>
__device__ inline double fdiv(double a, double b) { return a / b; }
template <bool HW>
__device__ inline float fsqrt(float x)
{
    if constexpr (HW) return __builtin_amdgcn_sqrtf(x);
    else return sqrtf(x);
}
template <bool HW>
__device__ inline double fsqrt(double x) { return sqrt(x); }
template <bool HW>
__device__ inline float frsq(float x)
{
    if constexpr (HW) return __builtin_amdgcn_rsqf(x);
    else return 1.0f / sqrtf(x);
}
template <bool HW>
__device__ inline double frsq(double x) { return 1.0 / sqrt(x); }
template <bool HW>
__device__ inline float fexp(float x)
{
    if constexpr (HW) return __builtin_amdgcn_exp2f(x * 1.44269504088896341f);
    else return expf(x);
}
template <bool HW>
__device__ inline double fexp(double x) { return exp(x); }

// unsigned division by an invariant divisor (Granlund and Montgomery,
// "Division by invariant integers using multiplication", 1994): the host
// precomputes g = (m, s1, s2); exact for every 32-bit dividend.
__device__ inline uint32_t udiv(uint32_t n, const uint32_t g[3])
{
    const uint32_t t = __umulhi(g[0], n);
    return (t + ((n - t) >> g[1])) >> g[2];
}

// grad(eps) (times eps) by sum_q w_q eps(x + v_q) v_q; a solid neighbour
// takes eps(x).  The caller scales by 3 / eps(x).  BB = false: no cell of the
// wave has a solid neighbour.
template <class R, bool BB, int Q = 1>
__device__ inline void eps_grad_each(const void *E, const Nbr &b, R e0, R &gx, R &gy, R &gz)
{
    R e;
    if constexpr (BB) e = shifted_solid<Q, 1>(b) ? e0 : ldg<R>(E, shifted<Q, 1>(b));
    else e = ldg<R>(E, shifted<Q, 1>(b));
    const R we = weight<R>(Q) * e;
    if (cx(Q)) gx += cx(Q) > 0 ? we : -we;
    if (cy(Q)) gy += cy(Q) > 0 ? we : -we;
    if (cz(Q)) gz += cz(Q) > 0 ? we : -we;
    if constexpr (Q + 1 < NQ) eps_grad_each<R, BB, Q + 1>(E, b, e0, gx, gy, gz);
}

// XS: the x-neighbours' values taken across the wave (nb_rows, nb_edges,
// nb_shift; the sums in the same order, so the result is bitwise the same).
// Kept for the split codecs only: 2% faster there at 256^3, while FP32 ran
// 0.3% slower and the deviation forms the same.
template <class R, bool XS = false>
__device__ inline void eps_grad_acc(const void *E, const Nbr &b, uint32_t idx, R e0, R &gx, R &gy, R &gz)
{
    if constexpr (XS) {
        const XLanes xl = xlanes(b, idx);
        if (!wave_near_solid(b) && !xl_general(xl)) {
            R v[NQ], e[NQ];
            v[0] = e0;
            nb_rows<R>(E, b, v);
            nb_edges<R>(E, b, xl, e);
            nb_shift<R>(xl, e, v);
#pragma unroll
            for (int q = 1; q < NQ; ++q) {
                const R we = weight<R>(q) * v[q];
                if (cx(q)) gx += cx(q) > 0 ? we : -we;
                if (cy(q)) gy += cy(q) > 0 ? we : -we;
                if (cz(q)) gz += cz(q) > 0 ? we : -we;
            }
            return;
        }
        eps_grad_each<R, true>(E, b, e0, gx, gy, gz);
    } else {
        if (wave_near_solid(b)) eps_grad_each<R, true>(E, b, e0, gx, gy, gz);
        else eps_grad_each<R, false>(E, b, e0, gx, gy, gz);
    }
}

// colour gradient, Eq. macros: F = sum_{q != 0} rho_1(x + v_q) v_q
template <class R, int Q = 1>
__device__ inline void colour_acc(const void *C1, const Nbr &b, R &Fx, R &Fy, R &Fz)
{
    const R r = ldg<R>(C1, shifted<Q, 1>(b));
    if (cx(Q)) Fx += cx(Q) > 0 ? r : -r;
    if (cy(Q)) Fy += cy(Q) > 0 ? r : -r;
    if (cz(Q)) Fz += cz(Q) > 0 ? r : -r;
    if constexpr (Q + 1 < NQ) colour_acc<R, Q + 1>(C1, b, Fx, Fy, Fz);
}

template <class R> struct Newton { static constexpr R tol = R(1e-7); };
template <> struct Newton<double> { static constexpr double tol = 1e-15; };

// |V'| of the implicit velocity V'_a = W_a / (lam_a + mu_a |V'|): Newton on
// phi(s) = s - R(s), R(s) = sqrt(sum_a W_a^2 / (lam_a + mu_a s)^2), from the
// Darcy-only value, an upper bound of the root (at most 8 iterations).
// Near the root phi' >= 1 and |phi''| = |R''| <= 3 R max_a (mu_a / (lam_a +
// mu_a s))^2 <= 3 / s, so the error left after an update ds is at most
// 1.5 ds^2 / s: the loop stops once that bound is below the working
// precision (tol s), which saves the iteration that would only confirm it.
template <class R, bool HW>
__device__ inline R solve_speed(const R W[3], const R lam[3], const R mu[3], const R ilam[3])
{
    R s = fsqrt<HW>((W[0] * ilam[0]) * (W[0] * ilam[0]) + (W[1] * ilam[1]) * (W[1] * ilam[1]) +
                (W[2] * ilam[2]) * (W[2] * ilam[2]));
    // the root lies in [s / (1 + max mu s / min lam), s]: when that bracket is
    // below the working precision the Darcy value is the answer
    const R mumax = fmax(mu[0], fmax(mu[1], mu[2]));
    const R lmin = fmin(lam[0], fmin(lam[1], lam[2]));
    if (s > R(0) && mumax * s > Newton<R>::tol * lmin) {
        for (int it = 0; it < 8; ++it) {
            R R2 = 0, dR = 0;
#pragma unroll
            for (int a = 0; a < 3; ++a) {
                const R id = rcp<HW>(lam[a] + mu[a] * s);
                const R t = W[a] * id;
                R2 += t * t;
                dR += t * t * mu[a] * id;
            }
            const R Rn = fsqrt<HW>(R2);
            const R phi = s - Rn;
            const R dphi = R(1) + (Rn > R(0) ? fdiv<HW>(dR, Rn) : R(0));
            const R ds = fdiv<HW>(phi, dphi);
            s = s - ds;
            s = s > R(0) ? s : R(0);
            if (!(R(1.5) * ds * ds > Newton<R>::tol * s * s)) break;
        }
    }
    return s;
}

// Moments after streaming; populations in deviation form.  Directions come
// in opposite pairs (q, q+1), q odd: their sum feeds the density, their
// difference the momentum.
template <class R, int P = 0>
__device__ inline void moments_acc(const R *d, R &drho, R &jx, R &jy, R &jz)
{
    constexpr int q = 2 * P + 1;
    if constexpr (P == 0) drho += d[0];
    const R s = d[q] + d[q + 1], t = d[q] - d[q + 1];
    drho += s;
    if (cx(q)) jx += cx(q) > 0 ? t : -t;
    if (cy(q)) jy += cy(q) > 0 ? t : -t;
    if (cz(q)) jz += cz(q) > 0 ? t : -t;
    if constexpr (P + 1 < (NQ - 1) / 2) moments_acc<R, P + 1>(d, drho, jx, jy, jz);
}

template <class R, int Q>
__device__ inline R cdot(const R v[3])
{
    R r = R(0);
    bool any = false;
    if constexpr (cx(Q) != 0) { r = cx(Q) > 0 ? v[0] : -v[0]; any = true; }
    if constexpr (cy(Q) != 0) { r = any ? (cy(Q) > 0 ? r + v[1] : r - v[1]) : (cy(Q) > 0 ? v[1] : -v[1]); any = true; }
    if constexpr (cz(Q) != 0) { r = any ? (cz(Q) > 0 ? r + v[2] : r - v[2]) : (cz(Q) > 0 ? v[2] : -v[2]); }
    return r;
}

// Per-cell constants of the collision.  The BGK update with the equilibria
// of Eqs. equilc1/2 and the forcing of Eq. coeffforce1 (weight w_q rho),
//   d' = d - omega (d - f^eq) + w rho T,
// is rearranged (exactly, in real arithmetic) as
//   d' = (1 - omega) d + omega w drho + w rho X_q + omega w ST_q,
//   X_q = 3 (v.a + v.b) + (v.u)(k45 v.a + k9 v.b) - K0,
// with a = omega u, b = (1 - omega/2) F^ext, k45 = 4.5/eps, k9 = 9/eps,
// K0 = omega 1.5 |u|^2 / eps + (1 - omega/2) 3 u.F^ext / eps.
template <class R>
struct Coll {
    R om1;                  // 1 - omega
    R u[3], a[3], b[3];
    R k45, k9, K0;
    R base[3], wr[3];       // per weight class: omega w drho (+ surface-tension constant), w rho
    R F[3], s1[3];          // colour gradient; per class omega w A eps tau / |F|
};

template <class R>
__device__ inline Coll<R> make_coll(R drho, R rho, R omega, R ie, const R u[3], const R Fx[3], R st,
                                    const R F[3], R Fn, R iFn)
{
    Coll<R> c;
    const R pre = R(1) - R(0.5) * omega;
    c.om1 = R(1) - omega;
    R uu = 0, uF = 0;
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        c.u[a] = u[a];
        c.a[a] = omega * u[a];
        c.b[a] = pre * Fx[a];
        c.F[a] = F[a];
        uu += u[a] * u[a];
        uF += u[a] * Fx[a];
    }
    c.k45 = R(4.5) * ie;
    c.k9 = R(9) * ie;
    c.K0 = omega * R(1.5) * ie * uu + pre * R(3) * ie * uF;
    const R w[3] = {weight<R>(0), weight<R>(1), weight<R>(7)};
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const R ost = omega * w[k] * st;          // omega w A eps tau (0 without |F|)
        c.wr[k] = w[k] * rho;
        c.base[k] = omega * w[k] * drho + (k == 0 ? ost * Fn : -ost * Fn);
        c.s1[k] = ost * iFn;
    }
    return c;
}

// Directions q (odd) and q+1 are opposite: with S = v.a + v.b and
// P = (v.u)(k45 v.a + k9 v.b) - K0 computed once, X_q = P + 3 S and
// X_{q+1} = P - 3 S (all dot products change sign, the quadratic term not).
template <class R, bool ST, int P = 0>
__device__ inline void collide_f(R *d, const Coll<R> &c)
{
    constexpr int q = 2 * P + 1, k = q <= 6 ? 1 : 2;
    if constexpr (P == 0) d[0] = fma(c.om1, d[0], c.base[0] - c.wr[0] * c.K0);
    const R cu = cdot<R, q>(c.u), ca = cdot<R, q>(c.a), cb = cdot<R, q>(c.b);
    const R S = ca + cb;
    const R Pq = fma(cu, fma(c.k45, ca, c.k9 * cb), -c.K0);
    R vq = fma(c.wr[k], fma(R(3), S, Pq), c.base[k]);
    R vo = fma(c.wr[k], fma(R(-3), S, Pq), c.base[k]);
    if constexpr (ST) {
        const R cG = cdot<R, q>(c.F);
        const R t = c.s1[k] * cG;
        vq = fma(t, cG, vq);
        vo = fma(t, cG, vo);
    }
    d[q] = fma(c.om1, d[q], vq);
    d[q + 1] = fma(c.om1, d[q + 1], vo);
    if constexpr (P + 1 < (NQ - 1) / 2) collide_f<R, ST, P + 1>(d, c);
}

// Solute BGK (Eqs. equild, boltzeqD):
// h' = (1 - omega_D) h + omega_D w eps C (1 + 3 v.V*), opposite pairs together.
template <class R, int P = 0>
__device__ inline void collide_h(R *h, R om1d, const R H[3], const R vs[3])
{
    constexpr int q = 2 * P + 1, k = q <= 6 ? 1 : 2;
    if constexpr (P == 0) h[0] = fma(om1d, h[0], H[0]);
    const R t = R(3) * H[k] * cdot<R, q>(vs);
    h[q] = fma(om1d, h[q], H[k] + t);
    h[q + 1] = fma(om1d, h[q + 1], H[k] - t);
    if constexpr (P + 1 < (NQ - 1) / 2) collide_h<R, P + 1>(h, om1d, H, vs);
}

// Two-fluid recolouring: g' = C f' + beta C (1 - C) rho w cos(v, F).
template <class R, int P = 0>
__device__ inline void recolour(R *g, const R *d, R C, const R Cw[3], const R rw[3], const R F[3])
{
    constexpr int q = 2 * P + 1, k = q <= 6 ? 1 : 2;
    if constexpr (P == 0) g[0] = fma(C, d[0], Cw[0]);
    const R t = rw[k] * cdot<R, q>(F);
    g[q] = fma(C, d[q], Cw[k]) + t;
    g[q + 1] = fma(C, d[q + 1], Cw[k]) - t;
    if constexpr (P + 1 < (NQ - 1) / 2) recolour<R, P + 1>(g, d, C, Cw, rw, F);
}

// Porous velocity and force (Eqs. forcement, expandV, expandVsub with eps on
// G, diagonal K, optional Forchheimer drag).  G is the body force in the
// frame of kinv.
template <class R, bool HW>
__device__ inline void porous_core(const LatDev *L, const R G[3], R eps, const R kinv[3], R nu, const R V[3],
                                   R u[3], R Fx[3])
{
    R W[3], lam[3], ilam[3], mu[3], sk[3];
    R Feps = R(0);
    const bool forch = L->forch != 0;
    if (forch) Feps = R(1.75) * frsq<HW>(R(150) * eps * eps * eps);
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        W[a] = V[a] + R(0.5) * eps * G[a];
        lam[a] = R(1) + R(0.5) * eps * nu * kinv[a];
        ilam[a] = rcp<HW>(lam[a]);
        sk[a] = forch ? fsqrt<HW>(kinv[a]) : R(0);
        mu[a] = R(0.5) * eps * Feps * sk[a];
    }
    if (forch) {
        const R s = solve_speed<R, HW>(W, lam, mu, ilam);
#pragma unroll
        for (int a = 0; a < 3; ++a) u[a] = W[a] * rcp<HW>(lam[a] + mu[a] * s);
    } else {
#pragma unroll
        for (int a = 0; a < 3; ++a) u[a] = W[a] * ilam[a];
    }
    const R sp = forch ? fsqrt<HW>(u[0] * u[0] + u[1] * u[1] + u[2] * u[2]) : R(0);
#pragma unroll
    for (int a = 0; a < 3; ++a)
        Fx[a] = eps * G[a] - eps * nu * kinv[a] * u[a] - eps * Feps * sp * sk[a] * u[a];
}

template <class R, bool HW>
__device__ inline void porous_force(const LatDev *L, R eps, const R kinv[3], R nu, const R V[3], R u[3], R Fx[3])
{
    const R G[3] = {R(L->G[0]), R(L->G[1]), R(L->G[2])};
    porous_core<R, HW>(L, G, eps, kinv, nu, V, u, Fx);
}

// Rotation matrix (columns: the eigenvectors of K^-1) of a unit quaternion
// (w, x, y, z).
template <class R>
__device__ inline void quat_matrix(const R q[4], R M[3][3])
{
    const R w = q[0], x = q[1], y = q[2], z = q[3];
    M[0][0] = R(1) - R(2) * (y * y + z * z);
    M[0][1] = R(2) * (x * y - z * w);
    M[0][2] = R(2) * (x * z + y * w);
    M[1][0] = R(2) * (x * y + z * w);
    M[1][1] = R(1) - R(2) * (x * x + z * z);
    M[1][2] = R(2) * (y * z - x * w);
    M[2][0] = R(2) * (x * z - y * w);
    M[2][1] = R(2) * (y * z + x * w);
    M[2][2] = R(1) - R(2) * (x * x + y * y);
}

// Full tensor K^-1 = Q diag(mu) Q^T: K^-1 and K^-1/2 share the frame Q, so in
// that frame Eqs. forcement and expandV (with the Forchheimer drag) are the
// diagonal ones.  V and G are rotated in, V' and F^ext rotated back.
template <class R, bool HW>
__device__ inline void porous_force_frame(const LatDev *L, R eps, const R q[4], const R mu[3], R nu, const R V[3],
                                          R u[3], R Fx[3])
{
    R M[3][3];
    quat_matrix<R>(q, M);
    R Vr[3], Gr[3];
    const R G[3] = {R(L->G[0]), R(L->G[1]), R(L->G[2])};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        Vr[a] = M[0][a] * V[0] + M[1][a] * V[1] + M[2][a] * V[2];
        Gr[a] = M[0][a] * G[0] + M[1][a] * G[1] + M[2][a] * G[2];
    }
    R ur[3], Fr[3];
    porous_core<R, HW>(L, Gr, eps, mu, nu, Vr, ur, Fr);
    // F^ext = eps G - Q (drag in the frame); eps G exactly, the drag rotated back
    R Dr[3];
#pragma unroll
    for (int a = 0; a < 3; ++a) Dr[a] = eps * Gr[a] - Fr[a];
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        u[a] = M[a][0] * ur[0] + M[a][1] * ur[1] + M[a][2] * ur[2];
        Fx[a] = eps * G[a] - (M[a][0] * Dr[0] + M[a][1] * Dr[1] + M[a][2] * Dr[2]);
    }
}

// ---------------------------------------------------------------------------
// FP64 block reduction of the diagnostic partial sums: wave64 butterfly,
// then the waves of the block in a fixed order.  Deterministic.
__device__ inline void block_reduce_store(double v[NPART], double *out)
{
    __shared__ double red[BLOCK / 64][NPART];
#pragma unroll
    for (int k = 0; k < NPART; ++k) {
        double x = v[k];
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double y = __shfl_xor(x, o, 64);
            x = (k == 7) ? fmax(x, y) : x + y;
        }
        v[k] = x;
    }
    const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
    if (lane == 0) {
#pragma unroll
        for (int k = 0; k < NPART; ++k) red[wv][k] = v[k];
    }
    __syncthreads();
    if (threadIdx.x < NPART) {
        const int k = threadIdx.x;
        double acc = red[0][k];
        for (int w = 1; w < BLOCK / 64; ++w) acc = (k == 7) ? fmax(acc, red[w][k]) : acc + red[w][k];
        out[k] = acc;
    }
}

// per-cell contribution: {rho, rho u (3), eps C | rho_1 | 0, |u - u_prev|^2,
// |u|^2, |u| (max), non-finite}
template <class R>
__device__ inline void diag_contrib(double v[NPART], R rho, const R u[3], R C, R s4, const R up[3])
{
    const bool fin = isfinite(rho) && isfinite(u[0]) && isfinite(u[1]) && isfinite(u[2]) && isfinite(C);
    // a non-finite cell only counts as such (selects, no branch)
    const double r = fin ? double(rho) : 0.0;
    const double ux = fin ? double(u[0]) : 0.0, uy = fin ? double(u[1]) : 0.0, uz = fin ? double(u[2]) : 0.0;
    const double px = fin ? double(up[0]) : 0.0, py = fin ? double(up[1]) : 0.0, pz = fin ? double(up[2]) : 0.0;
    v[0] = r;
    v[1] = r * ux;
    v[2] = r * uy;
    v[3] = r * uz;
    v[4] = fin ? double(s4) : 0.0;
    const double dx = ux - px, dy = uy - py, dz = uz - pz;
    v[5] = dx * dx + dy * dy + dz * dz;
    v[6] = ux * ux + uy * uy + uz * uz;
    v[7] = sqrt(v[6]);
    v[8] = fin ? 0.0 : 1.0;
}

// ---------------------------------------------------------------------------
// The step kernel: pull-stream both lattices, moments, viscosity, porous
// force, (colour gradient), collide, write the other copy.  FT: every lattice
// of the launch has a full permeability tensor (eigenframe form).  MS
// (miscible): the lattices may carry further solutes, updated after the
// first with the same V' (a runtime count per lattice, possibly 0).
// Waves per SIMD the step is compiled for.  The miscible step with plain
// 16-bit storage (diagonal K, one solute) fits in 95 VGPRs at 5 waves without
// spills and runs 5-18% faster there at 256^3 and 7-9% at 512^3.  The split
// forms (19 pair words and 9 + 5 mass-pair loads per pull) take 100-104 VGPRs
// and run at 4 waves: forced to 5, FP16 split spills a little and runs as fast,
// BF16 split spills more and runs 17% slower (with 19 mass loads both spilled,
// and issuing the pull in two halves to fit 5 waves measured 3% slower).
// Every other form keeps the compiler's own choice (1 = no constraint; the
// FP32 and FP64 code is the same as without the attribute).
template <int PHYS, class S, bool FT, bool MS> struct StepWaves { static constexpr int value = 1; };
template <> struct StepWaves<PH_MISCIBLE, bf16_t, false, false> { static constexpr int value = 5; };
template <> struct StepWaves<PH_MISCIBLE, f16_t, false, false> { static constexpr int value = 5; };
template <> struct StepWaves<PH_MISCIBLE, bf16s_t, false, false> { static constexpr int value = 4; };
template <> struct StepWaves<PH_MISCIBLE, f16s_t, false, false> { static constexpr int value = 4; };

template <int PHYS, class S, bool FT = false, bool MS = false>
__global__ PLBM_STEP_ATTR __attribute__((amdgpu_waves_per_eu(StepWaves<PHYS, S, FT, MS>::value))) void k_step(
    const BatchArgs a)
{
    using R = typename Codec<S>::R;
    constexpr bool HW = HwMath<S>::value;
    const int gb = xcd_remap(blockIdx.x, a.total_blocks);
    const int l = find_lattice(a, gb);
    const LatDev *__restrict__ L = a.lat[l];
    const int lb = step_block(gb - a.blk_start[l], a.blk_start[l + 1] - a.blk_start[l], L);
    if (lb < 0) return;   // padding of the lattice's block range (uniform over the block)
    const int flags = a.flags[l];
    const int src = flags & 1;
    const bool mom = (flags & 2) != 0;
    const R nuc = R(a.nuc[l]);

    const uint32_t ncell = L->ncell;
    const uint32_t idx = uint32_t(lb) * BLOCK + threadIdx.x;
    const uint32_t nx = L->nx, nxy = nx * uint32_t(L->ny);

    // moments kept for the diagnostics of this step
    bool has = false;
    R m_rho = 0, m_C = 0, m_s4 = 0, m_u[3] = {0, 0, 0}, m_up[3] = {0, 0, 0};
    int type = CELL_SOLID;
    int x = 0, y = 0, z = 0, face = -1;
    uint32_t lw = 0;
    if (idx < ncell) {
        z = udiv(idx, L->div_nxy);
        const uint32_t r = idx - uint32_t(z) * nxy;
        y = udiv(r, L->div_nx);
        x = r - uint32_t(y) * nx;
        lw = link_word(L, idx);
        type = cell_type(L, x, y, z, lw, face);
    }
    // Post-collision populations of both lattices.  Every cell of the box
    // stores them: fluid cells their update, reservoir cells their fixed
    // state (bitwise the set-up values), solid cells zeros.  Lanes that
    // skipped their stores would leave partially written cache lines at the
    // two reservoir cells of every x-row and at every obstacle, which
    // measured up to 30% slower (narrow rows) than the extra bytes.
    R d[NQ], hq[NQ];
    const int dst = src ^ 1;
    // what the further solutes take from the fluid branch
    [[maybe_unused]] Nbr bx{};
    [[maybe_unused]] R x_eps = 1, x_ie = 1, x_u[3] = {0, 0, 0}, x_g[3] = {0, 0, 0};
    if (type == CELL_FLUID) {
        const Nbr b = neighbours(L, x, y, z, lw);
        if constexpr (paired_v<PHYS, S>) {
            pull_pair<S>(L->f[src], L->fm[src], L->ppstride, idx, b, d, hq);
        } else {
            pull_all<S>(L->f[src], L->fm[src], L->pstride, idx, b, d);
            if constexpr (PHYS == PH_MISCIBLE) pull_all<S>(L->h[src], L->hm[src], L->pstride, idx, b, hq);
        }

        R drho = 0, jx = 0, jy = 0, jz = 0;
        moments_acc<R>(d, drho, jx, jy, jz);
        const R rho = R(1) + drho;
        const R irho = rcp<HW>(rho);
        const R V[3] = {jx * irho, jy * irho, jz * irho};

        const R eps = L->uniform_eps ? R(L->eps_u) : ldg<R>(L->eps, idx);
        const R ie = rcp<HW>(eps);

        R sh = 0, rho1 = 0, C = 0;
        if constexpr (PHYS == PH_MISCIBLE) {
#pragma unroll
            for (int q = 0; q < NQ; ++q) sh += hq[q];
            C = sh * ie;
        } else if constexpr (PHYS == PH_IMMISCIBLE) {
            rho1 = ldg<R>(L->rho1, idx);
            C = rho1 * irho;
        }

        R nu;
        if constexpr (PHYS == PH_IMMISCIBLE) {
            nu = C * R(L->nu1) + (R(1) - C) * R(L->nu2);
        } else if constexpr (PHYS == PH_MISCIBLE) {
            nu = nuc * fexp<HW>(R(L->k1) * C + R(L->k0));
        } else {
            nu = nuc * fexp<HW>(R(L->k0));
        }
        const R tau = R(0.5) + R(3) * nu;
        const R omega = rcp<HW>(tau);

        R u[3], Fx[3];
        if constexpr (FT) {
            const R q[4] = {ldg<R>(L->kinv, idx), ldp<R>(L->kinv, ncell, 1, idx), ldp<R>(L->kinv, ncell, 2, idx),
                            ldp<R>(L->kinv, ncell, 3, idx)};
            const R mu[3] = {ldp<R>(L->kinv, ncell, 4, idx), ldp<R>(L->kinv, ncell, 5, idx),
                             ldp<R>(L->kinv, ncell, 6, idx)};
            porous_force_frame<R, HW>(L, eps, q, mu, nu, V, u, Fx);
        } else {
            R kinv[3];
            if (L->uniform_kinv) {
                kinv[0] = R(L->kinv_u[0]);
                kinv[1] = R(L->kinv_u[1]);
                kinv[2] = R(L->kinv_u[2]);
            } else {
                kinv[0] = ldg<R>(L->kinv, idx);
                kinv[1] = ldp<R>(L->kinv, ncell, 1, idx);
                kinv[2] = ldp<R>(L->kinv, ncell, 2, idx);
            }
            porous_force<R, HW>(L, eps, kinv, nu, V, u, Fx);
        }

        R F[3] = {0, 0, 0};
        R Fn = 0, iFn = 0, st = 0;
        if constexpr (PHYS == PH_IMMISCIBLE) {
            colour_acc<R>(L->rho1, b, F[0], F[1], F[2]);
            Fn = sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]);
            iFn = Fn > R(0) ? rcp<HW>(Fn) : R(0);
            st = Fn > R(0) ? R(L->A) * eps * tau : R(0);
        }
        const Coll<R> cl = make_coll<R>(drho, rho, omega, ie, u, Fx, st, F, Fn, iFn);
        collide_f<R, PHYS == PH_IMMISCIBLE>(d, cl);

        if constexpr (PHYS == PH_MISCIBLE) {
            R vs[3] = {u[0], u[1], u[2]};
            if (L->eps_grad && !L->uniform_eps) {
                R gx = 0, gy = 0, gz = 0;
                eps_grad_acc<R, Codec<S>::split>(L->eps, b, idx, eps, gx, gy, gz);
                const R k = R(3) * R(L->D) * ie;
                vs[0] += k * gx;
                vs[1] += k * gy;
                vs[2] += k * gz;
                if constexpr (MS) {
                    x_g[0] = gx;
                    x_g[1] = gy;
                    x_g[2] = gz;
                }
            }
            if constexpr (MS) {
                bx = b;
                x_eps = eps;
                x_ie = ie;
                for (int c = 0; c < 3; ++c) x_u[c] = u[c];
            }
            const R omd = fdiv<HW>(R(1), R(L->tau_d));
            const R H[3] = {omd * weight<R>(0) * sh, omd * weight<R>(1) * sh, omd * weight<R>(7) * sh};
            collide_h<R>(hq, R(1) - omd, H, vs);
        } else if constexpr (PHYS == PH_IMMISCIBLE) {
            const R rec = Fn > R(0) ? R(L->beta) * C * (R(1) - C) * rho * iFn : R(0);
            const R Cw[3] = {C * weight<R>(0), C * weight<R>(1), C * weight<R>(7)};
            const R rw[3] = {R(0), rec * weight<R>(1), rec * weight<R>(7) * R(0.70710678118654752440)};
            recolour<R>(hq, d, C, Cw, rw, F);
        }

        if (mom) {
            void *M = L->mom;
            const R up[3] = {ldp<R>(M, ncell, 1, idx), ldp<R>(M, ncell, 2, idx), ldp<R>(M, ncell, 3, idx)};
            stg<R>(M, idx, rho);
            stp<R>(M, ncell, 1, idx, u[0]);
            stp<R>(M, ncell, 2, idx, u[1]);
            stp<R>(M, ncell, 3, idx, u[2]);
            stp<R>(M, ncell, 4, idx, C);
            has = true;
            m_rho = rho;
            m_C = C;
            m_s4 = PHYS == PH_MISCIBLE ? sh : (PHYS == PH_IMMISCIBLE ? rho1 : R(0));
            for (int k = 0; k < 3; ++k) {
                m_u[k] = u[k];
                m_up[k] = up[k];
            }
        }
    } else if (type == CELL_RES) {
        // the fixed reservoir state, as set up: f^eq(rho_bc, V' = 0) and
        // h^eq(eps C_bc, 0) or g = C_bc f
        // rho_bc - 1 is formed in double before rounding (1 + 3 x 0.0441 in
        // FP32 minus 1 would carry the FP32 error of 1.1323, 1.5e-7 of drho)
        const R rb = R(L->face_rho[face]), cb = R(L->face_conc[face]), drb = R(L->face_rho[face] - 1.0);
        R eps = R(1);
        if constexpr (PHYS == PH_MISCIBLE) eps = L->uniform_eps ? R(L->eps_u) : ldg<R>(L->eps, idx);
        if constexpr (MS) x_eps = eps;
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const R w = weight<R>(q);
            d[q] = w * drb;
            hq[q] = PHYS == PH_MISCIBLE ? w * eps * cb : (PHYS == PH_IMMISCIBLE ? cb * w * rb : R(0));
        }
    } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) d[q] = hq[q] = R(0);
    }
    // waves made of solid cells only (wall planes, obstacle interiors) skip
    if (idx < ncell && __builtin_amdgcn_ballot_w64(type != CELL_SOLID) != 0) {
        if constexpr (paired_v<PHYS, S>) {
            store_pair<S>(L->f[dst], L->fm[dst], L->ppstride, idx, d, hq);
        } else {
            if constexpr (PHYS != PH_SINGLE) store_all<S>(L->h[dst], L->hm[dst], L->pstride, idx, hq);
            store_all<S>(L->f[dst], L->fm[dst], L->pstride, idx, d);
        }
    }
    if constexpr (MS) {
        // further solutes: the first solute's update with their own D, tau_d
        // and reservoir concentrations, one at a time
        const GL MsDev *X = ms_of(L);
        const int nsx = X ? X->nsx : 0;
        for (int k = 0; k < nsx; ++k) {
            R hk[NQ];
            if (type == CELL_FLUID) {
                // an opaque copy of the neighbour offsets: without it the
                // compiler hoists the 18 (split codecs: 36) per-link byte
                // offsets out of the loop and keeps them live across it (split
                // forms 211-218 VGPRs, 2 waves per SIMD); computed inside,
                // every form fits in 116-120 and runs 4 waves
                Nbr bk = bx;
                asm volatile("" : "+v"(bk.xm), "+v"(bk.x0), "+v"(bk.xp), "+v"(bk.ym), "+v"(bk.y0), "+v"(bk.yp),
                             "+v"(bk.zm), "+v"(bk.z0), "+v"(bk.zp), "+v"(bk.bb));
                pull_all<S>(X->h[k][src], X->hm[k][src], L->pstride, idx, bk, hk);
                R sh = 0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) sh += hk[q];
                const R kk = R(3) * R(X->D[k]) * x_ie;
                const R vs[3] = {x_u[0] + kk * x_g[0], x_u[1] + kk * x_g[1], x_u[2] + kk * x_g[2]};
                const R omd = fdiv<HW>(R(1), R(X->tau_d[k]));
                const R H[3] = {omd * weight<R>(0) * sh, omd * weight<R>(1) * sh, omd * weight<R>(7) * sh};
                collide_h<R>(hk, R(1) - omd, H, vs);
                if (mom) stp<R>(L->mom, ncell, 5 + k, idx, sh * x_ie);
            } else if (type == CELL_RES) {
                const R cb = R(X->face_conc[k][face]);
#pragma unroll
                for (int q = 0; q < NQ; ++q) hk[q] = weight<R>(q) * x_eps * cb;
            } else {
#pragma unroll
                for (int q = 0; q < NQ; ++q) hk[q] = R(0);
            }
            if (idx < ncell && __builtin_amdgcn_ballot_w64(type != CELL_SOLID) != 0)
                store_all<S>(X->h[k][dst], X->hm[k][dst], L->pstride, idx, hk);
        }
    }
    if (mom) {
        double part[NPART] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
        if (has) diag_contrib<R>(part, m_rho, m_u, m_C, m_s4, m_up);
        block_reduce_store(part, L->partials + size_t(lb) * NPART);
    }
}

// Two-fluid, first pass of a step: the colour field rho_1 of the step being
// computed (fluid cells: sum of the streamed g; reservoir cells: C_bc rho_bc;
// solid cells: the wall colour (1 + cos theta)/2), which the step kernel
// reads at the 18 neighbours for the colour gradient.
template <class S>
__global__ __launch_bounds__(BLOCK) void k_colour(const BatchArgs a)
{
    using R = typename Codec<S>::R;
    const int gb = xcd_remap(blockIdx.x, a.total_blocks);
    const int l = find_lattice(a, gb);
    const LatDev *__restrict__ L = a.lat[l];
    const int lb = step_block(gb - a.blk_start[l], a.blk_start[l + 1] - a.blk_start[l], L);
    if (lb < 0) return;   // padding of the lattice's block range
    const int src = a.flags[l] & 1;
    const uint32_t ncell = L->ncell;
    const uint32_t idx = uint32_t(lb) * BLOCK + threadIdx.x;
    if (idx >= ncell) return;
    const uint32_t nx = L->nx, nxy = nx * uint32_t(L->ny);
    const int z = udiv(idx, L->div_nxy);
    const uint32_t r = idx - uint32_t(z) * nxy;
    const int y = udiv(r, L->div_nx);
    const int x = r - uint32_t(y) * nx;
    int face;
    const uint32_t lw = link_word(L, idx);
    const int type = cell_type(L, x, y, z, lw, face);
    R v;
    if (type == CELL_SOLID) {
        v = R(L->face_cw[face]);
    } else if (type == CELL_RES) {
        v = R(L->face_conc[face]) * R(L->face_rho[face]);
    } else {
        const Nbr b = neighbours(L, x, y, z, lw);
        R g[NQ];
        pull_all<S>(L->h[src], L->hm[src], L->pstride, idx, b, g);
        v = 0;
#pragma unroll
        for (int q = 0; q < NQ; ++q) v += g[q];
    }
    stg<R>(L->rho1, idx, v);
}

// Second stage of the diagnostics: one block per lattice sums the per-block
// partials in a fixed order.
__global__ __launch_bounds__(BLOCK) void k_diag_final(const BatchArgs a)
{
    const int l = blockIdx.x;
    const LatDev *__restrict__ L = a.lat[l];
    // four independent partial rows per iteration keep 36 loads in flight
    constexpr int U = 4;
    double w[U][NPART];
#pragma unroll
    for (int u = 0; u < U; ++u)
#pragma unroll
        for (int k = 0; k < NPART; ++k) w[u][k] = 0.0;
    const int nb = L->nblocks;
    for (int bk0 = threadIdx.x; bk0 < nb; bk0 += U * BLOCK) {
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int bk = bk0 + u * BLOCK;
            if (bk < nb) {
                const double *p = L->partials + size_t(bk) * NPART;
#pragma unroll
                for (int k = 0; k < NPART; ++k) w[u][k] = (k == 7) ? fmax(w[u][k], p[k]) : w[u][k] + p[k];
            }
        }
    }
    double v[NPART];
#pragma unroll
    for (int k = 0; k < NPART; ++k)
        v[k] = (k == 7) ? fmax(fmax(w[0][k], w[1][k]), fmax(w[2][k], w[3][k]))
                        : (w[0][k] + w[1][k]) + (w[2][k] + w[3][k]);
    __shared__ double out[NPART];
    block_reduce_store(v, out);
    __syncthreads();
    if (threadIdx.x == 0) {
        double *D = L->diag;
        for (int k = 0; k < 5; ++k) D[k] = out[k];
        D[5] = out[6] > 0.0 ? out[5] / out[6] : 0.0;
        D[6] = out[7];
        D[7] = out[8];
    }
}

// ---------------------------------------------------------------------------
// set-up kernels

template <class R>
struct InitArgs {
    const LatDev *L;
    const R *rho0, *vel0, *c0;   // NULL: uniform defaults 1, 0, 0
    double nuc0;                 // nu0 * min(a0 + a1, cap): time factor at t = 0
};

template <class R>
__device__ inline bool bad(R v) { return !isfinite(v); }

// Link words of the obstacle mask: bit 0 = the cell is solid (wall face or
// mask), bit q = the cell x - v_q is solid (periodic axes wrap).  Cells on
// the face plane of a non-periodic axis are never fluid and get bit 0 only.
// solid may be null (no obstacles: the words then encode the walls alone).
__global__ __launch_bounds__(BLOCK) void k_links(const LatDev *L, const unsigned char *solid, uint32_t *links)
{
    const uint32_t idx = blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= uint32_t(L->ncell)) return;
    const int n[3] = {L->nx, L->ny, L->nz};
    const uint32_t nxy = uint32_t(n[0]) * uint32_t(n[1]);
    const int z = idx / nxy;
    const uint32_t r = idx - uint32_t(z) * nxy;
    const int y = r / n[0], x = r - uint32_t(y) * n[0];
    const int c[3] = {x, y, z};
    const uint32_t on = faces_of(L, x, y, z);
    const bool edge = (on & (L->wall_faces | L->res_faces)) != 0;
    const bool wall = (on & L->wall_faces) != 0;
    uint32_t w = (wall || (solid && solid[idx])) ? 1u : 0u;
    if (!edge) {
        for (int q = 1; q < NQ; ++q) {
            const int d[3] = {cx(q), cy(q), cz(q)};
            int u[3];
            bool s = false;
            for (int a = 0; a < 3; ++a) {
                u[a] = c[a] - d[a];
                if (u[a] < 0) u[a] += n[a];
                if (u[a] >= n[a]) u[a] -= n[a];
                if (((L->wall_faces >> (2 * a)) & 1u) && u[a] == 0) s = true;
                if (((L->wall_faces >> (2 * a + 1)) & 1u) && u[a] == n[a] - 1) s = true;
            }
            const uint32_t j = uint32_t(u[0]) + uint32_t(n[0]) * (uint32_t(u[1]) + uint32_t(n[1]) * uint32_t(u[2]));
            if (s || (solid && solid[j])) w |= 1u << q;
        }
    }
    links[idx] = w;
}

// Eigen-decomposition of a symmetric 3x3 matrix A = V diag(d) V^T by the
// classical Jacobi method (rotate away the largest off-diagonal entry until
// all are negligible; Golub and Van Loan, Matrix Computations, Sec. 8.5).
__device__ inline void sym_eig3(double A[3][3], double d[3], double V[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) V[i][j] = i == j ? 1.0 : 0.0;
    for (int it = 0; it < 64; ++it) {
        int p = 0, q = 1;
        double big = fabs(A[0][1]);
        if (fabs(A[0][2]) > big) { p = 0; q = 2; big = fabs(A[0][2]); }
        if (fabs(A[1][2]) > big) { p = 1; q = 2; big = fabs(A[1][2]); }
        if (big == 0.0 || big <= 1e-18 * (fabs(A[p][p]) + fabs(A[q][q]))) break;
        const double h = A[q][q] - A[p][p];
        const double th = 0.5 * h / A[p][q];
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
        const double c = 1.0 / sqrt(1.0 + t * t), sn = t * c;
        for (int k = 0; k < 3; ++k) {
            const double kp = A[k][p], kq = A[k][q];
            A[k][p] = c * kp - sn * kq;
            A[k][q] = sn * kp + c * kq;
        }
        for (int k = 0; k < 3; ++k) {
            const double pk = A[p][k], qk = A[q][k];
            A[p][k] = c * pk - sn * qk;
            A[q][k] = sn * pk + c * qk;
        }
        for (int k = 0; k < 3; ++k) {
            const double vp = V[k][p], vq = V[k][q];
            V[k][p] = c * vp - sn * vq;
            V[k][q] = sn * vp + c * vq;
        }
    }
    for (int i = 0; i < 3; ++i) d[i] = A[i][i];
}

// Full permeability tensor, set-up: K^-1 given as 6 planes {xx, yy, zz, xy,
// xz, yz} becomes the unit quaternion of its eigenframe (planes 0-3 of the
// lattice's K^-1 section, a proper rotation) and its eigenvalues (planes 4-6),
// in FP64 before rounding to the real type.  Non-solid cells with a
// non-finite or not positive semi-definite K^-1 set the error flag.
template <class R>
__global__ __launch_bounds__(BLOCK) void k_frame(const LatDev *L, const R *kin)
{
    const uint32_t ncell = L->ncell;
    const uint32_t idx = blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= ncell) return;
    const size_t n = ncell;
    double A[3][3], k[6];
    bool fin = true;
    for (int c = 0; c < 6; ++c) {
        k[c] = double(kin[c * n + idx]);
        fin = fin && isfinite(k[c]);
    }
    if (!fin) for (int c = 0; c < 6; ++c) k[c] = 0.0;
    A[0][0] = k[0]; A[1][1] = k[1]; A[2][2] = k[2];
    A[0][1] = A[1][0] = k[3];
    A[0][2] = A[2][0] = k[4];
    A[1][2] = A[2][1] = k[5];
    double d[3], V[3][3];
    sym_eig3(A, d, V);
    const double dmax = fmax(fabs(d[0]), fmax(fabs(d[1]), fabs(d[2])));
    bool psd = true;
    for (int a = 0; a < 3; ++a) {
        if (d[a] < -1e-12 * dmax) psd = false;
        d[a] = fmax(d[a], 0.0);
    }
    // proper rotation: flip the last eigenvector if det V = -1
    const double det = V[0][0] * (V[1][1] * V[2][2] - V[1][2] * V[2][1]) -
                       V[0][1] * (V[1][0] * V[2][2] - V[1][2] * V[2][0]) +
                       V[0][2] * (V[1][0] * V[2][1] - V[1][1] * V[2][0]);
    if (det < 0.0)
        for (int r = 0; r < 3; ++r) V[r][2] = -V[r][2];
    // quaternion of the rotation V (Shepperd's branch on the largest term)
    double w, x, y, z;
    const double tr = V[0][0] + V[1][1] + V[2][2];
    if (tr > 0.0) {
        const double S = 2.0 * sqrt(tr + 1.0);
        w = 0.25 * S; x = (V[2][1] - V[1][2]) / S; y = (V[0][2] - V[2][0]) / S; z = (V[1][0] - V[0][1]) / S;
    } else if (V[0][0] > V[1][1] && V[0][0] > V[2][2]) {
        const double S = 2.0 * sqrt(1.0 + V[0][0] - V[1][1] - V[2][2]);
        w = (V[2][1] - V[1][2]) / S; x = 0.25 * S; y = (V[0][1] + V[1][0]) / S; z = (V[0][2] + V[2][0]) / S;
    } else if (V[1][1] > V[2][2]) {
        const double S = 2.0 * sqrt(1.0 + V[1][1] - V[0][0] - V[2][2]);
        w = (V[0][2] - V[2][0]) / S; x = (V[0][1] + V[1][0]) / S; y = 0.25 * S; z = (V[1][2] + V[2][1]) / S;
    } else {
        const double S = 2.0 * sqrt(1.0 + V[2][2] - V[0][0] - V[1][1]);
        w = (V[1][0] - V[0][1]) / S; x = (V[0][2] + V[2][0]) / S; y = (V[1][2] + V[2][1]) / S; z = 0.25 * S;
    }
    const double qn = 1.0 / sqrt(w * w + x * x + y * y + z * z);
    const double out[7] = {w * qn, x * qn, y * qn, z * qn, d[0], d[1], d[2]};
    for (int c = 0; c < 7; ++c) stp<R>(L->kinv, ncell, c, idx, R(out[c]));
    const uint32_t nx = L->nx, nxy = nx * uint32_t(L->ny);
    const int zc = idx / nxy;
    const uint32_t r = idx - uint32_t(zc) * nxy;
    const int yc = r / nx, xc = r - uint32_t(yc) * nx;
    int face;
    if ((!fin || !psd) && cell_type(L, xc, yc, zc, link_word(L, idx), face) != CELL_SOLID) *L->err = 1;
}

// colour field of the initial state (two-fluid): C0 rho0 in fluid cells.
template <class R>
__global__ __launch_bounds__(BLOCK) void k_init_colour(const InitArgs<R> ia)
{
    const LatDev *L = ia.L;
    const uint32_t idx = blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= uint32_t(L->ncell)) return;
    const uint32_t nx = L->nx, nxy = nx * uint32_t(L->ny);
    const int z = idx / nxy;
    const uint32_t r = idx - uint32_t(z) * nxy;
    const int y = r / nx, x = r - uint32_t(y) * nx;
    int face;
    const int type = cell_type(L, x, y, z, link_word(L, idx), face);
    R v;
    if (type == CELL_SOLID) v = R(L->face_cw[face]);
    else if (type == CELL_RES) v = R(L->face_conc[face]) * R(L->face_rho[face]);
    else v = (ia.c0 ? ia.c0[idx] : R(0)) * (ia.rho0 ? ia.rho0[idx] : R(1));
    stg<R>(L->rho1, idx, v);
}

// initial populations (flowchart: f = f^eq, h = h^eq from the fields), the
// fixed reservoir states, and the moments of step 0; validates the fields.
template <int PHYS, class S>
__global__ __launch_bounds__(BLOCK) void k_init(const InitArgs<typename Codec<S>::R> ia)
{
    using R = typename Codec<S>::R;
    const LatDev *L = ia.L;
    const uint32_t ncell = L->ncell;
    const size_t n = ncell;
    const uint32_t idx = blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= ncell) return;
    const uint32_t nx = L->nx, nxy = nx * uint32_t(L->ny);
    const int z = idx / nxy;
    const uint32_t r = idx - uint32_t(z) * nxy;
    const int y = r / nx, x = r - uint32_t(y) * nx;
    int face;
    const uint32_t lw = link_word(L, idx);
    const int type = cell_type(L, x, y, z, lw, face);

    const R eps = L->uniform_eps ? R(L->eps_u) : ldg<R>(L->eps, idx);
    R kinv[3];
    // full tensor: the eigenvalue planes (4-6) after the frame quaternion
    for (int a = 0; a < 3; ++a)
        kinv[a] = L->uniform_kinv ? R(L->kinv_u[a]) : ldp<R>(L->kinv, ncell, L->full_tensor ? 4 + a : a, idx);
    const R rho0 = ia.rho0 ? ia.rho0[idx] : R(1);
    R u0[3];
    for (int a = 0; a < 3; ++a) u0[a] = ia.vel0 ? ia.vel0[a * n + idx] : R(0);
    const R c0 = ia.c0 ? ia.c0[idx] : R(0);
    // solid cells carry no state: their fields are not used
    if (type != CELL_SOLID &&
        (!(eps > R(0) && eps <= R(1)) || bad(kinv[0]) || bad(kinv[1]) || bad(kinv[2]) ||
         kinv[0] < R(0) || kinv[1] < R(0) || kinv[2] < R(0) || !(rho0 > R(0)) || bad(rho0) ||
         bad(u0[0]) || bad(u0[1]) || bad(u0[2]) || bad(c0))) {
        *L->err = 1;
    }

    R d[NQ], hq[NQ];
    R mrho = 0, mu[3] = {0, 0, 0}, mC = 0;
    if (type == CELL_SOLID) {
        for (int q = 0; q < NQ; ++q) d[q] = hq[q] = R(0);
    } else if (type == CELL_RES) {
        const R rb = R(L->face_rho[face]), cb = R(L->face_conc[face]), drb = R(L->face_rho[face] - 1.0);
#pragma unroll
        for (int q = 0; q < NQ; ++q) {
            const R w = weight<R>(q);
            d[q] = w * drb;
            hq[q] = PHYS == PH_MISCIBLE ? w * eps * cb : (PHYS == PH_IMMISCIBLE ? cb * w * rb : R(0));
        }
        mrho = rb;
        mC = PHYS == PH_SINGLE ? R(0) : cb;
    } else {
        const Nbr b = neighbours(L, x, y, z, lw);
        const R C = PHYS == PH_SINGLE ? R(0) : c0;
        R nu;
        if constexpr (PHYS == PH_IMMISCIBLE) nu = C * R(L->nu1) + (R(1) - C) * R(L->nu2);
        else nu = R(ia.nuc0) * exp(R(L->k1) * (PHYS == PH_MISCIBLE ? C : R(0)) + R(L->k0));
        const R tau = R(0.5) + R(3) * nu;
        R F[3] = {0, 0, 0};
        R Fn = 0;
        if constexpr (PHYS == PH_IMMISCIBLE) {
            colour_acc<R>(L->rho1, b, F[0], F[1], F[2]);
            Fn = sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]);
        }
        const R iFn = Fn > R(0) ? R(1) / Fn : R(0);
        const R st = Fn > R(0) ? R(L->A) * eps * tau : R(0);
        const R zero3[3] = {0, 0, 0};
        for (int q = 0; q < NQ; ++q) d[q] = R(0);
        // with omega = 1 and no force the collision returns f^eq
        const Coll<R> cl = make_coll<R>(rho0 - R(1), rho0, R(1), R(1) / eps, u0, zero3, st, F, Fn, iFn);
        collide_f<R, PHYS == PH_IMMISCIBLE>(d, cl);
        if constexpr (PHYS == PH_MISCIBLE) {
            R vs[3] = {u0[0], u0[1], u0[2]};
            if (L->eps_grad && !L->uniform_eps) {
                R gx = 0, gy = 0, gz = 0;
                eps_grad_acc<R>(L->eps, b, 0u, eps, gx, gy, gz);
                const R k = R(3) * R(L->D) / eps;
                vs[0] += k * gx;
                vs[1] += k * gy;
                vs[2] += k * gz;
            }
            for (int q = 0; q < NQ; ++q) hq[q] = R(0);
            const R ec = eps * c0;
            const R H[3] = {weight<R>(0) * ec, weight<R>(1) * ec, weight<R>(7) * ec};
            collide_h<R>(hq, R(0), H, vs);
        } else if constexpr (PHYS == PH_IMMISCIBLE) {
            const R Cw[3] = {C * weight<R>(0), C * weight<R>(1), C * weight<R>(7)};
            const R rw[3] = {0, 0, 0};
            recolour<R>(hq, d, C, Cw, rw, F);
        } else {
            for (int q = 0; q < NQ; ++q) hq[q] = R(0);
        }
        mrho = rho0;
        mu[0] = u0[0];
        mu[1] = u0[1];
        mu[2] = u0[2];
        mC = C;
    }
    for (int cpy = 0; cpy < 2; ++cpy) {
        if constexpr (paired_v<PHYS, S>) {
            store_pair<S>(L->f[cpy], L->fm[cpy], L->ppstride, idx, d, hq);
        } else {
            store_all<S>(L->f[cpy], L->fm[cpy], L->pstride, idx, d);
            if constexpr (PHYS != PH_SINGLE) store_all<S>(L->h[cpy], L->hm[cpy], L->pstride, idx, hq);
        }
    }
    void *M = L->mom;
    stg<R>(M, idx, mrho);
    stp<R>(M, ncell, 1, idx, mu[0]);
    stp<R>(M, ncell, 2, idx, mu[1]);
    stp<R>(M, ncell, 3, idx, mu[2]);
    stp<R>(M, ncell, 4, idx, mC);
    if constexpr (PHYS == PH_MISCIBLE) {
        // further solutes: h = h^eq(eps C0_k, V0 + D_k grad(eps)/eps) from
        // plane k of c0, as the first solute; reservoirs w eps C_bc,k
        const GL MsDev *X = ms_of(L);
        const int nsx = X ? X->nsx : 0;
        for (int k = 0; k < nsx; ++k) {
            R hk[NQ], Ck = 0;
            if (type == CELL_SOLID) {
                for (int q = 0; q < NQ; ++q) hk[q] = R(0);
            } else if (type == CELL_RES) {
                Ck = R(X->face_conc[k][face]);
                for (int q = 0; q < NQ; ++q) hk[q] = weight<R>(q) * eps * Ck;
            } else {
                Ck = ia.c0 ? ia.c0[size_t(k + 1) * n + idx] : R(0);
                if (bad(Ck)) *L->err = 1;
                R vs[3] = {u0[0], u0[1], u0[2]};
                if (L->eps_grad && !L->uniform_eps) {
                    const Nbr b = neighbours(L, x, y, z, lw);
                    R gx = 0, gy = 0, gz = 0;
                    eps_grad_acc<R>(L->eps, b, 0u, eps, gx, gy, gz);
                    const R kk = R(3) * R(X->D[k]) / eps;
                    vs[0] += kk * gx;
                    vs[1] += kk * gy;
                    vs[2] += kk * gz;
                }
                for (int q = 0; q < NQ; ++q) hk[q] = R(0);
                const R ec = eps * Ck;
                const R H[3] = {weight<R>(0) * ec, weight<R>(1) * ec, weight<R>(7) * ec};
                collide_h<R>(hk, R(0), H, vs);
            }
            for (int cpy = 0; cpy < 2; ++cpy) store_all<S>(X->h[k][cpy], X->hm[k][cpy], L->pstride, idx, hk);
            stp<R>(M, ncell, 5 + k, idx, Ck);
        }
    }
}

// diagnostics of the moments buffer (used after set-up: residual 0)
template <class R>
__global__ __launch_bounds__(BLOCK) void k_diag_moments(const LatDev *L)
{
    const uint32_t ncell = L->ncell;
    const uint32_t idx = blockIdx.x * BLOCK + threadIdx.x;
    double part[NPART] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (idx < ncell) {
        const uint32_t nx = L->nx, nxy = nx * uint32_t(L->ny);
        const int z = idx / nxy;
        const uint32_t r = idx - uint32_t(z) * nxy;
        const int y = r / nx, x = r - uint32_t(y) * nx;
        int face;
        if (cell_type(L, x, y, z, link_word(L, idx), face) == CELL_FLUID) {
            const void *M = L->mom;
            const R u[3] = {ldp<R>(M, ncell, 1, idx), ldp<R>(M, ncell, 2, idx), ldp<R>(M, ncell, 3, idx)};
            const R rho = ldg<R>(M, idx), C = ldp<R>(M, ncell, 4, idx);
            R s4 = 0;
            if (L->physics == PH_MISCIBLE)
                s4 = (L->uniform_eps ? R(L->eps_u) : ldg<R>(L->eps, idx)) * C;
            else if (L->physics == PH_IMMISCIBLE)
                s4 = ldg<R>(L->rho1, idx);
            diag_contrib<R>(part, rho, u, C, s4, u);
        }
    }
    block_reduce_store(part, L->partials + size_t(blockIdx.x) * NPART);
}

// Solute masses Sum eps C_k over fluid cells from the moments buffer: per
// block partials (slots 0..nsp-1), then one block sums them in a fixed order
// and leaves the totals in the first nsp partial slots.
template <class R>
__global__ __launch_bounds__(BLOCK) void k_solute_partials(const LatDev *L, int nsp)
{
    const uint32_t ncell = L->ncell;
    const uint32_t idx = blockIdx.x * BLOCK + threadIdx.x;
    double part[NPART] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (idx < ncell) {
        const uint32_t nx = L->nx, nxy = nx * uint32_t(L->ny);
        const int z = idx / nxy;
        const uint32_t r = idx - uint32_t(z) * nxy;
        const int y = r / nx, x = r - uint32_t(y) * nx;
        int face;
        if (cell_type(L, x, y, z, link_word(L, idx), face) == CELL_FLUID) {
            const double e = L->uniform_eps ? L->eps_u : double(ldg<R>(L->eps, idx));
            for (int k = 0; k < nsp; ++k) part[k] = e * double(ldp<R>(L->mom, ncell, 4 + k, idx));
        }
    }
    block_reduce_store(part, L->partials + size_t(blockIdx.x) * NPART);
}

__global__ __launch_bounds__(BLOCK) void k_solute_final(const LatDev *L, int nsp)
{
    double v[NPART] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    for (int bk = threadIdx.x; bk < L->nblocks; bk += BLOCK) {
        const double *p = L->partials + size_t(bk) * NPART;
        for (int k = 0; k < nsp; ++k) v[k] += p[k];
    }
    __shared__ double out[NPART];
    block_reduce_store(v, out);
    __syncthreads();
    if (threadIdx.x < nsp) L->partials[threadIdx.x] = out[threadIdx.x];
}

// decode the current populations of one lattice to the compute type
template <class S>
__global__ __launch_bounds__(BLOCK) void k_export(const LatDev *L, int which, int src, typename Codec<S>::R *dst)
{
    const uint32_t ncell = L->ncell;
    const uint32_t idx = blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= ncell) return;
    using R = typename Codec<S>::R;
    if constexpr (sizeof(S) == 2) {
        if (L->physics == PH_MISCIBLE && which < 2) {
            // paired planes: half `which` of every word (and of the mass pair)
            using W = typename PairCodec<S>::W;
            R m = 0;
            if constexpr (Codec<S>::split) {
                const f32x2_t mp = ldg<f32x2_t>(L->fm[src], idx);
                m = which == 0 ? mp.x : mp.y;
            }
            for (int q = 0; q < NQ; ++q) {
                R a, c;
                PairCodec<S>::load(at(plane<W>(L->f[src], L->ppstride, q), idx), a, c);
                dst[size_t(q) * ncell + idx] = fma(weight<R>(q), m, which == 0 ? a : c);
            }
            return;
        }
    }
    const GL MsDev *X = ms_of(L);
    const void *P = which == 0 ? L->f[src] : (which == 1 ? L->h[src] : X->h[which - 2][src]);
    const void *M = which == 0 ? L->fm[src] : (which == 1 ? L->hm[src] : X->hm[which - 2][src]);
    const R m = Codec<S>::split ? ldg<R>(M, idx) : R(0);
    for (int q = 0; q < NQ; ++q)
        dst[size_t(q) * ncell + idx] = fma(weight<R>(q), m, Codec<S>::load(at(plane<S>(P, L->pstride, q), idx)));
}

}  // namespace plbm
