// freesurf.hpp -- the free-surface technique of Sec. 3 on gfx950: liquid,
// interface and gas cells, the liquid mass of interface cells (Eqs.
// massmacro, massevol, deltamass), populations rebuilt on links from gas
// cells (Eq. equilempty) and the conversion of cells as they fill and empty
// (flowchart of Sec. 4: stream the mass, redefine the cell classes).
//
// One step is five launches, plus one on moment steps:
//   k_fs_step        pull + gas-side reconstruction + mass exchange + collision
//                    of liquid and interface cells; conversion flags (w1) of
//                    interface cells
//   k_fs_mark_fill   filling cells mark their gas neighbours to become interface
//                    cells and keep emptying neighbours
//   k_fs_mark_empty  cells that empty mark their liquid neighbours to become
//                    interface cells; marked gas cells get the equilibrium of
//                    their neighbours' mean state
//   k_fs_excess      excess mass of each converted cell, split over its receivers
//   k_fs_final       new classes, masses and fill fractions
//   k_fs_moments     moments and FP64 diagnostics (moment steps only)
// Liquid cells cost one byte read and one byte written more than the
// single-fluid step; gas cells are skipped (waves made only of gas cells
// store nothing); the class passes read byte planes, 16 cells per thread, of
// the rows flagged as having work, and work only next to conversions.
#pragma once

#include <type_traits>

#include "kernels.hpp"

namespace plbm {

enum { FS_GAS = 0, FS_IF = 1, FS_LIQ = 2, FS_SOLID = 3 };
enum { FS_FILL = 1, FS_EMPTY = 2 };
constexpr double FS_KAPPA = 1e-3;   // conversion margin: m > (1 + k) rho fills, m < -k rho empties

// Free-surface state of one lattice, in its workspace.  Masses, densities
// and fill fractions are double in every storage mode, so the class
// decisions and the mass bookkeeping do not depend on the population format.
struct FsDev {
    unsigned char *cls;     // class of every cell after the last step (FS_*)
    unsigned char *w1;      // step work bytes: conversion flag, then the packed new class
    unsigned char *w2;      // step work bytes: resolved flag | 4 (gas cell to become interface)
    double *mass;           // liquid mass m of interface cells
    double *lam[2];         // fill fraction m / rho of interface cells, one plane per
                            // population copy (pass 1 reads the neighbours' in the
                            // source copy and writes its own in the other)
    double *rho;            // rho and V' (3 planes) of the step: interface cells every
    double *u;              // step, every liquid or interface cell on moment steps
    double *share;          // excess mass per receiver of each converting cell
    double *lost;           // accumulated excess mass that found no receiver
    // launch order of pass 1, one set per population copy (as lam): rows of
    // 256 cells that hold interface cells, in the order they were listed, the
    // number listed, and per row 1 + its position in the list (0: not listed)
    uint32_t *hlist[2];
    uint32_t *hcount[2];
    uint32_t *hpos[2];
    // per row of 256 cells, one byte per population copy: nonzero when pass 1
    // has work in the row (a liquid or interface cell, or a cell flagged in
    // the last step, whose flag pass 1 clears); written by the last class
    // pass for the next step, all rows set at set-up
    unsigned char *rowlive[2];
    // per row of 256 cells: nonzero when the class passes have work in it this
    // step (a conversion flag of pass 1, a mark written by a class pass, or a
    // wave of pass 1 without liquid or interface cells, whose liveness the last
    // pass recomputes); the class passes skip the other rows, the last pass
    // clears it; zero at set-up
    unsigned char *rowwork;
};

// List a row for the next pass 1 (buffer buf), once: the first caller claims
// it, takes a position and records it; later callers find it claimed.
// Positions stay below the row count nrow (a row is listed at most once
// until it is unlisted); the bound on the store guards the list regardless.
__device__ inline void fs_list_row(const GL FsDev *F, int buf, uint32_t row, uint32_t nrow)
{
    if (atomicCAS(F->hpos[buf] + row, 0u, ~0u) == 0u) {
        const uint32_t pos = atomicAdd(F->hcount[buf], 1u);
        if (pos < nrow) F->hlist[buf][pos] = row;
        atomicExch(F->hpos[buf] + row, pos + 1u);
    }
}

// The free-surface block lives in the workspace (global memory); naming its
// address space lets the compiler read its fields with scalar loads instead
// of a vector round trip per field.
__device__ inline const GL FsDev *fs_of(const LatDev *L)
{
    return static_cast<const GL FsDev *>((const GL void *)L->fs);
}

// f(std::integral_constant<int, Q>) for Q = 1 .. 18
template <int Q = 1, class Fn>
__device__ inline void for_links(Fn &&fn)
{
    fn(std::integral_constant<int, Q>{});
    if constexpr (Q + 1 < NQ) for_links<Q + 1>(fn);
}

// f(std::integral_constant<int, Q>) for Q = A .. B - 1
template <int A, int B, class Fn>
__device__ inline void for_range(Fn &&fn)
{
    if constexpr (A < B) {
        fn(std::integral_constant<int, A>{});
        for_range<A + 1, B>(fn);
    }
}

// Per-link neighbour data (classes, fill fractions) is read in groups of
// FS_GROUP links: all loads of a group are issued before any is used, so an
// interface cell waits for six round trips instead of one or two per link
// (measured on the 256^3 penetration step: 7-9% faster than per link; groups
// of 1, 2 and 6 are slower than 3, the larger ones from register pressure).
// Every neighbour index is wrapped into the lattice, so the loads need no
// guard; the values of solid links are replaced after the load.
constexpr int FS_GROUP = 3;
static_assert((NQ - 1) % FS_GROUP == 0, "whole groups cover the 18 links");

// fn(std::integral_constant<int, Q0>) for the first link Q0 of every group
template <int Q0 = 1, class Fn>
__device__ inline void for_groups(Fn &&fn)
{
    fn(std::integral_constant<int, Q0>{});
    if constexpr (Q0 + FS_GROUP < NQ) for_groups<Q0 + FS_GROUP>(fn);
}

// the 19 populations of cell idx of one copy, decoded
template <class S>
__device__ inline void load_cell(const void *P, const void *M, uint32_t n, uint32_t idx, typename Codec<S>::R *o)
{
    using R = typename Codec<S>::R;
    if constexpr (Codec<S>::split) {
        const R m = ldg<R>(M, idx);
#pragma unroll
        for (int q = 0; q < NQ; ++q) o[q] = fma(weight<R>(q), m, Codec<S>::load(at(plane<S>(P, n, q), idx)));
    } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) o[q] = Codec<S>::load(at(plane<S>(P, n, q), idx));
    }
}

// population q of cell idx of one copy, decoded as load_cell does
template <class S>
__device__ inline typename Codec<S>::R load_pop(const void *P, const void *M, uint32_t n, uint32_t idx, int q)
{
    using R = typename Codec<S>::R;
    if constexpr (Codec<S>::split)
        return fma(weight<R>(q), ldg<R>(M, idx), Codec<S>::load(at(plane<S>(P, n, q), idx)));
    else
        return Codec<S>::load(at(plane<S>(P, n, q), idx));
}

// equilibrium deviations f^eq - w at (rho, u) (Eqs. equilc1/2 without the
// surface-tension part): the collision with omega = 1 and no force of zeros
template <class R>
__device__ inline void equilibrium(R rho, const R u[3], R ie, R *e)
{
    const R zero3[3] = {0, 0, 0};
#pragma unroll
    for (int q = 0; q < NQ; ++q) e[q] = R(0);
    const Coll<R> c = make_coll<R>(rho - R(1), rho, R(1), ie, u, zero3, R(0), zero3, R(0), R(0));
    collide_f<R, false>(e, c);
}

struct FsCell {
    const LatDev *L;
    const GL FsDev *F;
    int l, lb, flags;
    uint32_t idx, ncell;
};

__device__ inline FsCell fs_cell(const BatchArgs &a)
{
    FsCell c;
    const int gb = xcd_remap(blockIdx.x, a.total_blocks);
    c.l = find_lattice(a, gb);
    c.L = a.lat[c.l];
    c.F = fs_of(c.L);
    // the pass-1 grid of a lattice (listed-row prefix + one block per row) is
    // not a whole number of planes: no slab or row-group remapping here
    c.lb = gb - a.blk_start[c.l];
    c.flags = a.flags[c.l];
    c.ncell = c.L->ncell;
    c.idx = uint32_t(c.lb) * BLOCK + threadIdx.x;
    return c;
}

__device__ inline void coords(const LatDev *L, uint32_t idx, int &x, int &y, int &z)
{
    const uint32_t nx = L->nx, nxy = nx * uint32_t(L->ny);
    z = udiv(idx, L->div_nxy);
    const uint32_t r = idx - uint32_t(z) * nxy;
    y = udiv(r, L->div_nx);
    x = r - uint32_t(y) * nx;
}

// fill fraction of the step's start of a cell of class c (1 liquid, 0 gas,
// m / rho interface)
__device__ inline double fs_lambda(const GL FsDev *F, int c, uint32_t j, int src)
{
    return c == FS_LIQ ? 1.0 : (c == FS_IF ? ldg<double>(F->lam[src], j) : 0.0);
}

// Pass 1.  Liquid and interface cells: pull; on links from gas cells the
// rebuilt population f_q = f^eq_q + f^eq_opp(q) - f~_opp(q)(x) at the gas
// density 1 and the velocity of the cell's own post-collision populations
// (Eq. equilempty); mass exchange over the links to liquid and interface
// neighbours (Eq. deltamass); the single-fluid collision with the porous
// terms and, ST, the surface-tension term of Eqs. equilc1/2 with the gradient
// of Eq. macros taken over the fill fraction, F = Sum lambda(x + v_q) v_q (a
// solid neighbour takes lambda(x)); interface cells store m and rho and flag
// FILL / EMPTY.
// Waves per SIMD the stream/collide pass is compiled for.  Without tensor or
// surface tension: FP32, BF16 and FP16 deviations and both split forms take 7
// waves (72 VGPRs, 0-20 bytes of spill per lane), FP16 deviations 6.  On the
// 256^3 penetration step, one wave more measured FP32 +13%, FP16 split +7%,
// BF16 +0.5%, and BF16 split (6 -> 7) -3%, FP16 deviations (5 -> 6) -7%.
// Every other form keeps the compiler's choice.
template <class S, bool FT, bool ST> struct FsWaves { static constexpr int value = 1; };
template <> struct FsWaves<bf16_t, false, false> { static constexpr int value = 7; };
template <> struct FsWaves<bf16s_t, false, false> { static constexpr int value = 7; };
template <> struct FsWaves<f16s_t, false, false> { static constexpr int value = 7; };
template <> struct FsWaves<f16_t, false, false> { static constexpr int value = 6; };
template <> struct FsWaves<float, false, false> { static constexpr int value = 7; };

//
// Launch order: a lattice's blocks are a prefix of `cap` blocks followed by one
// block per row of 256 cells.  Prefix block i processes the i-th listed row (a
// row that held interface cells at the previous step or gained them in its
// class passes) and exits if fewer are listed; a row block exits if its row
// was listed within the first `cap`.  Interface cells wait on their
// neighbours' classes and fill fractions, so their waves run longest; started
// first, they overlap with the bulk instead of trailing it.  Every row is
// processed exactly once, and no cell reads what another writes in this pass,
// so the order changes no result.

template <class S, bool FT, bool ST = false>
__global__ PLBM_STEP_ATTR __attribute__((amdgpu_waves_per_eu(FsWaves<S, FT, ST>::value))) void k_fs_step(const BatchArgs a)
{
    using R = typename Codec<S>::R;
    [[maybe_unused]] constexpr bool HW = HwMath<S>::value;
    FsCell c = fs_cell(a);
    const LatDev *__restrict__ L = c.L;
    const GL FsDev *__restrict__ F = c.F;
    const int src = c.flags & 1, dst = src ^ 1;
    const uint32_t nrow = (c.ncell + BLOCK - 1) / BLOCK;
    const uint32_t cap = uint32_t(a.blk_start[c.l + 1] - a.blk_start[c.l]) - nrow;
    const bool prefix = uint32_t(c.lb) < cap;
    uint32_t row;
    if (prefix) {
        if (uint32_t(c.lb) >= ldg<uint32_t>(F->hcount[src], 0)) return;   // uniform over the block
        row = ldg<uint32_t>(F->hlist[src], uint32_t(c.lb));
        if (row >= nrow) return;
    } else {
        row = uint32_t(c.lb) - cap;
        // a row without liquid, interface or flagged cells (all gas, solid):
        // its populations, classes and flags stay as they are (uniform)
        if (!ldg<uint8_t>(F->rowlive[src], row)) return;
    }
    c.idx = row * BLOCK + threadIdx.x;
    const uint32_t idx = c.idx, ncell = c.ncell;
    const bool mom = (c.flags & 2) != 0;
    const R nuc = R(a.nuc[c.l]);

    int cls = FS_SOLID, x = 0, y = 0, z = 0;
    uint32_t lw = 0;
    // a row block reads whether the prefix took its row with its class
    const uint32_t listed = prefix ? 0u : ldg<uint32_t>(F->hpos[src], row);
    if (idx < ncell) {
        coords(L, idx, x, y, z);
        lw = link_word(L, idx);
        cls = ldg<uint8_t>(F->cls, idx);
    }
    if (listed != 0u && listed <= cap) return;   // uniform over the block
    const bool live = cls == FS_IF || cls == FS_LIQ;
    R d[NQ];
    unsigned char flag = 0;
    if (live) {
        const Nbr b = neighbours(L, x, y, z, lw);
        // split codecs: the 19 mass loads (sharing the x-links' masses across
        // the wave measured 4% slower here in BF16, which spills at 7 waves)
        pull_all<S, false>(L->f[src], L->fm[src], L->pstride, idx, b, d);
        const R eps = L->uniform_eps ? R(L->eps_u) : ldg<R>(L->eps, idx);
        const R ie = rcp<HW>(eps);
        double m = 0.0;
        if (cls == FS_IF) {
            // velocity of the cell's own post-collision populations; they are
            // read again link by link below (cache hits) rather than held
            R ou[3];
            {
                R o[NQ];
                load_cell<S>(L->f[src], L->fm[src], L->pstride, idx, o);
                R odr = 0, ojx = 0, ojy = 0, ojz = 0;
                moments_acc<R>(o, odr, ojx, ojy, ojz);
                const R iro = rcp<HW>(R(1) + odr);
                ou[0] = ojx * iro;
                ou[1] = ojy * iro;
                ou[2] = ojz * iro;
            }
            // the rebuilt population needs f^eq_q + f^eq_opp(q) only: 9
            // distinct sums (addition commutes exactly), so the 19
            // equilibria die here
            R es[NQ];
            {
                R eA[NQ];
                equilibrium<R>(R(1), ou, ie, eA);
#pragma unroll
                for (int q = 1; q < NQ; ++q) es[q] = eA[q] + eA[opp(q)];
            }
            const double lx = ldg<double>(F->lam[src], idx);
            double dm = 0.0;
            for_groups([&](auto gc) {
                constexpr int Q0 = decltype(gc)::value;
                int cn[FS_GROUP];
                double ln[FS_GROUP];
                R oo[FS_GROUP];
                // the neighbours x - v_Q, whose population Q streams in and to
                // which the population opp(Q) of this cell streams out
                for_range<Q0, Q0 + FS_GROUP>([&](auto qc) {
                    constexpr int Q = decltype(qc)::value;
                    const uint32_t j = shifted<Q, -1>(b);
                    cn[Q - Q0] = ldg<uint8_t>(F->cls, j);
                    ln[Q - Q0] = ldg<double>(F->lam[src], j);
                    oo[Q - Q0] = load_pop<S>(L->f[src], L->fm[src], L->pstride, idx, opp(Q));
                });
                for_range<Q0, Q0 + FS_GROUP>([&](auto qc) {
                    constexpr int Q = decltype(qc)::value;
                    const int cj = shifted_solid<Q, -1>(b) ? FS_SOLID : cn[Q - Q0];
                    if (cj == FS_GAS) {
                        d[Q] = es[Q] - oo[Q - Q0];
                    } else if (cj != FS_SOLID) {
                        const double fl = double(d[Q]) - double(oo[Q - Q0]);
                        dm += cj == FS_LIQ ? fl : fl * (0.5 * (lx + ln[Q - Q0]));
                    }
                });
            });
            m = ldg<double>(F->mass, idx) + dm;
        }

        R drho = 0, jx = 0, jy = 0, jz = 0;
        moments_acc<R>(d, drho, jx, jy, jz);
        const R rho = R(1) + drho;
        const R irho = rcp<HW>(rho);
        const R V[3] = {jx * irho, jy * irho, jz * irho};
        const R nu = nuc * fexp<HW>(R(L->k0));
        const R omega = rcp<HW>(R(0.5) + R(3) * nu);
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
        R Fs[3] = {0, 0, 0}, Fn = 0, iFn = 0, st = 0;
        if constexpr (ST) {
            if (L->A != 0.0) {
                const double l0 = fs_lambda(F, cls, idx, src);
                double g[3] = {0.0, 0.0, 0.0};
                for_groups([&](auto gc) {
                    constexpr int Q0 = decltype(gc)::value;
                    int cn[FS_GROUP];
                    double ln[FS_GROUP];
                    for_range<Q0, Q0 + FS_GROUP>([&](auto qc) {
                        constexpr int Q = decltype(qc)::value;
                        cn[Q - Q0] = ldg<uint8_t>(F->cls, shifted<Q, 1>(b));
                    });
                    // the fill fraction is read only where the neighbour is an
                    // interface cell (interior liquid cells read none)
                    for_range<Q0, Q0 + FS_GROUP>([&](auto qc) {
                        constexpr int Q = decltype(qc)::value;
                        const int c = cn[Q - Q0];
                        ln[Q - Q0] = shifted_solid<Q, 1>(b) ? l0
                                   : (c == FS_LIQ ? 1.0 : (c == FS_IF ? ldg<double>(F->lam[src], shifted<Q, 1>(b)) : 0.0));
                    });
                    for_range<Q0, Q0 + FS_GROUP>([&](auto qc) {
                        constexpr int Q = decltype(qc)::value;
                        const double l = ln[Q - Q0];
                        if constexpr (cx(Q) != 0) g[0] += cx(Q) > 0 ? l : -l;
                        if constexpr (cy(Q) != 0) g[1] += cy(Q) > 0 ? l : -l;
                        if constexpr (cz(Q) != 0) g[2] += cz(Q) > 0 ? l : -l;
                    });
                });
                for (int c = 0; c < 3; ++c) Fs[c] = R(g[c]);
                Fn = sqrt(Fs[0] * Fs[0] + Fs[1] * Fs[1] + Fs[2] * Fs[2]);
                iFn = Fn > R(0) ? rcp<HW>(Fn) : R(0);
                st = Fn > R(0) ? R(L->A) * eps * (R(0.5) + R(3) * nu) : R(0);
            }
        }
        const Coll<R> cl = make_coll<R>(drho, rho, omega, ie, u, Fx, st, Fs, Fn, iFn);
        collide_f<R, ST>(d, cl);

        if (cls == FS_IF) {
            const double r = double(rho);
            stg<double>(F->mass, idx, m);
            stg<double>(F->rho, idx, r);
            for (int k = 0; k < 3; ++k) stp<double>(F->u, ncell, k, idx, double(u[k]));
            stg<double>(F->lam[dst], idx, m / r);   // before the shares of converting neighbours
            stg<uint8_t>(F->w2, idx, 0);            // a mark of the last step
            flag = m > (1.0 + FS_KAPPA) * r ? FS_FILL : (m < -FS_KAPPA * r ? FS_EMPTY : 0);
        } else if (mom) {
            stg<double>(F->rho, idx, double(rho));
            for (int k = 0; k < 3; ++k) stp<double>(F->u, ncell, k, idx, double(u[k]));
        }
    } else {
#pragma unroll
        for (int q = 0; q < NQ; ++q) d[q] = R(0);
    }
    if (idx < ncell) stg<uint8_t>(F->w1, idx, flag);
    // the class passes work on the rows with a flag, and recompute the
    // liveness of rows that have a wave without liquid or interface cells
    const bool any_live = __builtin_amdgcn_ballot_w64(live) != 0;
    if ((__builtin_amdgcn_ballot_w64(flag != 0) != 0 || !any_live) && (threadIdx.x & 63) == 0)
        stg<uint8_t>(F->rowwork, row, 1);
    // waves made only of gas and solid cells store nothing
    if (idx < ncell && any_live)
        store_all<S>(L->f[dst], L->fm[dst], L->pstride, idx, d);
    if (__builtin_amdgcn_ballot_w64(cls == FS_IF) != 0 && (threadIdx.x & 63) == 0) fs_list_row(F, dst, row, nrow);
}

// ---------------------------------------------------------------------------
// The class passes touch only the few cells next to conversions.  Each thread
// scans the bytes of FS_CPT consecutive cells with one 16-byte load per plane
// (planes are 256-byte aligned and padded, so the last load of a lattice stays
// inside its plane) and works only on the cells that need it; a cell's
// neighbours are reached by writing into their mark bytes (w2), so no thread
// has to look for conversions around itself.  Marks written by several cells
// into one byte carry the same value.
//   w1: the FILL / EMPTY flag of pass 1 (0 elsewhere)
//   w2: FS_BORN (gas cell next to a filling cell), FS_KEEP (emptying cell next
//       to a filling cell: it stays), FS_TO_IF (liquid cell next to a cell that
//       empties), FS_RECV (a receiver of excess mass); zero outside the marked
//       cells.  The last pass clears the marks of cells that were not interface
//       cells (it reads FS_KEEP marks of neighbours, so those stay); pass 1 of
//       the next step clears the marks of interface cells.
constexpr int FS_CPT = 16;
enum { FS_BORN = 1, FS_KEEP = 2, FS_TO_IF = 4, FS_RECV = 8 };
typedef uint32_t u32x4 __attribute__((ext_vector_type(4)));

struct FsTile {
    const LatDev *L;
    const GL FsDev *F;
    int flags;
    uint32_t base, ncell;
};

// blocks of BLOCK * FS_CPT cells
__device__ inline FsTile fs_tile(const BatchArgs &a)
{
    FsTile t;
    const int gb = blockIdx.x;
    const int l = find_lattice(a, gb);
    t.L = a.lat[l];
    t.F = fs_of(t.L);
    t.flags = a.flags[l];
    t.ncell = t.L->ncell;
    t.base = (uint32_t(gb - a.blk_start[l]) * BLOCK + threadIdx.x) * FS_CPT;
    return t;
}

__device__ inline u32x4 ld16(const unsigned char *p, uint32_t base) { return ldg<u32x4>(p, base / FS_CPT); }

__device__ inline int byte_of(const u32x4 &v, int k)
{
    const uint32_t w = k < 4 ? v.x : (k < 8 ? v.y : (k < 12 ? v.z : v.w));
    return int((w >> (8 * (k & 3))) & 0xffu);
}

__device__ inline bool any_byte(const u32x4 &v) { return (v.x | v.y | v.z | v.w) != 0u; }

// the cell empties after all: flagged EMPTY and not kept by a filling neighbour
__device__ inline bool empties(int w1, int w2) { return w1 == FS_EMPTY && !(w2 & FS_KEEP); }

// Position of the n-th set bit (from 0) of v, n < popcount(v), by halving.
__host__ __device__ inline int nth_set_bit(uint64_t v, uint32_t n)
{
    int pos = 0;
    for (int w = 32; w >= 1; w >>= 1) {
        const uint32_t c = uint32_t(__builtin_popcountll((v >> pos) & ((uint64_t(1) << w) - 1)));
        if (n >= c) {
            n -= c;
            pos += w;
        }
    }
    return pos;
}

// The work of a wave's class pass: lane l covers the FS_CPT cells from
// base(l) = wbase + FS_CPT l and marks item k (cell base(l) + k) in bit k of
// its mask.  The items are dealt to the lanes in rounds of 64 (k major, lane
// minor) and fn(idx) runs on the lane an item is dealt to, so the wave waits
// for ceil(items / 64) chains of dependent neighbour loads rather than up to
// FS_CPT chains one after the other on the lane that found them.  Cells are
// independent within a pass, so the dealing changes no result.  Every lane
// of the wave must call it.
template <class Fn>
__device__ inline void for_items(uint32_t mask, uint32_t base, Fn &&fn)
{
    const int lane = threadIdx.x & 63;
    const uint32_t wbase = base - uint32_t(FS_CPT * lane);
    uint64_t B[FS_CPT];
    uint32_t start[FS_CPT + 1];
    start[0] = 0;
#pragma unroll
    for (int k = 0; k < FS_CPT; ++k) {
        B[k] = __builtin_amdgcn_ballot_w64(((mask >> k) & 1u) != 0u);
        start[k + 1] = start[k] + uint32_t(__builtin_popcountll(B[k]));
    }
    const uint32_t total = start[FS_CPT];
    for (uint32_t r = 0; r < total; r += 64) {
        const uint32_t i = r + uint32_t(lane);
        if (i >= total) continue;
        // the item's k: the last k with start[k] <= i (B[k] is then not empty)
        int k = 0;
        uint64_t bits = B[0];
        uint32_t n = i;
#pragma unroll
        for (int kk = 1; kk < FS_CPT; ++kk) {
            if (i >= start[kk]) {
                k = kk;
                bits = B[kk];
                n = i - start[kk];
            }
        }
        fn(wbase + uint32_t(FS_CPT * nth_set_bit(bits, n) + k));
    }
}

// write mark byte v of cell j and note its row as one with work
__device__ inline void mark(const GL FsDev *F, uint32_t j, uint8_t v)
{
    stg<uint8_t>(F->w2, j, v);
    stg<uint8_t>(F->rowwork, j / BLOCK, 1);
}

// does the row of this thread's cells have work in this step's class passes
// (the FS_CPT cells of a thread lie in one row)
__device__ inline bool row_work(const FsTile &t)
{
    return t.base < t.ncell && ldg<uint8_t>(t.F->rowwork, t.base / BLOCK) != 0;
}

__device__ inline Nbr nbr_of(const LatDev *L, uint32_t idx)
{
    int x, y, z;
    coords(L, idx, x, y, z);
    return neighbours(L, x, y, z, 0u);
}

// Pass 2.  Every filling cell marks its gas neighbours FS_BORN and its
// emptying neighbours FS_KEEP.
__global__ __launch_bounds__(BLOCK) void k_fs_mark_fill(const BatchArgs a)
{
    const FsTile t = fs_tile(a);
    const GL FsDev *__restrict__ F = t.F;
    uint32_t mask = 0;
    if (t.base < t.ncell) {
        // the launch-order list pass 1 has just used serves the next step
        // again: unlist its rows (the count is cleared by the next pass)
        const int src = t.flags & 1;
        const uint32_t tn = t.base / FS_CPT, nrow = (t.ncell + BLOCK - 1) / BLOCK;
        if (tn < nrow && tn < ldg<uint32_t>(F->hcount[src], 0)) {
            const uint32_t r = ldg<uint32_t>(F->hlist[src], tn);
            if (r < nrow) stg<uint32_t>(F->hpos[src], r, 0u);
        }
        if (row_work(t)) {
            const u32x4 f = ld16(F->w1, t.base);
            if (any_byte(f))
                for (int k = 0; k < FS_CPT; ++k)
                    if (t.base + k < t.ncell && byte_of(f, k) == FS_FILL) mask |= 1u << k;
        }
    }
    if (__builtin_amdgcn_ballot_w64(mask != 0u) == 0) return;   // uniform over the wave
    for_items(mask, t.base, [&](uint32_t idx) {
        const Nbr b = nbr_of(t.L, idx);
        for_links([&](auto qc) {
            constexpr int Q = decltype(qc)::value;
            const uint32_t j = shifted<Q, 1>(b);
            const int cj = ldg<uint8_t>(F->cls, j), fj = ldg<uint8_t>(F->w1, j);
            if (cj == FS_GAS) mark(F, j, FS_BORN);
            else if (fj == FS_EMPTY) mark(F, j, FS_KEEP);
        });
    });
}

// Pass 3.  Every cell that empties marks its liquid neighbours FS_TO_IF;
// every FS_BORN cell takes the equilibrium of the mean density and velocity
// of the post-collision populations of its liquid and interface neighbours
// that do not empty, with m = 0.
template <class S>
__global__ __launch_bounds__(BLOCK) void k_fs_mark_empty(const BatchArgs a)
{
    using R = typename Codec<S>::R;
    [[maybe_unused]] constexpr bool HW = HwMath<S>::value;
    const FsTile t = fs_tile(a);
    const LatDev *__restrict__ L = t.L;
    const GL FsDev *__restrict__ F = t.F;
    const int dst = (t.flags & 1) ^ 1;
    if (t.base == 0) stg<uint32_t>(F->hcount[dst ^ 1], 0, 0u);   // the list unlisted by the last pass
    uint32_t mask = 0;
    if (row_work(t)) {
        const u32x4 f = ld16(F->w1, t.base), m2 = ld16(F->w2, t.base);
        if (any_byte(f) || any_byte(m2))
            for (int k = 0; k < FS_CPT; ++k) {
                const int w1 = byte_of(f, k), w2 = byte_of(m2, k);
                if (t.base + k < t.ncell && (empties(w1, w2) || (w2 & FS_BORN))) mask |= 1u << k;
            }
    }
    if (__builtin_amdgcn_ballot_w64(mask != 0u) == 0) return;   // uniform over the wave
    for_items(mask, t.base, [&](uint32_t idx) {
        // neither byte of a cell that empties or is born is written in this pass
        const int w1 = ldg<uint8_t>(F->w1, idx), w2 = ldg<uint8_t>(F->w2, idx);
        const Nbr b = nbr_of(L, idx);
        if (empties(w1, w2)) {
            for_links([&](auto qc) {
                constexpr int Q = decltype(qc)::value;
                const uint32_t j = shifted<Q, 1>(b);
                if (ldg<uint8_t>(F->cls, j) == FS_LIQ) mark(F, j, FS_TO_IF);
            });
        } else {
            // born: a gas cell has no liquid neighbour, so the qualifying
            // neighbours are interface cells, whose rho and V' pass 1 stored
            double rs = 0.0, us[3] = {0.0, 0.0, 0.0};
            int n = 0;
            for_links([&](auto qc) {
                constexpr int Q = decltype(qc)::value;
                const uint32_t j = shifted<Q, 1>(b);
                // an interface neighbour's mark byte is not written in this pass
                if (ldg<uint8_t>(F->cls, j) == FS_IF && !empties(ldg<uint8_t>(F->w1, j), ldg<uint8_t>(F->w2, j))) {
                    rs += ldg<double>(F->rho, j);
                    for (int c = 0; c < 3; ++c) us[c] += ldp<double>(F->u, t.ncell, c, j);
                    ++n;
                }
            });
            // n >= 1: the filling neighbour qualifies
            const double in = n ? 1.0 / n : 0.0;
            const double ra = n ? rs * in : 1.0;
            const double ua[3] = {us[0] * in, us[1] * in, us[2] * in};
            const R eps = L->uniform_eps ? R(L->eps_u) : ldg<R>(L->eps, idx);
            const R ur[3] = {R(ua[0]), R(ua[1]), R(ua[2])};
            R e[NQ];
            equilibrium<R>(R(ra), ur, rcp<HW>(eps), e);
            store_all<S>(L->f[dst], L->fm[dst], L->pstride, idx, e);
            stg<double>(F->mass, idx, 0.0);
            stg<double>(F->rho, idx, ra);
            for (int c = 0; c < 3; ++c) stp<double>(F->u, t.ncell, c, idx, ua[c]);
        }
    });
}

// does the neighbour j convert (fill, or empty after all)?
__device__ inline bool converts(const GL FsDev *F, uint32_t j)
{
    const int f = ldg<uint8_t>(F->w1, j);
    return f == FS_FILL || (f == FS_EMPTY && !(ldg<uint8_t>(F->w2, j) & FS_KEEP));
}

// Pass 4.  Excess mass of each converted cell (m - rho when it filled, m when
// it emptied), split equally over its neighbours that end the step as
// interface cells without converting; without any, it is lost (and counted).
__global__ __launch_bounds__(BLOCK) void k_fs_excess(const BatchArgs a)
{
    const FsTile t = fs_tile(a);
    const GL FsDev *__restrict__ F = t.F;
    uint32_t mask = 0;
    if (row_work(t)) {
        const u32x4 f = ld16(F->w1, t.base);
        if (any_byte(f)) {
            const u32x4 m2 = ld16(F->w2, t.base);
            for (int k = 0; k < FS_CPT; ++k) {
                const int w1 = byte_of(f, k);
                if (t.base + k < t.ncell && (w1 == FS_FILL || empties(w1, byte_of(m2, k)))) mask |= 1u << k;
            }
        }
    }
    if (__builtin_amdgcn_ballot_w64(mask != 0u) == 0) return;   // uniform over the wave
    for_items(mask, t.base, [&](uint32_t idx) {
        const int w1 = ldg<uint8_t>(F->w1, idx);
        const Nbr b = nbr_of(t.L, idx);
        int n = 0;
        for_links([&](auto qc) {
            constexpr int Q = decltype(qc)::value;
            const uint32_t j = shifted<Q, 1>(b);
            const int cj = ldg<uint8_t>(F->cls, j), mj = ldg<uint8_t>(F->w2, j);
            const bool recv = (cj == FS_IF && !converts(F, j)) || (mj & (FS_BORN | FS_TO_IF));
            n += recv ? 1 : 0;
        });
        const double m = ldg<double>(F->mass, idx);
        const double ex = w1 == FS_FILL ? m - ldg<double>(F->rho, idx) : m;
        stg<double>(F->share, idx, n ? ex / n : 0.0);
        if (!n) atomicAdd(F->lost, ex);
        // mark the receivers: every writer of a mark byte writes the same value
        // (the other bits do not change in this pass)
        if (n)
            for_links([&](auto qc) {
                constexpr int Q = decltype(qc)::value;
                const uint32_t j = shifted<Q, 1>(b);
                const int cj = ldg<uint8_t>(F->cls, j), mj = ldg<uint8_t>(F->w2, j);
                if ((cj == FS_IF && !converts(F, j)) || (mj & (FS_BORN | FS_TO_IF)))
                    mark(F, j, (uint8_t)(mj | FS_RECV));
            });
    });
}

// Pass 5.  New classes of the converted and marked cells; the final mass and
// fill fraction of the interface cells that changed: their own mass (rho for
// a liquid cell that became one, 0 for a gas cell that did) plus the shares
// of their converting neighbours (FS_RECV cells only); marks of cells that
// were not interface cells cleared.  The fill fraction of every other
// interface cell was written by pass 1.
// the bytes of a 16-byte group of classes that are liquid or interface
__device__ inline bool any_live(const u32x4 &c)
{
    bool r = false;
#pragma unroll
    for (int k = 0; k < FS_CPT; ++k) {
        const int b = byte_of(c, k);
        r = r || b == FS_IF || b == FS_LIQ;
    }
    return r;
}

template <class S>
__global__ __launch_bounds__(BLOCK) void k_fs_final(const BatchArgs a)
{
    using R = typename Codec<S>::R;
    const FsTile t = fs_tile(a);
    const LatDev *__restrict__ L = t.L;
    const GL FsDev *__restrict__ F = t.F;
    const int dst = (t.flags & 1) ^ 1;
    // do this thread's cells keep their row in the next pass 1: a cell that is
    // liquid or interface after this step (it was, or was born), or one
    // flagged in this step (pass 1 clears its flag)
    bool keep = false;
    uint32_t mask = 0;
    const bool work = row_work(t);
    if (work) {
        const u32x4 f = ld16(F->w1, t.base), m2 = ld16(F->w2, t.base), c0 = ld16(F->cls, t.base);
        keep = any_byte(f) || any_live(c0) || ((m2.x | m2.y | m2.z | m2.w) & 0x01010101u * FS_BORN) != 0u;
        if (any_byte(f) || any_byte(m2))
            for (int k = 0; k < FS_CPT; ++k)
                if (t.base + k < t.ncell && (byte_of(f, k) || byte_of(m2, k))) mask |= 1u << k;
    }
    if (__builtin_amdgcn_ballot_w64(mask != 0u) != 0) {
        for_items(mask, t.base, [&](uint32_t idx) {
            // a worked cell's own bytes are written in this pass only by itself
            const int w1 = ldg<uint8_t>(F->w1, idx), w2 = ldg<uint8_t>(F->w2, idx);
            if (w1 == FS_FILL) {
                stg<uint8_t>(F->cls, idx, FS_LIQ);
                return;
            }
            if (empties(w1, w2)) {
                stg<uint8_t>(F->cls, idx, FS_GAS);
                return;
            }
            if (!(w2 & (FS_BORN | FS_TO_IF | FS_RECV))) return;   // kept, no share
            double m, r;
            if (w2 & FS_BORN) {
                m = 0.0;
                r = ldg<double>(F->rho, idx);
            } else if (w2 & FS_TO_IF) {     // a liquid cell: m = its density
                R o[NQ];
                load_cell<S>(L->f[dst], L->fm[dst], L->pstride, idx, o);
                R dr = 0;
#pragma unroll
                for (int q = 0; q < NQ; ++q) dr += o[q];
                r = 1.0 + double(dr);
                m = r;
            } else {
                m = ldg<double>(F->mass, idx);
                r = ldg<double>(F->rho, idx);
            }
            if (w2 & FS_RECV) {
                const Nbr b = nbr_of(L, idx);
                for_links([&](auto qc) {
                    constexpr int Q = decltype(qc)::value;
                    const uint32_t j = shifted<Q, 1>(b);
                    if (converts(F, j)) m += ldg<double>(F->share, j);
                });
            }
            stg<double>(F->mass, idx, m);
            stg<double>(F->lam[dst], idx, m / r);
            if (w2 & (FS_BORN | FS_TO_IF)) {
                stg<uint8_t>(F->cls, idx, FS_IF);
                stg<uint8_t>(F->w2, idx, 0);
                fs_list_row(F, dst, idx / BLOCK, (t.ncell + BLOCK - 1) / BLOCK);
            }
        });
    }
    // one flag per row of BLOCK cells: the BLOCK / FS_CPT consecutive lanes
    // that cover a row with work vote, the first of them writes it and clears
    // the row's work byte; a row without work changed no class and has no
    // flag, so it keeps the flag pass 1 read
    constexpr int TPR = BLOCK / FS_CPT;
    static_assert(64 % TPR == 0, "a row's lanes lie in one wave");
    const uint64_t vote = __builtin_amdgcn_ballot_w64(keep);
    const int lane = threadIdx.x & 63;
    if (lane % TPR == 0 && t.base < t.ncell) {
        const uint32_t row = t.base / BLOCK;
        if (work) {
            stg<uint8_t>(F->rowlive[dst], row, ((vote >> lane) & ((uint64_t(1) << TPR) - 1)) != 0 ? 1 : 0);
            stg<uint8_t>(F->rowwork, row, 0);
        } else {
            stg<uint8_t>(F->rowlive[dst], row, ldg<uint8_t>(F->rowlive[dst ^ 1], row));
        }
    }
}

// Moment steps, after pass 5 (one thread per cell, the step grid): rho, V'
// and lambda of the step into the moments buffer (gas and solid cells 0) and
// the FP64 diagnostic partials over liquid and interface cells, with
// diag[4] = the liquid mass (m of interface cells, rho of liquid cells).
template <class S>
__global__ __launch_bounds__(BLOCK) void k_fs_moments(const BatchArgs a)
{
    using R = typename Codec<S>::R;
    [[maybe_unused]] constexpr bool HW = HwMath<S>::value;
    const FsCell c = fs_cell(a);
    const LatDev *__restrict__ L = c.L;
    const GL FsDev *__restrict__ F = c.F;
    const uint32_t idx = c.idx, ncell = c.ncell;
    const int dst = (c.flags & 1) ^ 1;
    double part[NPART] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (idx < ncell) {
        const int nt = ldg<uint8_t>(F->cls, idx);
        const bool live = nt == FS_IF || nt == FS_LIQ;
        void *M = L->mom;
        R rho = 0, u[3] = {0, 0, 0}, lam = 0;
        double m = 0.0;
        if (live) {
            rho = R(ldg<double>(F->rho, idx));
            for (int k = 0; k < 3; ++k) u[k] = R(ldp<double>(F->u, ncell, k, idx));
            lam = nt == FS_LIQ ? R(1) : R(ldg<double>(F->lam[dst], idx));
            m = nt == FS_LIQ ? ldg<double>(F->rho, idx) : ldg<double>(F->mass, idx);
        }
        const R up[3] = {ldp<R>(M, ncell, 1, idx), ldp<R>(M, ncell, 2, idx), ldp<R>(M, ncell, 3, idx)};
        stg<R>(M, idx, rho);
        stp<R>(M, ncell, 1, idx, u[0]);
        stp<R>(M, ncell, 2, idx, u[1]);
        stp<R>(M, ncell, 3, idx, u[2]);
        stp<R>(M, ncell, 4, idx, lam);
        if (live) {
            diag_contrib<R>(part, rho, u, lam, R(0), up);
            part[4] = m;
        }
    }
    block_reduce_store(part, L->partials + size_t(c.lb) * NPART);
}

// ---------------------------------------------------------------------------
// set-up: classes from the initial fill fraction c0 (>= 1 liquid, <= 0 gas,
// else interface), then liquid cells next to gas cells become interface
// cells; masses m = lambda rho0, fill fractions, the moments of step 0
// (gas cells read 0) and their diagnostics.

template <class R>
__global__ __launch_bounds__(BLOCK) void k_fs_init_classes(const LatDev *L, const R *c0)
{
    const uint32_t idx = blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= uint32_t(L->ncell)) return;
    const GL FsDev *F = fs_of(L);
    int x, y, z, face;
    coords(L, idx, x, y, z);
    const int type = cell_type(L, x, y, z, link_word(L, idx), face);
    const R l = c0 ? c0[idx] : R(0);
    stg<uint8_t>(F->w1, idx, type != CELL_FLUID ? FS_SOLID : (l >= R(1) ? FS_LIQ : (l <= R(0) ? FS_GAS : FS_IF)));
}

template <class R>
__global__ __launch_bounds__(BLOCK) void k_fs_init_state(const LatDev *L, const R *c0, const R *rho0)
{
    const uint32_t ncell = L->ncell;
    const uint32_t idx = blockIdx.x * BLOCK + threadIdx.x;
    const GL FsDev *F = fs_of(L);
    double part[NPART] = {0, 0, 0, 0, 0, 0, 0, 0, 0};
    if (idx < ncell) {
        int cls = ldg<uint8_t>(F->w1, idx);
        if (cls == FS_LIQ) {
            int x, y, z;
            coords(L, idx, x, y, z);
            const Nbr b = neighbours(L, x, y, z, 0u);
            bool near_gas = false;
            for_links([&](auto qc) {
                constexpr int Q = decltype(qc)::value;
                near_gas = near_gas || ldg<uint8_t>(F->w1, shifted<Q, 1>(b)) == FS_GAS;
            });
            if (near_gas) cls = FS_IF;
        }
        const double r0 = rho0 ? double(rho0[idx]) : 1.0;
        double l = c0 ? double(c0[idx]) : 0.0;
        l = cls == FS_LIQ ? 1.0 : (cls == FS_IF ? fmin(fmax(l, 0.0), 1.0) : 0.0);
        stg<uint8_t>(F->cls, idx, (unsigned char)cls);
        stg<uint8_t>(F->w2, idx, 0);
        stg<double>(F->lam[0], idx, l);
        stg<double>(F->lam[1], idx, l);
        stg<double>(F->mass, idx, l * r0);
        stg<double>(F->rho, idx, cls == FS_IF || cls == FS_LIQ ? r0 : 0.0);
        void *M = L->mom;
        const bool live = cls == FS_IF || cls == FS_LIQ;
        if (!live) {
            stg<R>(M, idx, R(0));
            for (int k = 1; k < 4; ++k) stp<R>(M, ncell, k, idx, R(0));
        }
        stp<R>(M, ncell, 4, idx, R(l));
        if (live) {
            const R u[3] = {ldp<R>(M, ncell, 1, idx), ldp<R>(M, ncell, 2, idx), ldp<R>(M, ncell, 3, idx)};
            diag_contrib<R>(part, ldg<R>(M, idx), u, R(l), R(0), u);
            part[4] = l * r0;
        }
    }
    // empty launch-order lists; every row visited by the first pass 1
    if (threadIdx.x == 0) {
        stg<uint32_t>(F->hpos[0], blockIdx.x, 0u);
        stg<uint32_t>(F->hpos[1], blockIdx.x, 0u);
        stg<uint8_t>(F->rowlive[0], blockIdx.x, 1);
        stg<uint8_t>(F->rowlive[1], blockIdx.x, 1);
        stg<uint8_t>(F->rowwork, blockIdx.x, 0);
        if (blockIdx.x == 0) {
            stg<uint32_t>(F->hcount[0], 0, 0u);
            stg<uint32_t>(F->hcount[1], 0, 0u);
        }
    }
    block_reduce_store(part, L->partials + size_t(blockIdx.x) * NPART);
}

// classes, masses and fill fractions for lbm_free_surface: m of interface
// cells, rho (from the current populations) of liquid cells, 0 elsewhere;
// lambda = m / rho of interface cells as the step stored it, 1 for liquid
// cells, 0 elsewhere
template <class S>
__global__ __launch_bounds__(BLOCK) void k_fs_export(const LatDev *L, int src, unsigned char *cls, double *mass,
                                                     double *lam)
{
    using R = typename Codec<S>::R;
    [[maybe_unused]] constexpr bool HW = HwMath<S>::value;
    const uint32_t idx = blockIdx.x * BLOCK + threadIdx.x;
    if (idx >= uint32_t(L->ncell)) return;
    const GL FsDev *F = fs_of(L);
    const int c = ldg<uint8_t>(F->cls, idx);
    if (cls) cls[idx] = (unsigned char)c;
    if (mass) {
        double m = 0.0;
        if (c == FS_IF) {
            m = ldg<double>(F->mass, idx);
        } else if (c == FS_LIQ) {
            R o[NQ];
            load_cell<S>(L->f[src], L->fm[src], L->pstride, idx, o);
            R dr = 0;
#pragma unroll
            for (int q = 0; q < NQ; ++q) dr += o[q];
            m = 1.0 + double(dr);
        }
        mass[idx] = m;
    }
    if (lam) lam[idx] = c == FS_IF ? ldg<double>(F->lam[src], idx) : (c == FS_LIQ ? 1.0 : 0.0);
}

}  // namespace plbm
