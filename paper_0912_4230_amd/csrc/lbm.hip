// lbm.hip -- host side of the C ABI declared in include/lbm.h: argument
// validation, workspace layout, kernel launch sequencing and diagnostics
// read-back.  The library never allocates device memory; every buffer lives
// in the caller's workspace.
#include "lbm.h"

#include <math.h>
#include <stdint.h>
#include <string.h>

#include <algorithm>
#include <mutex>
#include <new>

#include "kernels.hpp"
#include "freesurf.hpp"

using namespace plbm;

namespace {

constexpr size_t ALIGN = 256;

size_t align_up(size_t v) { return (v + ALIGN - 1) / ALIGN * ALIGN; }

size_t storage_bytes(int storage)
{
    switch (storage) {
    case LBM_F64: return 8;
    case LBM_F32: return 4;
    default: return 2;
    }
}

size_t real_bytes(int storage) { return storage == LBM_F64 ? 8 : 4; }

// Elements from one population plane to the next.  Every plane starts on a
// 256-byte boundary (so that a wave's stores cover whole cache lines; with
// planes at odd offsets two waves share the lines at every boundary) and is
// followed by 512 bytes of padding: the 38 read and 38 write streams of a
// step then do not all sit at the same offset modulo a power-of-two plane
// size.  Measured against unpadded planes: FP32 256^3 -2%, 512^3 -7%; 16-bit
// -4 to -7% (256, 768, 1024 and 2048 bytes measured no better).  Planes of a
// whole number of MiB and at least 256 MiB (512^3 in FP32 and 16 bits) take
// 512 KiB more: with the 512-byte stagger alone their streams still crowd
// the same HBM channels (512^3, two runs each: BF16 5.52 -> 4.38-4.57 ms,
// FP16 5.49 -> 4.49, FP32 8.29 -> 8.03, split forms unchanged), while at
// 256^3 (64 MiB planes) the larger pad measured 12% slower in FP32.
#ifndef PLBM_BIG_PAD
#define PLBM_BIG_PAD (512 * 1024 + 512)
#endif
size_t plane_stride_of(size_t n, size_t sb)
{
    const size_t per = 256 / sb;
    const size_t base = (n + per - 1) / per * per, bytes = base * sb;
    const size_t MiB = size_t(1) << 20;
    const size_t pad = (bytes >= 256 * MiB && bytes % MiB == 0) ? size_t(PLBM_BIG_PAD) : 512;
    return base + pad / sb;
}

size_t plane_stride(const lbm_desc *d)
{
    return plane_stride_of((size_t)d->nx * d->ny * d->nz, storage_bytes(d->storage));
}

// Miscible lattices in 16-bit storage keep f and h in paired planes of
// 32-bit words (and split codecs their two masses as one 8-byte pair per
// cell); the planes are padded as planes of 4-byte elements.
bool paired_storage(const lbm_desc *d) { return d->physics == LBM_MISCIBLE && storage_bytes(d->storage) == 2; }

size_t pair_plane_stride(const lbm_desc *d)
{
    return plane_stride_of((size_t)d->nx * d->ny * d->nz, 2 * storage_bytes(d->storage));
}

struct Layout {
    size_t lat, err, diag, partials, eps, kinv, mom, rho1, links, f0, f1, h0, h1, fm0, fm1, hm0, hm1;
    size_t fs, fs_cls, fs_w1, fs_w2, fs_mass, fs_lam, fs_rho, fs_share, fs_u, fs_hot;
    size_t ms, msx[MAXSPX][2], msm[MAXSPX][2], total;
};

// solutes beyond the first
int extra_species(const lbm_desc *d) { return (d->physics == LBM_MISCIBLE && d->nspecies > 1) ? d->nspecies - 1 : 0; }

bool split_storage(int storage) { return storage == LBM_BF16_SPLIT || storage == LBM_F16_SPLIT; }

// a second lattice (solute or fluid 1)
bool two_lattices(int physics) { return physics == LBM_MISCIBLE || physics == LBM_IMMISCIBLE; }

bool is_fin(double v) { return isfinite(v) != 0; }

// Validation of a description; no GPU call.
bool valid_desc(const lbm_desc *d)
{
    if (!d) return false;
    if (d->nx < 1 || d->ny < 1 || d->nz < 1) return false;
    const long long ncell = (long long)d->nx * d->ny * d->nz;
    if (ncell > (1LL << 31) - BLOCK) return false;
    // planes are addressed by 32-bit byte offsets from a uniform base: a
    // field plane, or a pair of population planes for the bounce-back selects
    if (d->physics < LBM_SINGLE || d->physics > LBM_FREESURF) return false;
    if (d->storage < LBM_F64 || d->storage > LBM_F16_SPLIT) return false;
    const unsigned long long pair = 2ULL * plane_stride(d) * storage_bytes(d->storage);
    if ((unsigned long long)ncell * real_bytes(d->storage) > (1ULL << 32) || pair > (1ULL << 32)) return false;
    if (paired_storage(d) && 2ULL * pair_plane_stride(d) * 2 * storage_bytes(d->storage) > (1ULL << 32)) return false;
    // free surface: per-cell doubles addressed by 32-bit byte offsets; no reservoirs
    if (d->physics == LBM_FREESURF) {
        if ((unsigned long long)ncell * 8ULL > (1ULL << 32)) return false;
        for (int f = 0; f < 6; ++f)
            if (d->face[f].kind == LBM_FACE_RESERVOIR) return false;
    }
    const int n[3] = {d->nx, d->ny, d->nz};
    for (int a = 0; a < 3; ++a) {
        const int k0 = d->face[2 * a].kind, k1 = d->face[2 * a + 1].kind;
        for (int k : {k0, k1})
            if (k < LBM_FACE_PERIODIC || k > LBM_FACE_RESERVOIR) return false;
        if ((k0 == LBM_FACE_PERIODIC) != (k1 == LBM_FACE_PERIODIC)) return false;
        if (k0 != LBM_FACE_PERIODIC && n[a] < 3) return false;
    }
    for (int f = 0; f < 6; ++f) {
        const lbm_face &F = d->face[f];
        if (F.kind == LBM_FACE_RESERVOIR && !(F.rho > 0.0 && is_fin(F.rho) && is_fin(F.conc))) return false;
        if (F.kind == LBM_FACE_WALL && !is_fin(F.contact_angle_deg)) return false;
    }
    for (int a = 0; a < 3; ++a)
        if (!is_fin(d->G[a])) return false;
    if (d->physics == LBM_IMMISCIBLE) {
        if (!(d->tau1 > 0.5) || !(d->tau2 > 0.5) || !is_fin(d->tau1) || !is_fin(d->tau2)) return false;
        if (!(d->A >= 0.0) || !is_fin(d->A)) return false;
        if (!(d->beta >= 0.0 && d->beta <= 1.0)) return false;
    } else {
        if (!(d->nu0 > 0.0) || !is_fin(d->nu0)) return false;
        if (!(d->a0 >= 0.0) || !(d->a1 >= 0.0) || !(d->a0 + d->a1 > 0.0)) return false;
        if (!is_fin(d->a0) || !is_fin(d->a1) || !is_fin(d->alpha) || !is_fin(d->k1) || !is_fin(d->k0)) return false;
        if (!(d->cap > 0.0)) return false;
        // surface tension: the two-fluid model, or a free surface
        if (d->physics == LBM_FREESURF ? !(d->A >= 0.0 && is_fin(d->A)) : d->A != 0.0) return false;
    }
    if (d->physics == LBM_MISCIBLE && (!(d->tau_d > 0.5) || !is_fin(d->tau_d))) return false;
    if (d->diag_every < 0) return false;
    if (d->solid_mask != 0 && d->solid_mask != 1) return false;
    if (d->full_tensor != 0 && d->full_tensor != 1) return false;
    if (d->solid_mask && d->physics == LBM_IMMISCIBLE && !is_fin(d->solid_contact_angle_deg)) return false;
    if (d->nspecies < 0 || d->nspecies > LBM_MAX_SPECIES) return false;
    if (d->nspecies > 1 && d->physics != LBM_MISCIBLE) return false;
    for (int k = 0; k < extra_species(d); ++k) {
        if (!(d->tau_d_x[k] > 0.5) || !is_fin(d->tau_d_x[k])) return false;
        for (int f = 0; f < 6; ++f)
            if (d->face[f].kind == LBM_FACE_RESERVOIR && !is_fin(d->face_conc_x[k][f])) return false;
    }
    return true;
}

Layout layout(const lbm_desc *d)
{
    Layout L;
    const size_t n = (size_t)d->nx * d->ny * d->nz;
    const size_t nb = (n + BLOCK - 1) / BLOCK;
    const size_t sb = storage_bytes(d->storage), rb = real_bytes(d->storage);
    size_t o = 0;
    L.lat = o;       o = align_up(o + sizeof(LatDev));
    L.err = o;       o = align_up(o + sizeof(int));
    L.diag = o;      o = align_up(o + 8 * sizeof(double));
    L.partials = o;  o = align_up(o + nb * NPART * sizeof(double));
    L.eps = o;       o = align_up(o + n * rb);
    L.kinv = o;      o = align_up(o + (d->full_tensor ? 7 : 3) * n * rb);
    L.mom = o;       o = align_up(o + (5 + extra_species(d)) * n * rb);
    L.rho1 = o;      if (d->physics == LBM_IMMISCIBLE) o = align_up(o + n * rb);
    L.links = o;     if (d->solid_mask) o = align_up(o + n * sizeof(uint32_t));
    const size_t ps = plane_stride(d);
    const bool sp = split_storage(d->storage), two = two_lattices(d->physics), pr = paired_storage(d);
    // paired: f0 / f1 hold both lattices, fm0 / fm1 both masses
    const size_t fbytes = pr ? NQ * pair_plane_stride(d) * 2 * sb : NQ * ps * sb;
    L.f0 = o;        o = align_up(o + fbytes);
    L.f1 = o;        o = align_up(o + fbytes);
    L.h0 = o;        if (two && !pr) o = align_up(o + NQ * ps * sb);
    L.h1 = o;        if (two && !pr) o = align_up(o + NQ * ps * sb);
    L.fm0 = o;       if (sp) o = align_up(o + n * sizeof(float) * (pr ? 2 : 1));
    L.fm1 = o;       if (sp) o = align_up(o + n * sizeof(float) * (pr ? 2 : 1));
    L.hm0 = o;       if (sp && two && !pr) o = align_up(o + n * sizeof(float));
    L.hm1 = o;       if (sp && two && !pr) o = align_up(o + n * sizeof(float));
    const bool fs = d->physics == LBM_FREESURF;
    // free surface: the FsDev block (+ the lost-mass counter), three byte
    // planes, five double planes (m, two of lambda, rho, share) and the 3
    // double planes of V', two launch-order sets (row list, per-row
    // positions, count, per-row live flags) and the per-row work flags of the
    // class passes
    L.fs = o;        if (fs) o = align_up(o + sizeof(FsDev) + sizeof(double));
    L.fs_cls = o;    if (fs) o = align_up(o + n);
    L.fs_w1 = o;     if (fs) o = align_up(o + n);
    L.fs_w2 = o;     if (fs) o = align_up(o + n);
    L.fs_mass = o;   if (fs) o = align_up(o + n * sizeof(double));
    L.fs_lam = o;    if (fs) o = align_up(o + 2 * n * sizeof(double));
    L.fs_rho = o;    if (fs) o = align_up(o + n * sizeof(double));
    L.fs_share = o;  if (fs) o = align_up(o + n * sizeof(double));
    L.fs_u = o;      if (fs) o = align_up(o + 3 * n * sizeof(double));
    const size_t rows4 = align_up((n + BLOCK - 1) / BLOCK * 4), rows1 = align_up((n + BLOCK - 1) / BLOCK);
    L.fs_hot = o;    if (fs) o = align_up(o + 2 * (2 * rows4 + 256 + rows1) + rows1);
    // further solutes: the MsDev block, per solute two population copies and,
    // split storage, two mass planes
    const int nsx = extra_species(d);
    L.ms = o;        if (nsx) o = align_up(o + sizeof(MsDev));
    for (int k = 0; k < MAXSPX; ++k)
        for (int c = 0; c < 2; ++c) {
            L.msx[k][c] = o;
            if (k < nsx) o = align_up(o + NQ * ps * sb);
        }
    for (int k = 0; k < MAXSPX; ++k)
        for (int c = 0; c < 2; ++c) {
            L.msm[k][c] = o;
            if (k < nsx && sp) o = align_up(o + n * sizeof(float));
        }
    L.total = o;
    return L;
}

// (m, s1, s2) of the division by d >= 1 (Granlund and Montgomery 1994):
// l = ceil(log2 d), m = floor(2^32 (2^l - d) / d) + 1, s1 = min(l, 1),
// s2 = max(l - 1, 0); then n / d = (t + ((n - t) >> s1)) >> s2, t = mulhi(m, n).
void magic_divisor(uint32_t d, uint32_t g[3])
{
    uint32_t l = 0;
    while ((uint64_t(1) << l) < d) ++l;
    const uint64_t m = ((uint64_t(1) << 32) * ((uint64_t(1) << l) - d)) / d + 1;
    g[0] = uint32_t(m);
    g[1] = l < 1 ? l : 1;
    g[2] = l > 0 ? l - 1 : 0;
}

double time_factor(const lbm_desc *d, double t)
{
    double tf = d->a0 + d->a1 * exp(d->alpha * t);
    if (tf > d->cap) tf = d->cap;
    return tf;
}

}  // namespace

struct lbm_sim {
    lbm_desc d;
    hipStream_t stream;
    char *ws;
    size_t ws_bytes;
    Layout lay;
    LatDev host;        // host copy of the device parameter block
    FsDev fs;           // host copy of the free-surface block (free surface only)
    MsDev ms;           // host copy of the further-solute block (several solutes only)
    LatDev *dev;        // the device parameter block (inside ws)
    long long steps;    // completed steps
    int cur;            // copy holding the current state
    int ready;          // medium set
    int nblocks;
    int device;
    int in_scratch;     // workspace = this device's scratch array (lbm_create_static)
};

namespace {

lbm_status dev_err(hipError_t e) { return e == hipSuccess ? LBM_OK : LBM_EDEVICE; }

using Launch = void (*)(const BatchArgs &, int blocks, hipStream_t);

// Dynamic LDS reserved by every step launch (unused by the kernel): it caps
// residency at 4 blocks of 256 threads per CU, i.e. 4 waves per SIMD.  Step
// kernels that fit in fewer than 103 VGPRs would otherwise run 5 waves per
// SIMD, which measured 2-3% slower on the FP32 miscible and two-fluid steps.
constexpr size_t STEP_LDS_RESERVE = 33 * 1024;

template <int P, class S, bool FT, bool MS = false>
void launch_step(const BatchArgs &a, int blocks, hipStream_t s)
{
    const size_t lds = StepWaves<P, S, FT, MS>::value == 5 ? 0 : STEP_LDS_RESERVE;
    hipLaunchKernelGGL((k_step<P, S, FT, MS>), dim3(blocks), dim3(BLOCK), lds, s, a);
}

template <class S>
void launch_colour(const BatchArgs &a, int blocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_colour<S>), dim3(blocks), dim3(BLOCK), 0, s, a);
}

template <int P, bool FT, bool MS = false>
Launch step_for_storage(int storage)
{
    switch (storage) {
    case LBM_F64: return launch_step<P, double, FT, MS>;
    case LBM_F32: return launch_step<P, float, FT, MS>;
    case LBM_BF16_DEV: return launch_step<P, bf16_t, FT, MS>;
    case LBM_F16_DEV: return launch_step<P, f16_t, FT, MS>;
    case LBM_BF16_SPLIT: return launch_step<P, bf16s_t, FT, MS>;
    default: return launch_step<P, f16s_t, FT, MS>;
    }
}

template <int P>
Launch step_for_tensor(int storage, bool full_tensor)
{
    return full_tensor ? step_for_storage<P, true>(storage) : step_for_storage<P, false>(storage);
}

// miscible lattices with further solutes
Launch step_for_species(int storage, bool full_tensor)
{
    return full_tensor ? step_for_storage<PH_MISCIBLE, true, true>(storage)
                       : step_for_storage<PH_MISCIBLE, false, true>(storage);
}

// Free surface: the stream/collide pass on the step grid (a), the class
// passes on the grid of BLOCK * FS_CPT cells per block (a16), the moments
// pass on the step grid of the lattices at a moment step (am, may be empty).
// Blocks of the free-surface pass 1 that take the listed rows first: 1/32 of
// the rows, at least 64 (all rows of a smaller lattice).
int fs_prefix_blocks(int rows) { return std::min(rows, std::max(64, rows / 32)); }

struct FsGrids {
    BatchArgs a, a16, am;
    int blocks, blocks16, blocksm;
};

#ifndef PLBM_FS_LDS
#define PLBM_FS_LDS 0
#endif

template <class S, bool FT, bool ST>
void launch_fs(const FsGrids &g, hipStream_t s)
{
    hipLaunchKernelGGL((k_fs_step<S, FT, ST>), dim3(g.blocks), dim3(BLOCK), PLBM_FS_LDS, s, g.a);
    hipLaunchKernelGGL(k_fs_mark_fill, dim3(g.blocks16), dim3(BLOCK), 0, s, g.a16);
    hipLaunchKernelGGL((k_fs_mark_empty<S>), dim3(g.blocks16), dim3(BLOCK), 0, s, g.a16);
    hipLaunchKernelGGL(k_fs_excess, dim3(g.blocks16), dim3(BLOCK), 0, s, g.a16);
    hipLaunchKernelGGL((k_fs_final<S>), dim3(g.blocks16), dim3(BLOCK), 0, s, g.a16);
    if (g.blocksm) hipLaunchKernelGGL((k_fs_moments<S>), dim3(g.blocksm), dim3(BLOCK), 0, s, g.am);
}

using FsLaunch = void (*)(const FsGrids &, hipStream_t);

template <bool FT, bool ST>
FsLaunch fs_for_storage(int storage)
{
    switch (storage) {
    case LBM_F64: return launch_fs<double, FT, ST>;
    case LBM_F32: return launch_fs<float, FT, ST>;
    case LBM_BF16_DEV: return launch_fs<bf16_t, FT, ST>;
    case LBM_F16_DEV: return launch_fs<f16_t, FT, ST>;
    case LBM_BF16_SPLIT: return launch_fs<bf16s_t, FT, ST>;
    default: return launch_fs<f16s_t, FT, ST>;
    }
}

// the surface-tension form when any lattice of the batch has A != 0 (with
// A = 0 it computes exactly what the plain form does)
FsLaunch fs_launcher(int storage, bool full_tensor, bool st)
{
    if (st) return full_tensor ? fs_for_storage<true, true>(storage) : fs_for_storage<false, true>(storage);
    return full_tensor ? fs_for_storage<true, false>(storage) : fs_for_storage<false, false>(storage);
}

Launch step_launcher(int physics, int storage, bool full_tensor)
{
    switch (physics) {
    case LBM_SINGLE: return step_for_tensor<PH_SINGLE>(storage, full_tensor);
    case LBM_MISCIBLE: return step_for_tensor<PH_MISCIBLE>(storage, full_tensor);
    default: return step_for_tensor<PH_IMMISCIBLE>(storage, full_tensor);
    }
}

Launch colour_launcher(int storage)
{
    switch (storage) {
    case LBM_F64: return launch_colour<double>;
    case LBM_F32: return launch_colour<float>;
    case LBM_BF16_DEV: return launch_colour<bf16_t>;
    case LBM_F16_DEV: return launch_colour<f16_t>;
    case LBM_BF16_SPLIT: return launch_colour<bf16s_t>;
    default: return launch_colour<f16s_t>;
    }
}

template <int P, class S>
void launch_init(const lbm_sim *h, const lbm_medium *m, int blocks)
{
    using R = typename Codec<S>::R;
    InitArgs<R> ia;
    ia.L = h->dev;
    ia.rho0 = static_cast<const R *>(m->rho0);
    ia.vel0 = static_cast<const R *>(m->vel0);
    ia.c0 = static_cast<const R *>(m->c0);
    ia.nuc0 = h->d.nu0 * time_factor(&h->d, 0.0);
    if (P == PH_IMMISCIBLE)
        hipLaunchKernelGGL((k_init_colour<R>), dim3(blocks), dim3(BLOCK), 0, h->stream, ia);
    hipLaunchKernelGGL((k_init<P, S>), dim3(blocks), dim3(BLOCK), 0, h->stream, ia);
    hipLaunchKernelGGL((k_diag_moments<R>), dim3(blocks), dim3(BLOCK), 0, h->stream, (const LatDev *)h->dev);
}

// free surface: the single-fluid set-up of the populations, then the classes,
// masses and fill fractions, the moments of step 0 and their diagnostic partials
template <class S>
void launch_fs_init(const lbm_sim *h, const lbm_medium *m, int blocks)
{
    using R = typename Codec<S>::R;
    InitArgs<R> ia;
    ia.L = h->dev;
    ia.rho0 = static_cast<const R *>(m->rho0);
    ia.vel0 = static_cast<const R *>(m->vel0);
    ia.c0 = static_cast<const R *>(m->c0);
    ia.nuc0 = h->d.nu0 * time_factor(&h->d, 0.0);
    const LatDev *L = h->dev;
    hipLaunchKernelGGL((k_init<PH_SINGLE, S>), dim3(blocks), dim3(BLOCK), 0, h->stream, ia);
    hipLaunchKernelGGL(k_fs_init_classes<R>, dim3(blocks), dim3(BLOCK), 0, h->stream, L, ia.c0);
    hipLaunchKernelGGL(k_fs_init_state<R>, dim3(blocks), dim3(BLOCK), 0, h->stream, L, ia.c0, ia.rho0);
}

void fs_init(const lbm_sim *h, const lbm_medium *m, int blocks)
{
    switch (h->d.storage) {
    case LBM_F64: launch_fs_init<double>(h, m, blocks); break;
    case LBM_F32: launch_fs_init<float>(h, m, blocks); break;
    case LBM_BF16_DEV: launch_fs_init<bf16_t>(h, m, blocks); break;
    case LBM_F16_DEV: launch_fs_init<f16_t>(h, m, blocks); break;
    case LBM_BF16_SPLIT: launch_fs_init<bf16s_t>(h, m, blocks); break;
    default: launch_fs_init<f16s_t>(h, m, blocks); break;
    }
}

template <int P>
void init_for_storage(const lbm_sim *h, const lbm_medium *m, int blocks)
{
    switch (h->d.storage) {
    case LBM_F64: launch_init<P, double>(h, m, blocks); break;
    case LBM_F32: launch_init<P, float>(h, m, blocks); break;
    case LBM_BF16_DEV: launch_init<P, bf16_t>(h, m, blocks); break;
    case LBM_F16_DEV: launch_init<P, f16_t>(h, m, blocks); break;
    case LBM_BF16_SPLIT: launch_init<P, bf16s_t>(h, m, blocks); break;
    default: launch_init<P, f16s_t>(h, m, blocks); break;
    }
}

// Is step t (1-based) of this handle a diagnostic step?
bool diag_step(const lbm_sim *h, long long t, bool last)
{
    return last || (h->d.diag_every > 0 && t % h->d.diag_every == 0);
}

// One batched step for lattices hs[0..n) of the same physics, storage and
// permeability form (diagonal or full tensor):
// [colour pass,] step kernel, [diagnostics second stage].
lbm_status launch_batch_step(lbm_sim *const *hs, const bool *last, int n)
{
    BatchArgs a;
    memset(&a, 0, sizeof(a));
    a.n = n;
    int total = 0;
    int ndiag = 0;
    BatchArgs diag;
    memset(&diag, 0, sizeof(diag));
    for (int i = 0; i < n; ++i) {
        const lbm_sim *h = hs[i];
        // every lattice's range starts on a whole XCD row group (row_group_remap)
        a.blk_start[i] = total;
        total += (h->nblocks + XCD_GROUP - 1) / XCD_GROUP * XCD_GROUP;
        a.lat[i] = h->dev;
        const long long t = h->steps + 1;
        const bool dg = diag_step(h, t, last[i]);
        a.flags[i] = h->cur | (dg ? 2 : 0);
        a.nuc[i] = h->d.nu0 * time_factor(&h->d, double(t));
        if (dg) diag.lat[ndiag++] = h->dev;
    }
    a.blk_start[n] = total;
    a.total_blocks = total;
    const lbm_sim *h0 = hs[0];
    if (h0->d.physics == LBM_FREESURF) {
        // pass 1: per lattice a prefix of blocks for the rows listed as
        // holding interface cells, then one block per row
        FsGrids g;
        g.a = a;
        int tp = 0;
        for (int i = 0; i < n; ++i) {
            g.a.blk_start[i] = tp;
            tp += fs_prefix_blocks(hs[i]->nblocks) + hs[i]->nblocks;
        }
        g.a.blk_start[n] = tp;
        g.a.total_blocks = tp;
        g.blocks = tp;
        memset(&g.a16, 0, sizeof(g.a16));
        memset(&g.am, 0, sizeof(g.am));
        int t16 = 0, tm = 0, nm = 0;
        for (int i = 0; i < n; ++i) {
            const lbm_sim *h = hs[i];
            const int nb16 = (h->host.ncell + BLOCK * FS_CPT - 1) / (BLOCK * FS_CPT);
            g.a16.blk_start[i] = t16;
            g.a16.lat[i] = h->dev;
            g.a16.flags[i] = a.flags[i];
            t16 += nb16;
            if (a.flags[i] & 2) {
                g.am.blk_start[nm] = tm;
                g.am.lat[nm] = h->dev;
                g.am.flags[nm] = a.flags[i];
                tm += h->nblocks;
                ++nm;
            }
        }
        g.a16.n = n;
        g.a16.blk_start[n] = t16;
        g.a16.total_blocks = t16;
        g.am.n = nm;
        g.am.blk_start[nm] = tm;
        g.am.total_blocks = tm;
        g.blocks16 = t16;
        g.blocksm = tm;
        bool st = false;
        for (int i = 0; i < n; ++i) st = st || hs[i]->d.A != 0.0;
        fs_launcher(h0->d.storage, h0->host.full_tensor != 0, st)(g, h0->stream);
    } else if (h0->host.ms) {
        step_for_species(h0->d.storage, h0->host.full_tensor != 0)(a, total, h0->stream);
    } else {
        if (h0->d.physics == LBM_IMMISCIBLE) colour_launcher(h0->d.storage)(a, total, h0->stream);
        step_launcher(h0->d.physics, h0->d.storage, h0->host.full_tensor != 0)(a, total, h0->stream);
    }
    if (ndiag) {
        diag.n = ndiag;
        hipLaunchKernelGGL(k_diag_final, dim3(ndiag), dim3(BLOCK), 0, h0->stream, diag);
    }
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return LBM_EDEVICE;
    for (int i = 0; i < n; ++i) {
        hs[i]->cur ^= 1;
        hs[i]->steps += 1;
    }
    return LBM_OK;
}

}  // namespace

extern "C" {

size_t lbm_workspace_bytes(const lbm_desc *d)
{
    if (!valid_desc(d)) return 0;
    return layout(d).total;
}

}  // extern "C"

namespace {

// Fill the zeroed handle h for description d (valid) with its workspace at
// dev_workspace (ws_bytes >= the layout's total) on device `device`.  No GPU
// call.
void setup_handle(lbm_sim *h, const lbm_desc *d, void *dev_workspace, size_t ws_bytes, void *hip_stream, int device)
{
    const Layout L = layout(d);
    h->d = *d;
    h->stream = static_cast<hipStream_t>(hip_stream);
    h->ws = static_cast<char *>(dev_workspace);
    h->ws_bytes = ws_bytes;
    h->lay = L;
    h->device = device;
    const size_t n = (size_t)d->nx * d->ny * d->nz;
    h->nblocks = int((n + BLOCK - 1) / BLOCK);

    LatDev &D = h->host;
    D.nx = d->nx;
    D.ny = d->ny;
    D.nz = d->nz;
    D.ncell = int(n);
    D.nblocks = h->nblocks;
    {
        const size_t plane_cells = (size_t)d->nx * d->ny;
        const size_t bpp = plane_cells / BLOCK;
        D.bpp = (PLBM_SLAB && plane_cells % BLOCK == 0 && bpp % 8 == 0) ? int(bpp) : 0;
    }
    D.pstride = uint32_t(plane_stride(d));
    D.ppstride = paired_storage(d) ? uint32_t(pair_plane_stride(d)) : 0;
    magic_divisor(uint32_t(d->nx), D.div_nx);
    magic_divisor(uint32_t(d->nx) * uint32_t(d->ny), D.div_nxy);
    D.physics = d->physics;
    D.forch = d->forchheimer ? 1 : 0;
    D.eps_grad = d->eps_gradient ? 1 : 0;
    for (int a = 0; a < 3; ++a) {
        for (int f = 2 * a; f < 2 * a + 2; ++f) {
            if (d->face[f].kind == LBM_FACE_WALL) D.wall_faces |= 1u << f;
            if (d->face[f].kind == LBM_FACE_RESERVOIR) D.res_faces |= 1u << f;
        }
        D.G[a] = d->G[a];
    }
    D.k1 = d->k1;
    D.k0 = d->k0;
    D.nu1 = (d->tau1 - 0.5) / 3.0;
    D.nu2 = (d->tau2 - 0.5) / 3.0;
    D.tau_d = d->tau_d;
    D.D = (d->tau_d - 0.5) / 3.0;
    D.A = d->A;
    D.beta = d->beta;
    const double pi = 3.14159265358979323846;
    for (int f = 0; f < 6; ++f) {
        D.face_rho[f] = d->face[f].rho;
        D.face_conc[f] = d->face[f].conc;
        D.face_cw[f] = 0.5 * (1.0 + cos(d->face[f].contact_angle_deg * pi / 180.0));
    }
    D.face_cw[6] = d->solid_mask ? 0.5 * (1.0 + cos(d->solid_contact_angle_deg * pi / 180.0)) : 0.5;
    char *w = h->ws;
    D.f[0] = w + L.f0;
    D.f[1] = w + L.f1;
    const bool sp = split_storage(d->storage), two = two_lattices(d->physics), pr = paired_storage(d);
    D.h[0] = two && !pr ? w + L.h0 : nullptr;
    D.h[1] = two && !pr ? w + L.h1 : nullptr;
    D.fm[0] = sp ? w + L.fm0 : nullptr;
    D.fm[1] = sp ? w + L.fm1 : nullptr;
    D.hm[0] = sp && two && !pr ? w + L.hm0 : nullptr;
    D.hm[1] = sp && two && !pr ? w + L.hm1 : nullptr;
    D.eps = w + L.eps;
    D.kinv = w + L.kinv;
    D.mom = w + L.mom;
    D.rho1 = d->physics == LBM_IMMISCIBLE ? w + L.rho1 : nullptr;
    D.links = d->solid_mask ? w + L.links : nullptr;
    if (extra_species(d)) {
        MsDev &X = h->ms;
        X.nsx = extra_species(d);
        for (int k = 0; k < X.nsx; ++k) {
            for (int c = 0; c < 2; ++c) {
                X.h[k][c] = w + L.msx[k][c];
                X.hm[k][c] = sp ? w + L.msm[k][c] : nullptr;
            }
            X.tau_d[k] = d->tau_d_x[k];
            X.D[k] = (d->tau_d_x[k] - 0.5) / 3.0;
            for (int f = 0; f < 6; ++f) X.face_conc[k][f] = d->face_conc_x[k][f];
        }
        D.ms = w + L.ms;
    }
    if (d->physics == LBM_FREESURF) {
        FsDev &F = h->fs;
        F.cls = reinterpret_cast<unsigned char *>(w + L.fs_cls);
        F.w1 = reinterpret_cast<unsigned char *>(w + L.fs_w1);
        F.w2 = reinterpret_cast<unsigned char *>(w + L.fs_w2);
        F.mass = reinterpret_cast<double *>(w + L.fs_mass);
        F.lam[0] = reinterpret_cast<double *>(w + L.fs_lam);
        F.lam[1] = F.lam[0] + n;
        F.rho = reinterpret_cast<double *>(w + L.fs_rho);
        F.share = reinterpret_cast<double *>(w + L.fs_share);
        F.u = reinterpret_cast<double *>(w + L.fs_u);
        F.lost = reinterpret_cast<double *>(w + L.fs + sizeof(FsDev));
        const size_t rows4 = align_up((n + BLOCK - 1) / BLOCK * 4), rows1 = align_up((n + BLOCK - 1) / BLOCK);
        for (int c = 0; c < 2; ++c) {
            char *base = w + L.fs_hot + c * (2 * rows4 + 256 + rows1);
            F.hlist[c] = reinterpret_cast<uint32_t *>(base);
            F.hpos[c] = reinterpret_cast<uint32_t *>(base + rows4);
            F.hcount[c] = reinterpret_cast<uint32_t *>(base + 2 * rows4);
            F.rowlive[c] = reinterpret_cast<unsigned char *>(base + 2 * rows4 + 256);
        }
        F.rowwork = reinterpret_cast<unsigned char *>(w + L.fs_hot + 2 * (2 * rows4 + 256 + rows1));
        D.fs = w + L.fs;
    }
    D.partials = reinterpret_cast<double *>(w + L.partials);
    D.diag = reinterpret_cast<double *>(w + L.diag);
    D.err = reinterpret_cast<int *>(w + L.err);
    h->dev = reinterpret_cast<LatDev *>(w + L.lat);
}

// ---------------------------------------------------------------------------
// Checkpoints.  A lattice's state is its workspace (populations of both
// copies, masses, medium planes, diagnostics, free-surface planes and lists,
// further solutes) plus three host values: the completed steps, the copy
// holding the current state and the medium's form (uniform or per cell).
// Three blocks of the workspace hold absolute device pointers (the parameter
// block at its start, the free-surface and further-solute blocks) and belong
// to the workspace they sit in; a checkpoint is every other byte, after a
// header that records what the layout depends on, so that it can be loaded
// into another workspace of the same description and medium.
struct CkptHeader {
    uint64_t magic;
    uint32_t version, cur;
    int64_t steps;
    uint64_t total, payload;
    int32_t nx, ny, nz, physics, storage, nspecies, full_tensor, solid_mask;
    int32_t uniform_eps, uniform_kinv, medium_tensor, pad;
    double eps_u, kinv_u[3];
};
constexpr uint64_t CKPT_MAGIC = 0x54504b434d424c50ull;   // "PLBMCKPT"

struct Span {
    size_t off, len;
};

// the byte ranges of the workspace a checkpoint holds, in layout order
int state_spans(const lbm_sim *h, Span out[3])
{
    const Layout &L = h->lay;
    size_t at = L.err;
    int n = 0;
    if (h->host.fs) {
        out[n++] = {at, L.fs - at};
        at = L.fs + sizeof(FsDev);
    }
    if (h->host.ms) {
        out[n++] = {at, L.ms - at};
        at = L.ms + sizeof(MsDev);
    }
    out[n++] = {at, L.total - at};
    return n;
}

CkptHeader ckpt_header(const lbm_sim *h)
{
    CkptHeader H;
    memset(&H, 0, sizeof(H));
    H.magic = CKPT_MAGIC;
    H.version = 1;
    H.cur = uint32_t(h->cur);
    H.steps = h->steps;
    H.total = h->lay.total;
    Span sp[3];
    const int n = state_spans(h, sp);
    for (int k = 0; k < n; ++k) H.payload += sp[k].len;
    H.nx = h->d.nx;
    H.ny = h->d.ny;
    H.nz = h->d.nz;
    H.physics = h->d.physics;
    H.storage = h->d.storage;
    H.nspecies = h->d.nspecies;
    H.full_tensor = h->d.full_tensor;
    H.solid_mask = h->d.solid_mask;
    H.uniform_eps = h->host.uniform_eps;
    H.uniform_kinv = h->host.uniform_kinv;
    H.medium_tensor = h->host.full_tensor;
    H.eps_u = h->host.uniform_eps ? h->host.eps_u : 0.0;
    for (int a = 0; a < 3; ++a) H.kinv_u[a] = h->host.uniform_kinv ? h->host.kinv_u[a] : 0.0;
    return H;
}

// a checkpoint header fits a handle: same layout and the same medium form
bool ckpt_fits(const CkptHeader &H, const CkptHeader &E)
{
    return H.magic == CKPT_MAGIC && H.version == E.version && H.cur <= 1 && H.steps >= 0 && H.total == E.total &&
           H.payload == E.payload && H.nx == E.nx && H.ny == E.ny && H.nz == E.nz && H.physics == E.physics &&
           H.storage == E.storage && H.nspecies == E.nspecies && H.full_tensor == E.full_tensor &&
           H.solid_mask == E.solid_mask && H.uniform_eps == E.uniform_eps && H.uniform_kinv == E.uniform_kinv &&
           H.medium_tensor == E.medium_tensor && H.eps_u == E.eps_u && H.kinv_u[0] == E.kinv_u[0] &&
           H.kinv_u[1] == E.kinv_u[1] && H.kinv_u[2] == E.kinv_u[2];
}

// ---------------------------------------------------------------------------
// Lattices for callers that cannot allocate (lbm_create_static): the
// workspace is this file-scope array, one copy per GPU, placed on every
// device the library runs on when the code object is loaded and held until
// the process ends.  In host code `scratch` names a host-side stand-in: its
// device address on each device comes from hipGetSymbolAddress (taken once
// per device, with that device current) and only that address is used.
// One lattice at a time holds a device's array (with its handle in a static
// slot); the set-up of lbm_set_medium writes every byte of the layout that a
// step reads, so the contents left by an earlier lattice do not matter.
constexpr size_t SCRATCH_BYTES = size_t(64) << 20;
constexpr int MAX_DEVICES = 64;

__device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

std::mutex scratch_mu;
void *scratch_ptr[MAX_DEVICES];        // device address of scratch per device, once looked up
lbm_sim scratch_sim[MAX_DEVICES];      // the handle of the lattice holding it
bool scratch_held[MAX_DEVICES];

}  // namespace

extern "C" {

lbm_status lbm_create(const lbm_desc *d, void *dev_workspace, size_t ws_bytes, void *hip_stream, lbm_t *out)
{
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (!valid_desc(d) || !dev_workspace) return LBM_EINVAL;
    if (reinterpret_cast<uintptr_t>(dev_workspace) % ALIGN) return LBM_EINVAL;
    if (ws_bytes < layout(d).total) return LBM_ENOMEM;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return LBM_EDEVICE;
    lbm_sim *h = new (std::nothrow) lbm_sim;
    if (!h) return LBM_ENOMEM;
    memset(h, 0, sizeof(*h));
    setup_handle(h, d, dev_workspace, ws_bytes, hip_stream, device);
    *out = h;
    return LBM_OK;
}

lbm_status lbm_create_static(const lbm_desc *d, void *hip_stream, lbm_t *out)
{
    if (!out) return LBM_EINVAL;
    *out = nullptr;
    if (!valid_desc(d)) return LBM_EINVAL;
    if (layout(d).total > SCRATCH_BYTES) return LBM_ENOMEM;
    int device = 0;
    if (hipGetDevice(&device) != hipSuccess) return LBM_EDEVICE;
    if (device < 0 || device >= MAX_DEVICES) return LBM_EDEVICE;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (scratch_held[device]) return LBM_ESTATE;
    if (!scratch_ptr[device]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return LBM_EDEVICE;
        if (reinterpret_cast<uintptr_t>(p) % ALIGN) return LBM_EDEVICE;
        scratch_ptr[device] = p;
    }
    lbm_sim *h = &scratch_sim[device];
    memset(h, 0, sizeof(*h));
    setup_handle(h, d, scratch_ptr[device], SCRATCH_BYTES, hip_stream, device);
    h->in_scratch = 1;
    scratch_held[device] = true;
    *out = h;
    return LBM_OK;
}

lbm_status lbm_set_medium(lbm_t h, const lbm_medium *m)
{
    if (!h || !m) return LBM_EINVAL;
    // Host-side checks before the handle is touched: a rejected call leaves
    // a handle (ready or not) exactly as it was.
    if (!m->eps && !(m->eps_uniform > 0.0 && m->eps_uniform <= 1.0)) return LBM_EINVAL;
    if (!m->kinv)
        for (int a = 0; a < 3; ++a)
            if (!(m->kinv_uniform[a] >= 0.0) || !is_fin(m->kinv_uniform[a])) return LBM_EINVAL;
    if (m->solid && !h->d.solid_mask) return LBM_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return LBM_EDEVICE;
    // From here on the device state is rewritten: the handle is ready again
    // only when the whole set-up has succeeded.
    h->ready = 0;
    const size_t n = (size_t)h->host.ncell;
    const size_t rb = real_bytes(h->d.storage);
    LatDev &D = h->host;
    D.uniform_eps = m->eps ? 0 : 1;
    D.uniform_kinv = m->kinv ? 0 : 1;
    D.full_tensor = (h->d.full_tensor && m->kinv) ? 1 : 0;
    D.eps_u = m->eps_uniform;
    for (int a = 0; a < 3; ++a) D.kinv_u[a] = m->kinv_uniform[a];
    lbm_status st;
    if ((st = dev_err(hipMemcpyAsync(h->dev, &D, sizeof(LatDev), hipMemcpyHostToDevice, h->stream)))) return st;
    static const int zero = 0;
    if ((st = dev_err(hipMemcpyAsync(D.err, &zero, sizeof(int), hipMemcpyHostToDevice, h->stream)))) return st;
    if (D.ms &&
        (st = dev_err(hipMemcpyAsync(const_cast<void *>(D.ms), &h->ms, sizeof(MsDev), hipMemcpyHostToDevice, h->stream))))
        return st;
    if (D.fs) {
        static const double zero_mass = 0.0;
        if ((st = dev_err(hipMemcpyAsync(const_cast<void *>(D.fs), &h->fs, sizeof(FsDev), hipMemcpyHostToDevice,
                                         h->stream))))
            return st;
        if ((st = dev_err(hipMemcpyAsync(h->fs.lost, &zero_mass, sizeof(double), hipMemcpyHostToDevice, h->stream))))
            return st;
    }
    if (m->eps && (st = dev_err(hipMemcpyAsync(D.eps, m->eps, n * rb, hipMemcpyDeviceToDevice, h->stream)))) return st;
    if (m->kinv && !D.full_tensor &&
        (st = dev_err(hipMemcpyAsync(D.kinv, m->kinv, 3 * n * rb, hipMemcpyDeviceToDevice, h->stream))))
        return st;
    if (D.links) {
        uint32_t *links = static_cast<uint32_t *>(const_cast<void *>(D.links));
        hipLaunchKernelGGL(k_links, dim3(h->nblocks), dim3(BLOCK), 0, h->stream, (const LatDev *)h->dev, m->solid, links);
    }
    if (D.full_tensor) {
        if (h->d.storage == LBM_F64)
            hipLaunchKernelGGL(k_frame<double>, dim3(h->nblocks), dim3(BLOCK), 0, h->stream, (const LatDev *)h->dev,
                               static_cast<const double *>(m->kinv));
        else
            hipLaunchKernelGGL(k_frame<float>, dim3(h->nblocks), dim3(BLOCK), 0, h->stream, (const LatDev *)h->dev,
                               static_cast<const float *>(m->kinv));
    }
    switch (h->d.physics) {
    case LBM_SINGLE: init_for_storage<PH_SINGLE>(h, m, h->nblocks); break;
    case LBM_FREESURF: fs_init(h, m, h->nblocks); break;
    case LBM_MISCIBLE: init_for_storage<PH_MISCIBLE>(h, m, h->nblocks); break;
    default: init_for_storage<PH_IMMISCIBLE>(h, m, h->nblocks); break;
    }
    BatchArgs diag;
    memset(&diag, 0, sizeof(diag));
    diag.n = 1;
    diag.lat[0] = h->dev;
    hipLaunchKernelGGL(k_diag_final, dim3(1), dim3(BLOCK), 0, h->stream, diag);
    if ((st = dev_err(hipGetLastError()))) return st;
    int err = 0;
    if ((st = dev_err(hipMemcpyAsync(&err, D.err, sizeof(int), hipMemcpyDeviceToHost, h->stream)))) return st;
    if ((st = dev_err(hipStreamSynchronize(h->stream)))) return st;
    h->steps = 0;
    h->cur = 0;
    if (err) return LBM_EINVAL;
    h->ready = 1;
    return LBM_OK;
}

lbm_status lbm_step(lbm_t h, int nsteps)
{
    if (!h || nsteps < 0) return LBM_EINVAL;
    if (!h->ready) return LBM_ESTATE;
    if (hipSetDevice(h->device) != hipSuccess) return LBM_EDEVICE;
    for (int s = 0; s < nsteps; ++s) {
        const bool last = s + 1 == nsteps;
        lbm_sim *one[1] = {h};
        const lbm_status st = launch_batch_step(one, &last, 1);
        if (st) return st;
    }
    return LBM_OK;
}

lbm_status lbm_step_batch(lbm_t *hs, const int *nsteps, int n)
{
    if (!hs || !nsteps || n < 0) return LBM_EINVAL;
    int maxs = 0;
    for (int i = 0; i < n; ++i) {
        if (!hs[i] || nsteps[i] < 0) return LBM_EINVAL;
        if (!hs[i]->ready) return LBM_ESTATE;
        if (hs[i]->stream != hs[0]->stream || hs[i]->device != hs[0]->device) return LBM_EINVAL;
        for (int j = 0; j < i; ++j)
            if (hs[j] == hs[i]) return LBM_EINVAL;
        if (nsteps[i] > maxs) maxs = nsteps[i];
    }
    if (n == 0) return LBM_OK;
    if (hipSetDevice(hs[0]->device) != hipSuccess) return LBM_EDEVICE;
    lbm_sim *grp[MAXB];
    bool last[MAXB];
    for (int s = 0; s < maxs; ++s) {
        // group the lattices still running by (physics, storage, permeability
        // form, further solutes)
        for (int phys = LBM_SINGLE; phys <= LBM_FREESURF; ++phys)
            for (int grp_key = 0; grp_key < 4 * (LBM_F16_SPLIT + 1); ++grp_key) {
                const int stg = grp_key >> 2, ft = grp_key & 1, ms = (grp_key >> 1) & 1;
                int k = 0;
                for (int i = 0; i < n; ++i) {
                    lbm_sim *h = hs[i];
                    if (s >= nsteps[i] || h->d.physics != phys || h->d.storage != stg || h->host.full_tensor != ft)
                        continue;
                    if ((h->host.ms != nullptr) != (ms != 0)) continue;
                    grp[k] = h;
                    last[k] = s + 1 == nsteps[i];
                    if (++k == MAXB) {
                        const lbm_status st = launch_batch_step(grp, last, k);
                        if (st) return st;
                        k = 0;
                    }
                }
                if (k) {
                    const lbm_status st = launch_batch_step(grp, last, k);
                    if (st) return st;
                }
            }
    }
    return LBM_OK;
}

lbm_status lbm_moments(lbm_t h, void *rho, void *vel3, void *conc, double diag[8])
{
    if (!h) return LBM_EINVAL;
    if (!h->ready) return LBM_ESTATE;
    if (hipSetDevice(h->device) != hipSuccess) return LBM_EDEVICE;
    const size_t n = (size_t)h->host.ncell;
    const size_t rb = real_bytes(h->d.storage);
    const char *M = static_cast<const char *>(h->host.mom);
    lbm_status st;
    if (rho && (st = dev_err(hipMemcpyAsync(rho, M, n * rb, hipMemcpyDeviceToDevice, h->stream)))) return st;
    if (vel3 && (st = dev_err(hipMemcpyAsync(vel3, M + n * rb, 3 * n * rb, hipMemcpyDeviceToDevice, h->stream)))) return st;
    const size_t nconc = 1 + extra_species(&h->d);
    if (conc && (st = dev_err(hipMemcpyAsync(conc, M + 4 * n * rb, nconc * n * rb, hipMemcpyDeviceToDevice, h->stream))))
        return st;
    double dg[8];
    if ((st = dev_err(hipMemcpyAsync(dg, h->host.diag, sizeof(dg), hipMemcpyDeviceToHost, h->stream)))) return st;
    if ((st = dev_err(hipStreamSynchronize(h->stream)))) return st;
    if (diag) memcpy(diag, dg, sizeof(dg));
    return dg[7] != 0.0 ? LBM_EUNSTABLE : LBM_OK;
}

lbm_status lbm_populations(lbm_t h, int lattice, void *dst)
{
    if (!h || !dst || lattice < 0 || lattice > 1 + extra_species(&h->d)) return LBM_EINVAL;
    if (lattice == 1 && !two_lattices(h->d.physics)) return LBM_EINVAL;
    if (!h->ready) return LBM_ESTATE;
    if (hipSetDevice(h->device) != hipSuccess) return LBM_EDEVICE;
    const LatDev *L = h->dev;
    switch (h->d.storage) {
    case LBM_F64:
        hipLaunchKernelGGL(k_export<double>, dim3(h->nblocks), dim3(BLOCK), 0, h->stream, L, lattice, h->cur, static_cast<double *>(dst));
        break;
    case LBM_F32:
        hipLaunchKernelGGL(k_export<float>, dim3(h->nblocks), dim3(BLOCK), 0, h->stream, L, lattice, h->cur, static_cast<float *>(dst));
        break;
    case LBM_BF16_DEV:
        hipLaunchKernelGGL(k_export<bf16_t>, dim3(h->nblocks), dim3(BLOCK), 0, h->stream, L, lattice, h->cur, static_cast<float *>(dst));
        break;
    case LBM_F16_DEV:
        hipLaunchKernelGGL(k_export<f16_t>, dim3(h->nblocks), dim3(BLOCK), 0, h->stream, L, lattice, h->cur, static_cast<float *>(dst));
        break;
    case LBM_BF16_SPLIT:
        hipLaunchKernelGGL(k_export<bf16s_t>, dim3(h->nblocks), dim3(BLOCK), 0, h->stream, L, lattice, h->cur, static_cast<float *>(dst));
        break;
    default:
        hipLaunchKernelGGL(k_export<f16s_t>, dim3(h->nblocks), dim3(BLOCK), 0, h->stream, L, lattice, h->cur, static_cast<float *>(dst));
        break;
    }
    lbm_status st;
    if ((st = dev_err(hipGetLastError()))) return st;
    return dev_err(hipStreamSynchronize(h->stream));
}

lbm_status lbm_solute_totals(lbm_t h, double *totals)
{
    if (!h || !totals || h->d.physics != LBM_MISCIBLE) return LBM_EINVAL;
    if (!h->ready) return LBM_ESTATE;
    if (hipSetDevice(h->device) != hipSuccess) return LBM_EDEVICE;
    const int nsp = 1 + extra_species(&h->d);
    if (h->d.storage == LBM_F64)
        hipLaunchKernelGGL(k_solute_partials<double>, dim3(h->nblocks), dim3(BLOCK), 0, h->stream, (const LatDev *)h->dev, nsp);
    else
        hipLaunchKernelGGL(k_solute_partials<float>, dim3(h->nblocks), dim3(BLOCK), 0, h->stream, (const LatDev *)h->dev, nsp);
    hipLaunchKernelGGL(k_solute_final, dim3(1), dim3(BLOCK), 0, h->stream, (const LatDev *)h->dev, nsp);
    lbm_status st;
    if ((st = dev_err(hipGetLastError()))) return st;
    double out[LBM_MAX_SPECIES];
    if ((st = dev_err(hipMemcpyAsync(out, h->host.partials, nsp * sizeof(double), hipMemcpyDeviceToHost, h->stream))))
        return st;
    if ((st = dev_err(hipStreamSynchronize(h->stream)))) return st;
    memcpy(totals, out, nsp * sizeof(double));
    return LBM_OK;
}

lbm_status lbm_free_surface(lbm_t h, unsigned char *cls, double *mass, double *lambda, double *lost)
{
    if (!h || h->d.physics != LBM_FREESURF) return LBM_EINVAL;
    if (!h->ready) return LBM_ESTATE;
    if (hipSetDevice(h->device) != hipSuccess) return LBM_EDEVICE;
    const LatDev *L = h->dev;
    if (cls || mass || lambda) {
        const dim3 g(h->nblocks), b(BLOCK);
        const int c = h->cur;
        switch (h->d.storage) {
        case LBM_F64: hipLaunchKernelGGL(k_fs_export<double>, g, b, 0, h->stream, L, c, cls, mass, lambda); break;
        case LBM_F32: hipLaunchKernelGGL(k_fs_export<float>, g, b, 0, h->stream, L, c, cls, mass, lambda); break;
        case LBM_BF16_DEV: hipLaunchKernelGGL(k_fs_export<bf16_t>, g, b, 0, h->stream, L, c, cls, mass, lambda); break;
        case LBM_F16_DEV: hipLaunchKernelGGL(k_fs_export<f16_t>, g, b, 0, h->stream, L, c, cls, mass, lambda); break;
        case LBM_BF16_SPLIT: hipLaunchKernelGGL(k_fs_export<bf16s_t>, g, b, 0, h->stream, L, c, cls, mass, lambda); break;
        default: hipLaunchKernelGGL(k_fs_export<f16s_t>, g, b, 0, h->stream, L, c, cls, mass, lambda); break;
        }
    }
    lbm_status st;
    if ((st = dev_err(hipGetLastError()))) return st;
    double lo = 0.0;
    if ((st = dev_err(hipMemcpyAsync(&lo, h->fs.lost, sizeof(double), hipMemcpyDeviceToHost, h->stream)))) return st;
    if ((st = dev_err(hipStreamSynchronize(h->stream)))) return st;
    if (lost) *lost = lo;
    return LBM_OK;
}

lbm_status lbm_set_stream(lbm_t h, void *hip_stream)
{
    if (!h) return LBM_EINVAL;
    h->stream = static_cast<hipStream_t>(hip_stream);
    return LBM_OK;
}

long long lbm_steps_done(lbm_t h) { return h ? h->steps : -1; }

size_t lbm_state_bytes(lbm_t h)
{
    return h ? size_t(sizeof(CkptHeader) + ckpt_header(h).payload) : 0;
}

lbm_status lbm_save_state(lbm_t h, void *host_dst, size_t bytes)
{
    if (!h || !host_dst) return LBM_EINVAL;
    if (!h->ready) return LBM_ESTATE;
    const CkptHeader H = ckpt_header(h);
    if (bytes < sizeof(CkptHeader) + H.payload) return LBM_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return LBM_EDEVICE;
    memcpy(host_dst, &H, sizeof(H));
    char *o = static_cast<char *>(host_dst) + sizeof(H);
    Span sp[3];
    const int n = state_spans(h, sp);
    lbm_status st;
    for (int k = 0; k < n; ++k) {
        if ((st = dev_err(hipMemcpyAsync(o, h->ws + sp[k].off, sp[k].len, hipMemcpyDeviceToHost, h->stream)))) return st;
        o += sp[k].len;
    }
    return dev_err(hipStreamSynchronize(h->stream));
}

lbm_status lbm_load_state(lbm_t h, const void *host_src, size_t bytes)
{
    if (!h || !host_src) return LBM_EINVAL;
    if (!h->ready) return LBM_ESTATE;
    if (bytes < sizeof(CkptHeader)) return LBM_EINVAL;
    CkptHeader H;
    memcpy(&H, host_src, sizeof(H));
    if (!ckpt_fits(H, ckpt_header(h)) || bytes < sizeof(CkptHeader) + H.payload) return LBM_EINVAL;
    if (hipSetDevice(h->device) != hipSuccess) return LBM_EDEVICE;
    // the workspace is rewritten from here on: the handle is ready again only
    // when every copy has completed
    h->ready = 0;
    const char *o = static_cast<const char *>(host_src) + sizeof(H);
    Span sp[3];
    const int n = state_spans(h, sp);
    lbm_status st;
    for (int k = 0; k < n; ++k) {
        if ((st = dev_err(hipMemcpyAsync(h->ws + sp[k].off, o, sp[k].len, hipMemcpyHostToDevice, h->stream)))) return st;
        o += sp[k].len;
    }
    if ((st = dev_err(hipStreamSynchronize(h->stream)))) return st;
    h->steps = H.steps;
    h->cur = int(H.cur);
    h->ready = 1;
    return LBM_OK;
}

lbm_status lbm_destroy(lbm_t h)
{
    if (!h) return LBM_EINVAL;
    if (h->in_scratch) {
        // the array stays on the device; only the hold is released
        std::lock_guard<std::mutex> lock(scratch_mu);
        scratch_held[h->device] = false;
        h->in_scratch = 0;
        return LBM_OK;
    }
    delete h;
    return LBM_OK;
}

void lbm_lattice(int vel[57], double w[19])
{
    for (int q = 0; q < NQ; ++q) {
        if (vel) {
            vel[3 * q] = cx(q);
            vel[3 * q + 1] = cy(q);
            vel[3 * q + 2] = cz(q);
        }
        if (w) w[q] = weight<double>(q);
    }
}

const char *lbm_strerror(lbm_status s)
{
    switch (s) {
    case LBM_OK: return "ok";
    case LBM_EINVAL: return "invalid argument";
    case LBM_ENOMEM: return "workspace too small";
    case LBM_EDEVICE: return "HIP runtime or kernel launch failure";
    case LBM_EUNSTABLE: return "non-finite moments (unstable run)";
    case LBM_ESTATE: return "call out of order";
    }
    return "unknown status";
}

}  // extern "C"
