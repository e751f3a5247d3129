/*
 * lbm.h -- C ABI of the MI355X (gfx950) porous-media lattice Boltzmann library.
 *
 * The library advances the 3D lattice Boltzmann model of Mendoza, Wittel and
 * Herrmann, "Simulation of Flow of Mixtures Through Anisotropic Porous Media
 * using a Lattice Boltzmann Model" (arXiv:0912.4230) on one GPU:
 *   - a D3Q19 hydrodynamic lattice with BGK collision and forcing terms for
 *     the porous medium (Sec. 2.1, Eqs. lbe2, coeffforce1, forcement,
 *     expandV, expandVsub, equilc1, equilc2): porosity eps, an anisotropic
 *     permeability K (diagonal, or a full symmetric tensor), body force G,
 *     Darcy drag and (optionally) a
 *     Forchheimer drag, with a local viscosity nu(C, t) for hardening fluids
 *     (family of Eq. nuall);
 *   - a second D3Q19 lattice that is either the solute of a miscible mixture
 *     (Sec. 2.2, Eqs. equild, boltzeqD) or fluid 1 of a two-fluid
 *     (immiscible) mixture whose colour gradient (Eq. macros) drives the
 *     surface-tension term of Eqs. equilc1/2 (tensor of Eq. eqsurftens);
 *   - walls (halfway bounce-back, with a wall colour that sets the contact
 *     angle in two-fluid mode), fixed-state reservoirs (pressure inlet /
 *     outlet) and periodic faces (Sec. 4, boundary conditions), and optional
 *     obstacle cells anywhere in the box given by a per-cell mask;
 *   - or, instead of the second lattice, the free-surface technique of
 *     Sec. 3 (liquid penetrating empty space): liquid, interface and gas
 *     cells, the liquid mass of interface cells (Eqs. massmacro, massevol,
 *     deltamass), populations rebuilt on links from gas cells (Eq.
 *     equilempty) and the conversion of cells as they fill and empty.
 *
 * One time step follows the simulation procedure of Sec. 4 (flowchart):
 * stream both lattices, take the moments, form the colour gradient, collide.
 *
 * Memory: the library never allocates or frees device memory.  The caller
 * allocates one device workspace of lbm_workspace_bytes() bytes (for example
 * a torch uint8 tensor) and owns it; the handle keeps a pointer to it until
 * lbm_destroy().  All field pointers passed to the library are device
 * pointers unless stated otherwise.
 *
 * Layout of every field: structure of arrays, x fastest,
 * idx = x + nx * (y + ny * z); a vector field is 3 consecutive planes of
 * nx*ny*nz values (x, y, z components).  The real type of fields ("real")
 * is double when storage == LBM_F64 and float otherwise.
 *
 * Errors: every call returns an lbm_status; no call aborts or throws.
 * Argument checks happen before any GPU call.  Kernel faults are reported by
 * the next call that synchronises (lbm_set_medium, lbm_moments).
 *
 * Threading: a handle is used by one host thread at a time.  All work of a
 * handle is issued on the HIP stream given to lbm_create (NULL = default).
 */
#ifndef PORO_LBM_H
#define PORO_LBM_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    LBM_OK = 0,
    LBM_EINVAL = 1,     /* an argument is out of range or inconsistent */
    LBM_ENOMEM = 2,     /* the workspace is too small */
    LBM_EDEVICE = 3,    /* a HIP runtime call or a kernel launch failed */
    LBM_EUNSTABLE = 4,  /* the diagnostics found a non-finite moment */
    LBM_ESTATE = 5      /* call out of order (e.g. lbm_step before lbm_set_medium) */
} lbm_status;

typedef enum {
    LBM_SINGLE = 0,      /* hydrodynamic lattice only */
    LBM_MISCIBLE = 1,    /* + solute lattice (Sec. 2.2) */
    LBM_IMMISCIBLE = 2,  /* + fluid-1 lattice of a two-fluid colour model */
    LBM_FREESURF = 3     /* hydrodynamic lattice + free surface (Sec. 3) */
} lbm_physics;
/* Free surface (LBM_FREESURF).  Every non-solid cell is liquid, interface
 * or gas.  Gas cells carry no state.  Liquid and interface cells stream and
 * collide like the single-fluid model (porous medium, force and viscosity
 * law included).  Each step:
 *  1. an interface cell x exchanges liquid mass with every liquid or
 *     interface neighbour y = x + v_i: dm_i = w (f~_opp(i)(y) - f~_i(x)),
 *     with w = 1 for a liquid y and (lambda(x) + lambda(y)) / 2 for an
 *     interface y (Eq. deltamass; weight 1 on liquid links is what conserves
 *     mass);
 *  2. a population that would stream in from a gas cell is
 *     f_i = f^eq_i + f^eq_opp(i) - f~_opp(i)(x), the equilibria taken at the
 *     gas density 1 and the velocity of x's own post-collision populations
 *     (Eq. equilempty);
 *  3. after the collision, an interface cell with m > (1 + 1e-3) rho fills
 *     (becomes liquid) and one with m < -1e-3 rho empties (becomes gas),
 *     unless it touches a filling cell; gas cells next to a filling cell
 *     become interface cells with the equilibrium of the mean density and
 *     velocity (rho and V' of the step) of their liquid and interface
 *     neighbours that do not empty, and m = 0; liquid cells
 *     next to an emptying cell become interface cells with m = rho;
 *  4. the excess m - rho of a filled cell, or m of an emptied one, is shared
 *     equally among its neighbours that are interface cells after the step
 *     and did not convert (if there is none, it is lost and counted).
 * Then lambda = m / rho (1 for liquid, 0 for gas).  lbm_medium.c0 holds the
 * initial fill fraction: >= 1 liquid, <= 0 gas, else an interface cell with
 * m = c0 rho0; a liquid cell next to a gas cell starts as an interface cell
 * with m = rho0.  With A > 0 the surface-tension term of Eqs. equilc1/2 acts
 * (Sec. 5.4) with the gradient of Eq. macros taken over the fill fraction,
 * F = Sum_i lambda(x + v_i) v_i (a solid neighbour counts lambda(x)).
 * Reservoir faces are rejected.  lbm_moments reports lambda
 * as the concentration; rho and V' of gas cells read 0; the diagnostics run
 * over liquid and interface cells, with diag[4] = the total liquid mass
 * (Sum of m over interface cells + Sum of rho over liquid cells).  The
 * conversion decisions are taken in double precision on masses kept in
 * double precision in every storage mode. */

#define LBM_MAX_SPECIES 4

typedef enum {
    LBM_F64 = 0,         /* populations and fields in double */
    LBM_F32 = 1,         /* populations and fields in float */
    LBM_BF16_DEV = 2,    /* populations stored in bfloat16, compute in float */
    LBM_F16_DEV = 3,     /* populations stored in IEEE half, compute in float */
    LBM_BF16_SPLIT = 4,  /* per-cell FP32 mass + bfloat16 remainders, compute in float */
    LBM_F16_SPLIT = 5    /* per-cell FP32 mass + IEEE half remainders, compute in float */
} lbm_storage;
/* The hydrodynamic populations are stored as deviations f_i - w_i from the
 * rest-state weights in every storage mode (in reduced precision this is
 * what makes 16-bit storage usable); the second lattice is stored as is.
 * The split modes store, per lattice and cell, m = sum_i of the stored
 * values in FP32 and the remainders (value_i - w_i m) in 16 bits: the
 * density (or solute mass) part of every population is then exact to FP32
 * and only the velocity / non-equilibrium part is rounded to 16 bits
 * (4 more bytes per cell and lattice, read and written).  Rounding to 16 bits
 * is round-to-nearest-even. */

typedef enum {
    LBM_FACE_PERIODIC = 0,   /* both faces of an axis must be periodic together */
    LBM_FACE_WALL = 1,       /* the boundary plane of cells is solid */
    LBM_FACE_RESERVOIR = 2   /* the boundary plane holds a fixed equilibrium state */
} lbm_face_kind;

typedef struct {
    int kind;                   /* lbm_face_kind */
    double rho;                 /* RESERVOIR: density (pressure p = rho / 3 / eps) */
    double conc;                /* RESERVOIR: concentration C of the reservoir */
    double contact_angle_deg;   /* WALL, two-fluid mode: contact angle of fluid 1 */
} lbm_face;

typedef struct {
    int nx, ny, nz;             /* cells per axis, each >= 1 (>= 3 on a non-periodic axis) */
    int physics;                /* lbm_physics */
    int storage;                /* lbm_storage */
    int forchheimer;            /* 1: Forchheimer drag -eps F_eps |V'| K^-1/2 V',
                                   F_eps = 1.75 / sqrt(150 eps^3) */
    int eps_gradient;           /* 1: solute drift V* = V' + D grad(eps)/eps (Eq. equild) */
    double G[3];                /* body force (acceleration), lattice units */
    /* viscosity (single / miscible): nu = nu0 * min(a0 + a1 e^{alpha t}, cap)
       * e^{k1 C + k0}, t = index of the step being computed; tau = 1/2 + 3 nu.
       The paper's Eq. nuall is (nu_g, 1, a, alpha, inf, -beta, beta). */
    double nu0, a0, a1, alpha, cap, k1, k0;
    double tau1, tau2;          /* two-fluid: relaxation times of fluid 1 and 2;
                                   nu = C nu_1 + (1 - C) nu_2 with C = rho_1 / rho */
    double tau_d;               /* miscible: solute relaxation time, D = (tau_d - 1/2)/3 */
    double A;                   /* two-fluid or free surface: surface-tension strength
                                   (Eq. equilc1); must be 0 in the other modes */
    double beta;                /* two-fluid: recolouring strength in [0, 1] */
    lbm_face face[6];           /* order: -x, +x, -y, +y, -z, +z */
    int diag_every;             /* FP64 diagnostics every k steps (0: only at the end
                                   of each lbm_step call) */
    int solid_mask;             /* 1: lbm_set_medium takes a per-cell obstacle mask
                                   (lbm_medium.solid); the workspace then holds one
                                   32-bit link word per cell */
    double solid_contact_angle_deg;  /* two-fluid: contact angle of fluid 1 on the
                                   obstacle cells of the mask */
    int full_tensor;            /* 1: lbm_medium.kinv holds a full symmetric K^-1 per cell
                                   (the rotated tensor of Eq. Ktensor), 6 planes
                                   {xx, yy, zz, xy, xz, yz}; 0: the diagonal, 3 planes */
    int nspecies;               /* miscible: number of solutes, 1 to LBM_MAX_SPECIES
                                   (0 means 1); each further solute has its own lattice */
    double tau_d_x[LBM_MAX_SPECIES - 1];       /* relaxation times of solutes 2.. */
    double face_conc_x[LBM_MAX_SPECIES - 1][6]; /* RESERVOIR faces: concentrations of
                                   solutes 2.., in the face order of face[] */
} lbm_desc;
/* Several solutes (the extension to "various species" that Sec. 2.2 prepares):
 * solute k has its own D3Q19 lattice, relaxation time (D_k = (tau_d,k - 1/2)/3)
 * and reservoir concentrations, and follows Eqs. equild and boltzeqD with the
 * shared corrected velocity V' and its own drift D_k grad(eps)/eps.  The
 * viscosity law reads the first solute's concentration.  lbm_medium.c0 then
 * holds nspecies planes (solute-major), lbm_moments writes nspecies
 * concentration planes, lbm_populations takes lattice 1..nspecies for the
 * solutes, and lbm_solute_totals reduces every solute's mass. */

/* Medium and initial fields (flowchart of Sec. 4: set rho, V, C, the
 * porosity and the permeability).  Device pointers of the real type; NULL
 * selects the uniform value.  The library copies them into the workspace on
 * the handle's stream; the caller may reuse the buffers once that stream has
 * passed the call (lbm_set_medium synchronises before returning). */
typedef struct {
    const void *eps;            /* ncell values in (0, 1]; NULL: eps_uniform */
    const void *kinv;           /* 3 planes: 1/K_xx, 1/K_yy, 1/K_zz >= 0 (full_tensor: 6 planes
                                   {xx, yy, zz, xy, xz, yz} of a positive semi-definite
                                   K^-1); NULL: kinv_uniform (diagonal) */
    const void *rho0;           /* ncell initial densities > 0; NULL: 1 */
    const void *vel0;           /* 3 planes, initial velocity V' ; NULL: 0 */
    const void *c0;             /* ncell initial concentrations (free surface: initial
                                   fill fractions); NULL: 0 */
    double eps_uniform;
    double kinv_uniform[3];
    const unsigned char *solid; /* ncell bytes, nonzero = obstacle cell; only with
                                   desc.solid_mask = 1 (NULL there: no obstacles) */
} lbm_medium;
/* A full tensor enters Eqs. forcement and expandV as the matrix K^-1 and the
 * Forchheimer drag as its positive square root K^-1/2 (they share the
 * eigenframe of K); lbm_set_medium stores each cell's eigenframe (a unit
 * quaternion) and eigenvalues, 7 planes in the workspace.
 *
 * Obstacle cells of the mask are solid exactly like the cells of a wall face
 * (Sec. 4: bounce-back on every link into them, no state, moments read 0);
 * a cell on a wall face is a wall cell, else a masked cell is an obstacle,
 * else a cell on a reservoir face belongs to the reservoir.  Their porosity
 * and permeability values are ignored; in the porosity gradient a solid
 * neighbour takes the porosity of the cell itself.  The link word of a cell
 * holds bit 0 = the cell is solid and bit q = the cell x - v_q is solid (q in
 * the order of lbm_lattice), built once by lbm_set_medium. */

typedef struct lbm_sim *lbm_t;

/* Bytes of device workspace a lattice of this description needs; 0 if the
 * description is invalid. */
size_t lbm_workspace_bytes(const lbm_desc *d);

/* Validate d, lay the lattice out in dev_workspace (>= lbm_workspace_bytes(d)
 * bytes, 256-byte aligned, owned by the caller) and return a host handle.
 * hip_stream is a hipStream_t (NULL: default stream).  No GPU call is made
 * when the arguments are rejected. */
lbm_status lbm_create(const lbm_desc *d, void *dev_workspace, size_t ws_bytes,
                      void *hip_stream, lbm_t *out);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): lbm_create
 * without a workspace argument.  The lattice lives in a static workspace
 * that the library holds on every GPU it runs on (64 MiB per device, in its
 * code object, kept until the process ends), so neither this call nor any
 * later call on the handle allocates anything, on the device or the host.
 * One such lattice per device at a time: LBM_ESTATE while another handle of
 * this call on the current device is alive (lbm_destroy releases it);
 * LBM_ENOMEM if the lattice needs more than 64 MiB (lbm_workspace_bytes);
 * LBM_EINVAL for an invalid description.  Results are bitwise those of
 * lbm_create with a caller workspace.  Every other call takes the handle as
 * usual (lbm_step_batch may mix it with lattices in caller workspaces). */
lbm_status lbm_create_static(const lbm_desc *d, void *hip_stream, lbm_t *out);

/* Copy the medium and the initial fields in and set the populations to their
 * equilibria (Eqs. equilc1/2, equild; two-fluid: g = C f).  Validates the
 * fields of every non-solid cell on the device (eps in (0,1], K^-1 >= 0,
 * rho0 > 0, all finite) and returns LBM_EINVAL if a value is out of range,
 * or if m->solid is set on a handle created without solid_mask.  Resets the
 * step count.  Synchronises the handle's stream.  The uniform values and the
 * mask flag are checked on the host first: such a rejection leaves the
 * handle untouched (a ready handle stays ready with its medium).  A
 * rejection by the device checks, or a device error, leaves the handle not
 * ready (lbm_step returns LBM_ESTATE) until a later call succeeds. */
lbm_status lbm_set_medium(lbm_t h, const lbm_medium *m);

/* Advance nsteps >= 0 time steps, asynchronously on the handle's stream. */
lbm_status lbm_step(lbm_t h, int nsteps);

/* Advance n lattices by nsteps[i] steps each, with one launch sequence per
 * step for all lattices of the same physics, storage, permeability form
 * (diagonal or full tensor) and solute count form (one, or more) (continuous
 * batching; up to 64 lattices per launch).  All handles must share one
 * stream.  Per-lattice results are bitwise identical to lbm_step on the same
 * handle. */
lbm_status lbm_step_batch(lbm_t *hs, const int *nsteps, int n);

/* Copy the moments of the last step (density rho, corrected velocity V' as
 * 3 planes, concentration C; after 0 steps: the initial fields) into caller
 * device buffers of the real type (each may be NULL), and the FP64
 * diagnostics of the last diagnostic step into the host array diag (may be
 * NULL): {Sum rho, Sum rho V'_x, Sum rho V'_y, Sum rho V'_z, Sum eps C
 * (miscible) or Sum rho_1 (two-fluid) or 0, |V' - V'_prev|^2 / |V'|^2
 * relative to the previous diagnostic, max |V'|, count of non-finite cells},
 * all over fluid cells.  Solid cells read 0; reservoir cells read their fixed
 * state.  Synchronises the stream; returns LBM_EUNSTABLE when the count of
 * non-finite cells is not zero. */
lbm_status lbm_moments(lbm_t h, void *rho, void *vel3, void *conc, double diag[8]);

/* Current post-collision populations of lattice 0 (hydrodynamic, as
 * deviations f_i - w_i) or 1 (second lattice, as is; with several solutes
 * 1..nspecies are the solutes), decoded to the real type: 19 planes in the
 * direction order of lbm_lattice().  Free surface: the values of gas cells
 * are left over from earlier steps and carry no meaning. */
lbm_status lbm_populations(lbm_t h, int lattice, void *dst);

/* Miscible mode: the mass of every solute over the fluid cells of the last
 * step, Sum eps C_k (Eq. diffusionporous), in FP64 with a fixed summation
 * order, into the host array totals[nspecies].  LBM_EINVAL for another
 * physics.  Synchronises the stream. */
lbm_status lbm_solute_totals(lbm_t h, double *totals);

/* Free surface (Sec. 3): the cell classes after the last step (ncell bytes:
 * 0 gas, 1 interface, 2 liquid, 3 solid), the liquid mass per cell (ncell
 * doubles: m for interface cells, rho for liquid cells, 0 for gas and
 * solid) and the fill fraction per cell (ncell doubles: lambda = m / rho of
 * interface cells as the last step stored it, 1 for liquid cells, 0 for gas
 * and solid), into caller device buffers (each may be NULL), and into *lost
 * (host, may be NULL) the excess mass that found no interface cell to take
 * it since lbm_set_medium.  LBM_EINVAL for a handle of another physics.
 * Synchronises the stream. */
lbm_status lbm_free_surface(lbm_t h, unsigned char *cls, double *mass, double *lambda, double *lost);

/* Issue the handle's later calls on hip_stream (a hipStream_t, NULL: the
 * default stream) instead of the stream given to lbm_create.  No GPU call:
 * the library does not order the new stream after work already issued on
 * the old one, the caller does (an event, or a synchronisation).  Serving
 * uses it to set lattices up and read them back on a second stream while the
 * batched steps of the others run on the first (lbm_step_batch takes handles
 * of one stream).  LBM_EINVAL for a NULL handle. */
lbm_status lbm_set_stream(lbm_t h, void *hip_stream);

/* Completed steps since lbm_set_medium, or -1 for a NULL handle. */
long long lbm_steps_done(lbm_t h);

/* Checkpoint and resume (the paper runs a simulation to a steady state in one
 * go, Sec. 4; a server that pre-empts lattices, or a long run that outlives
 * its process, saves and restores them).  A checkpoint is opaque host bytes:
 * a header, then every byte of the lattice's workspace (populations of both
 * copies, masses, medium planes, diagnostics, free-surface state, further
 * solutes) except the blocks that hold device addresses.
 *
 * lbm_state_bytes: the size of a checkpoint of h (about its workspace size),
 * or 0 for a NULL handle.
 * lbm_save_state: writes the checkpoint of h's state after the work issued on
 * its stream into host_dst (host memory of at least `bytes` >=
 * lbm_state_bytes(h) bytes, the caller's).  Synchronises the stream.
 * LBM_ESTATE before lbm_set_medium, LBM_EINVAL for NULL pointers or a short
 * buffer.
 * lbm_load_state: replaces h's state by the checkpoint in host_src and sets
 * its completed steps to the saved count; h must have been created from the
 * same description (sizes, physics, storage, solutes, tensor and mask flags)
 * and given a medium of the same form (uniform eps and K^-1 with the same
 * values, or per-cell fields) by lbm_set_medium; its other parameters (tau,
 * G, ...) and its workspace address may differ, and the next steps use them;
 * with the same parameters they are bitwise the steps the saved lattice would
 * have taken.
 * Synchronises the stream.  LBM_ESTATE before lbm_set_medium; LBM_EINVAL for
 * a checkpoint that does not fit h (nothing is written then); on a device
 * error during the copy (LBM_EDEVICE) the state is partly written and h
 * needs lbm_set_medium again (LBM_ESTATE until then). */
size_t lbm_state_bytes(lbm_t h);
lbm_status lbm_save_state(lbm_t h, void *host_dst, size_t bytes);
lbm_status lbm_load_state(lbm_t h, const void *host_src, size_t bytes);

/* Free the host handle (the workspace stays the caller's). */
lbm_status lbm_destroy(lbm_t h);

/* The library's D3Q19 direction order: vel[3*q + a], weights w[q]. */
void lbm_lattice(int vel[57], double w[19]);

/* Static text for a status code. */
const char *lbm_strerror(lbm_status s);

#ifdef __cplusplus
}
#endif

#endif /* PORO_LBM_H */
