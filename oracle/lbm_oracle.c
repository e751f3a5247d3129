/*
 * lbm_oracle.c -- plain FP64 CPU oracle for the porous-media lattice
 * Boltzmann update of Mendoza, Wittel & Herrmann, "Simulation of Flow of
 * Mixtures Through Anisotropic Porous Media using a Lattice Boltzmann Model"
 * (arXiv:0912.4230).
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, obviously-correct
 * reference that the GPU library is checked against.  Only the test suite,
 * the smoke check and the CPU-baseline leg of the benchmark load it; the
 * product path never does.  It shares no code, header or table with the GPU
 * library.
 *
 * Everything is double precision, plain loops over cells and directions,
 * compiled with -ffp-contract=off.  OpenMP splits the outer (z, y) loops only.
 *
 * Method, in the paper's order (simulation procedure of the flowchart in
 * Sec. 4):
 *   init : f = f^eq, h = h^eq from the initial fields   (Eqs. equilc1/2, equild)
 *   loop : t <- t+1
 *          stream f and h to the neighbours              (Eqs. lbe2, boltzeqD)
 *          moments rho, rho V, C                         (Eqs. macros1, macros)
 *          colour gradient F                             (Eq. macros)
 *          collide f with BGK + forcing, h with BGK      (Eqs. lbe2, coeffforce1,
 *                                                         forcement, expandV,
 *                                                         expandVsub, boltzeqD)
 *
 * Readings of points the paper leaves open (each is listed with its reason
 * in the design notes of the repository):
 *  - density sums all 19 populations, the rest one included (Eq. macros1
 *    prints the sum over the 18 moving ones; Sum f^eq = rho needs f_0);
 *  - the forcing term carries the factor w_i rho (Guo forcing, cited by the
 *    paper for Eq. coeffforce1; without it Sum_i T_i != 0);
 *  - V' = Lambda^{-1} (V + eps G / 2): Eqs. forcement and expandV combined,
 *    the printed Eq. expandVsub drops the porosity on G;
 *  - collision sign: f~ = f - (f - f^eq)/tau + T  (BGK of Sec. 2.1);
 *  - optional Forchheimer drag -eps F_eps |V'| K^{-1/2} V' in F^ext with
 *    F_eps = 1.75 / sqrt(150 eps^3) (Ergun constant n = 150 of Eq. KvsDp);
 *  - local viscosity nu(C,t) = nu0 min(a0 + a1 e^{alpha t}, cap) e^{k1 C + k0}
 *    (the family of Eq. nuall) sets the local tau = 1/2 + 3 nu;
 *  - solute concentration C = Sum_i h_i / eps (Eq. equild: Sum h^eq = eps C);
 *  - grad(eps) by the isotropic stencil 3 Sum_i w_i eps(x + v_i) v_i;
 *  - two-fluid (immiscible) mode: second lattice g = fluid-1 populations,
 *    colour field rho_1 = Sum g, C = rho_1 / rho, nu = C nu_1 + (1-C) nu_2,
 *    recolouring g~_i = C f~_i + beta C (1-C) rho w_i cos(v_i, F);
 *  - several solutes (miscible mode): each its own lattice, tau_d and
 *    reservoir concentrations, all advected by V'; the viscosity law reads
 *    the first solute's concentration;
 *  - free-surface mode (Sec. 3): liquid, interface and gas cells, mass
 *    exchange, reconstruction from gas cells and class conversion, with the
 *    readings stated beside fs_step below; with surface tension (Sec. 5.4)
 *    the gradient of Eq. macros is taken over the fill fraction lambda;
 *  - walls: halfway bounce-back; reservoirs: cells held at the equilibrium
 *    of (rho_bc, V' = 0, C_bc); the cells of an optional obstacle mask are
 *    solid like wall cells, with their own contact angle.
 *  - populations of the hydrodynamic lattice are held as deviations
 *    d_i = f_i - w_i (an exact change of variable) so that the round-off of
 *    the moments scales with the deviations and not with 1.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define NQ 19

enum { PHYS_SINGLE = 0, PHYS_MISCIBLE = 1, PHYS_IMMISCIBLE = 2, PHYS_FREESURF = 3 };
/* free-surface cell classes (Sec. 3) */
enum { FS_GAS = 0, FS_IF = 1, FS_LIQ = 2 };
enum { FACE_PERIODIC = 0, FACE_WALL = 1, FACE_RESERVOIR = 2 };
enum { CELL_FLUID = 0, CELL_SOLID = 1, CELL_RESERVOIR = 2 };

/* ------------------------------------------------------------------------ */
/* D3Q19 in the paper's enumeration (Sec. 2.1, Fig. d3q19): vectors v_i^p with
 * plane p = 0,1,2 and orientation i = 1..6, plus the rest vector.  Plane p is
 * spanned by the axes a = p and b = (p+1) mod 3; i = 1..4 are the four face
 * diagonals of that plane, i = 5,6 the two axis vectors +-e_a.  Weights:
 * w_0 = 1/3, w_{1..4} = 1/36, w_{5,6} = 1/18 (Sec. 2.1, after Eq. equilc2).
 * Flat index: q = 0 for rest, q = 1 + 6 p + (i - 1).                        */
static int    VEL[NQ][3];
static double WGT[NQ];
static int    OPP[NQ];
static int    lattice_ready = 0;

static void lattice_setup(void)
{
    if (lattice_ready) return;
    static const int sa[4] = {1, -1, 1, -1};
    static const int sb[4] = {1, -1, -1, 1};
    memset(VEL, 0, sizeof(VEL));
    WGT[0] = 1.0 / 3.0;
    for (int p = 0; p < 3; ++p) {
        int a = p, b = (p + 1) % 3;
        int q0 = 1 + 6 * p;
        for (int i = 0; i < 4; ++i) {
            VEL[q0 + i][a] = sa[i];
            VEL[q0 + i][b] = sb[i];
            WGT[q0 + i] = 1.0 / 36.0;
        }
        VEL[q0 + 4][a] = 1;
        VEL[q0 + 5][a] = -1;
        WGT[q0 + 4] = 1.0 / 18.0;
        WGT[q0 + 5] = 1.0 / 18.0;
    }
    for (int q = 0; q < NQ; ++q)
        for (int r = 0; r < NQ; ++r)
            if (VEL[r][0] == -VEL[q][0] && VEL[r][1] == -VEL[q][1] && VEL[r][2] == -VEL[q][2])
                OPP[q] = r;
    lattice_ready = 1;
}

/* ------------------------------------------------------------------------ */
typedef struct {
    int nx, ny, nz;
    int physics;        /* PHYS_* */
    int forchheimer;    /* 1: add the Forchheimer drag to F^ext */
    int eps_grad;       /* 1: V* = V' + D grad(eps)/eps (Eq. equild); 0: V* = V' */
    double G[3];        /* body force (acceleration) */
    double nu0, a0, a1, alpha, cap, k1, k0;   /* viscosity law (single, miscible) */
    double tau1, tau2;  /* immiscible: relaxation times of fluid 1 and fluid 2 */
    double tau_d;       /* solute relaxation time, D = (tau_d - 1/2)/3 */
    double A, beta;     /* surface-tension strength, recolouring strength */
    int face_kind[6];   /* -x,+x,-y,+y,-z,+z : FACE_* */
    double face_rho[6], face_conc[6], face_angle[6];  /* reservoir rho, C; wall angle (deg) */
    double solid_angle; /* contact angle (deg) of the obstacle cells of a solid mask */
    int full_tensor;    /* 1: K^-1 is a full symmetric tensor, 6 planes {xx,yy,zz,xy,xz,yz} */
    int nspecies;       /* miscible: number of solutes (0 or 1: one; at most ORC_MAXSP) */
    double tau_dx[3];   /* relaxation times of solutes 2.. */
    double face_concx[3][6];  /* reservoir concentrations of solutes 2.. */
} orc_params;
#define ORC_MAXSP 4

typedef struct {
    orc_params p;
    long n;                   /* number of cells */
    double *eps, *kinv;       /* porosity; inverse permeability: diagonal (3 planes) or
                                 full symmetric tensor (6 planes {xx,yy,zz,xy,xz,yz}) */
    double *ksqrt;            /* full tensor only: K^-1/2, 6 planes like kinv */
    unsigned char *type, *tface;
    double *f[2], *h[2];      /* [q*n + idx]; f as deviations f - w, h absolute */
    int cur;                  /* f[cur], h[cur] hold the current post-collision state */
    double *rho, *vel, *conc; /* moments of the last step (pre-collision, Sec. 4) */
    double *vsnap;            /* V' at the previous diagnostic call */
    double *rho1;             /* colour field (immiscible) */
    unsigned char *fst;       /* free surface: FS_GAS / FS_IF / FS_LIQ per non-solid cell */
    double *mass, *lam;       /* free surface: liquid mass m and fill fraction lambda = m / rho */
    double fs_lost;           /* free surface: excess mass without an interface neighbour */
    int nsx;                  /* miscible: number of solutes beyond the first */
    double *hx[2];            /* their populations, [k][q][idx], copies like h */
    double *concx;            /* their concentrations of the last step, [k][idx] */
    long step;                /* number of completed steps */
} orc_state;

static long cidx(const orc_state *s, int x, int y, int z)
{
    return (long)x + (long)s->p.nx * ((long)y + (long)s->p.ny * (long)z);
}

/* neighbour of (x,y,z) shifted by (dx,dy,dz): periodic faces wrap, any other
 * step out of the box returns -1 (treated as solid by the streaming). */
static long neighbour(const orc_state *s, int x, int y, int z, int dx, int dy, int dz)
{
    int c[3] = {x + dx, y + dy, z + dz};
    int n[3] = {s->p.nx, s->p.ny, s->p.nz};
    for (int a = 0; a < 3; ++a) {
        if (c[a] < 0 || c[a] >= n[a]) {
            if (s->p.face_kind[2 * a] != FACE_PERIODIC) return -1;
            c[a] = (c[a] + n[a]) % n[a];
        }
    }
    return cidx(s, c[0], c[1], c[2]);
}

/* Cell classes: a cell on a wall face is solid; otherwise a cell marked in
 * the optional obstacle mask is solid (its wall index is 6); otherwise a
 * cell on a reservoir face belongs to that reservoir; all others are fluid. */
static void classify(orc_state *s, const unsigned char *solid)
{
    int n[3] = {s->p.nx, s->p.ny, s->p.nz};
    for (int z = 0; z < n[2]; ++z)
        for (int y = 0; y < n[1]; ++y)
            for (int x = 0; x < n[0]; ++x) {
                int c[3] = {x, y, z};
                long i = cidx(s, x, y, z);
                unsigned char t = CELL_FLUID, tf = 255;
                for (int f = 0; f < 6 && t == CELL_FLUID; ++f) {
                    int a = f / 2, pos = (f % 2) ? n[a] - 1 : 0;
                    if (s->p.face_kind[f] == FACE_WALL && c[a] == pos) { t = CELL_SOLID; tf = (unsigned char)f; }
                }
                if (t == CELL_FLUID && solid && solid[i]) { t = CELL_SOLID; tf = 6; }
                for (int f = 0; f < 6 && t == CELL_FLUID; ++f) {
                    int a = f / 2, pos = (f % 2) ? n[a] - 1 : 0;
                    if (s->p.face_kind[f] == FACE_RESERVOIR && c[a] == pos) { t = CELL_RESERVOIR; tf = (unsigned char)f; }
                }
                s->type[i] = t;
                s->tface[i] = tf;
            }
}

/* wall colour C_w = (1 + cos theta)/2 of wall face f, or of the obstacle
 * cells for f = 6 (reference density 1). */
static double wall_colour(const orc_state *s, int f)
{
    const double pi = 3.14159265358979323846;
    const double th = f == 6 ? s->p.solid_angle : s->p.face_angle[f];
    return 0.5 * (1.0 + cos(th * pi / 180.0));
}

/* ------------------------------------------------------------------------ */
/* Local viscosity and relaxation time.  Single / miscible: the family of
 * Eq. nuall, nu = nu0 min(a0 + a1 e^{alpha t}, cap) e^{k1 C + k0}.  Two-fluid:
 * nu = C nu_1 + (1 - C) nu_2 with nu_k = (tau_k - 1/2)/3.  tau = 1/2 + 3 nu
 * (nu_e = (tau - 1/2)/3, Sec. 2).                                           */
static double viscosity(const orc_params *p, double C, double t)
{
    if (p->physics == PHYS_IMMISCIBLE) {
        double nu1 = (p->tau1 - 0.5) / 3.0, nu2 = (p->tau2 - 0.5) / 3.0;
        return C * nu1 + (1.0 - C) * nu2;
    }
    double tf = p->a0 + p->a1 * exp(p->alpha * t);
    if (tf > p->cap) tf = p->cap;
    double cc = (p->physics == PHYS_MISCIBLE) ? C : 0.0;
    return p->nu0 * tf * exp(p->k1 * cc + p->k0);
}

/* |V'| from s = | W / (lambda + mu s) | (componentwise), the implicit form of
 * Eqs. expandV + forcement with the Forchheimer term.  Safeguarded Newton on
 * phi(s) = s - R(s), R(s) = sqrt(sum_a W_a^2 / (lambda_a + mu_a s)^2); phi is
 * increasing, phi(0) < 0 <= phi(R(0)), so the root is unique in [0, R(0)].  */
double orc_solve_speed(const double W[3], const double lam[3], const double mu[3])
{
    double hi = 0.0;
    for (int a = 0; a < 3; ++a) hi += (W[a] / lam[a]) * (W[a] / lam[a]);
    hi = sqrt(hi);
    if (hi == 0.0 || (mu[0] == 0.0 && mu[1] == 0.0 && mu[2] == 0.0)) return hi;
    double lo = 0.0, s = hi;
    for (int it = 0; it < 200; ++it) {
        double R2 = 0.0, dR = 0.0;
        for (int a = 0; a < 3; ++a) {
            double d = lam[a] + mu[a] * s;
            R2 += W[a] * W[a] / (d * d);
            dR += W[a] * W[a] * mu[a] / (d * d * d);
        }
        double R = sqrt(R2);
        double phi = s - R;
        if (phi > 0.0) hi = s; else lo = s;
        double dphi = 1.0 + (R > 0.0 ? dR / R : 0.0);
        double sn = s - phi / dphi;
        if (!(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
        if (fabs(sn - s) <= 1e-16 * s || hi - lo <= 1e-16 * hi) { s = sn; break; }
        s = sn;
    }
    return s;
}

/* Corrected velocity V' and total external force F^ext (Eqs. forcement,
 * expandV, expandVsub; diagonal K; optional Forchheimer).                  */
static void porous_velocity(const orc_params *p, double eps, const double kinv[3], double nu,
                            const double V[3], double Vp[3], double Fext[3])
{
    double W[3], lam[3], mu[3];
    double Feps = p->forchheimer ? 1.75 / sqrt(150.0 * eps * eps * eps) : 0.0;
    for (int a = 0; a < 3; ++a) {
        W[a] = V[a] + 0.5 * eps * p->G[a];
        lam[a] = 1.0 + 0.5 * eps * nu * kinv[a];
        mu[a] = 0.5 * eps * Feps * sqrt(kinv[a]);
    }
    double s = orc_solve_speed(W, lam, mu);
    for (int a = 0; a < 3; ++a) {
        Vp[a] = W[a] / (lam[a] + mu[a] * s);
    }
    double sp = sqrt(Vp[0] * Vp[0] + Vp[1] * Vp[1] + Vp[2] * Vp[2]);
    for (int a = 0; a < 3; ++a)
        Fext[a] = eps * p->G[a] - eps * nu * kinv[a] * Vp[a] - eps * Feps * sp * sqrt(kinv[a]) * Vp[a];
}

/* ------------------------------------------------------------------------ */
/* Full permeability tensor (the rotated K of Eq. Ktensor).  A symmetric 3x3
 * matrix is held as {xx, yy, zz, xy, xz, yz}.                              */
static void sym_full(const double k[6], double M[3][3])
{
    M[0][0] = k[0]; M[1][1] = k[1]; M[2][2] = k[2];
    M[0][1] = M[1][0] = k[3];
    M[0][2] = M[2][0] = k[4];
    M[1][2] = M[2][1] = k[5];
}

/* Eigen-decomposition M = Q diag(d) Q^T of a symmetric 3x3 matrix by the
 * cyclic Jacobi method (Golub and Van Loan, Matrix Computations, Sec. 8.5):
 * plane rotations annihilate the off-diagonal entries in turn until they
 * vanish to rounding.  Columns of Q are the eigenvectors.                  */
static void jacobi3(const double Min[3][3], double d[3], double Q[3][3])
{
    double A[3][3];
    memcpy(A, Min, sizeof(A));
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) Q[i][j] = (i == j) ? 1.0 : 0.0;
    for (int sweep = 0; sweep < 60; ++sweep) {
        double off = A[0][1] * A[0][1] + A[0][2] * A[0][2] + A[1][2] * A[1][2];
        double diag = A[0][0] * A[0][0] + A[1][1] * A[1][1] + A[2][2] * A[2][2];
        if (off <= 1e-40 * diag || off == 0.0) break;
        for (int p = 0; p < 2; ++p)
            for (int q = p + 1; q < 3; ++q) {
                if (A[p][q] == 0.0) continue;
                /* rotation in the (p, q) plane that zeroes A[p][q] */
                double theta = (A[q][q] - A[p][p]) / (2.0 * A[p][q]);
                double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
                double c = 1.0 / sqrt(t * t + 1.0), sn = t * c;
                for (int k = 0; k < 3; ++k) {       /* A <- A J */
                    double akp = A[k][p], akq = A[k][q];
                    A[k][p] = c * akp - sn * akq;
                    A[k][q] = sn * akp + c * akq;
                }
                for (int k = 0; k < 3; ++k) {       /* A <- J^T A */
                    double apk = A[p][k], aqk = A[q][k];
                    A[p][k] = c * apk - sn * aqk;
                    A[q][k] = sn * apk + c * aqk;
                }
                for (int k = 0; k < 3; ++k) {       /* Q <- Q J */
                    double qkp = Q[k][p], qkq = Q[k][q];
                    Q[k][p] = c * qkp - sn * qkq;
                    Q[k][q] = sn * qkp + c * qkq;
                }
            }
    }
    for (int i = 0; i < 3; ++i) d[i] = A[i][i];
}

/* K^-1/2: the symmetric positive semi-definite square root of K^-1,
 * Q diag(sqrt(d)) Q^T (negative rounding residues of d taken as 0).       */
static void sym_sqrt(const double k[6], double out[6])
{
    double M[3][3], Q[3][3], d[3];
    sym_full(k, M);
    jacobi3(M, d, Q);
    double r[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double acc = 0.0;
            for (int a = 0; a < 3; ++a) acc += Q[i][a] * sqrt(d[a] > 0.0 ? d[a] : 0.0) * Q[j][a];
            r[i][j] = acc;
        }
    out[0] = r[0][0]; out[1] = r[1][1]; out[2] = r[2][2];
    out[3] = 0.5 * (r[0][1] + r[1][0]);
    out[4] = 0.5 * (r[0][2] + r[2][0]);
    out[5] = 0.5 * (r[1][2] + r[2][1]);
}

/* x = A^-1 b by Cramer's rule */
static void solve3(const double A[3][3], const double b[3], double x[3])
{
    double det = A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
               - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
               + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
    for (int c = 0; c < 3; ++c) {
        double B[3][3];
        memcpy(B, A, sizeof(B));
        for (int r = 0; r < 3; ++r) B[r][c] = b[r];
        x[c] = (B[0][0] * (B[1][1] * B[2][2] - B[1][2] * B[2][1])
              - B[0][1] * (B[1][0] * B[2][2] - B[1][2] * B[2][0])
              + B[0][2] * (B[1][0] * B[2][1] - B[1][1] * B[2][0])) / det;
    }
}

/* Corrected velocity and force with a full tensor: Eqs. forcement + expandV
 * give Lambda(s) V' = W with W = V + eps G / 2 and
 *   Lambda(s) = I + (eps nu / 2) K^-1 + (eps F_eps s / 2) K^-1/2,  s = |V'|.
 * The speed solves s = |Lambda(s)^-1 W|; Lambda(s) is symmetric positive
 * definite and grows with s, so s - |Lambda(s)^-1 W| is increasing and the
 * root lies in [0, |Lambda(0)^-1 W|]: safeguarded Newton, the derivative of
 * |x(s)| with x = Lambda^-1 W being -x.(Lambda^-1 B x)/|x|, B = dLambda/ds. */
static void porous_velocity_full(const orc_params *p, double eps, const double kinv[6],
                                 const double ksq[6], double nu, const double V[3],
                                 double Vp[3], double Fext[3])
{
    double Kf[3][3], Sf[3][3], A0[3][3], B[3][3], W[3];
    double Feps = p->forchheimer ? 1.75 / sqrt(150.0 * eps * eps * eps) : 0.0;
    sym_full(kinv, Kf);
    sym_full(ksq, Sf);
    for (int a = 0; a < 3; ++a) {
        W[a] = V[a] + 0.5 * eps * p->G[a];
        for (int b = 0; b < 3; ++b) {
            A0[a][b] = (a == b ? 1.0 : 0.0) + 0.5 * eps * nu * Kf[a][b];
            B[a][b] = 0.5 * eps * Feps * Sf[a][b];
        }
    }
    double x[3];
    solve3(A0, W, x);
    double hi = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
    double s = hi;
    if (Feps > 0.0 && hi > 0.0) {
        double lo = 0.0;
        for (int it = 0; it < 200; ++it) {
            double A[3][3], Bx[3], y[3];
            for (int a = 0; a < 3; ++a)
                for (int b = 0; b < 3; ++b) A[a][b] = A0[a][b] + s * B[a][b];
            solve3(A, W, x);
            double g = sqrt(x[0] * x[0] + x[1] * x[1] + x[2] * x[2]);
            double phi = s - g;
            if (phi > 0.0) hi = s; else lo = s;
            for (int a = 0; a < 3; ++a) Bx[a] = B[a][0] * x[0] + B[a][1] * x[1] + B[a][2] * x[2];
            solve3(A, Bx, y);
            double dg = g > 0.0 ? -(x[0] * y[0] + x[1] * y[1] + x[2] * y[2]) / g : 0.0;
            double sn = s - phi / (1.0 - dg);
            if (!(sn > lo && sn < hi)) sn = 0.5 * (lo + hi);
            if (fabs(sn - s) <= 1e-16 * s || hi - lo <= 1e-16 * hi) { s = sn; break; }
            s = sn;
        }
    }
    double A[3][3];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) A[a][b] = A0[a][b] + s * B[a][b];
    solve3(A, W, Vp);
    double sp = sqrt(Vp[0] * Vp[0] + Vp[1] * Vp[1] + Vp[2] * Vp[2]);
    for (int a = 0; a < 3; ++a) {
        double kv = Kf[a][0] * Vp[0] + Kf[a][1] * Vp[1] + Kf[a][2] * Vp[2];
        double sv = Sf[a][0] * Vp[0] + Sf[a][1] * Vp[1] + Sf[a][2] * Vp[2];
        Fext[a] = eps * p->G[a] - eps * nu * kv - eps * Feps * sp * sv;
    }
}

/* Equilibrium of the hydrodynamic lattice, Eqs. equilc1 and equilc2, returned
 * as deviations f^eq_i - w_i.  rho = 1 + drho.  The surface-tension part is
 * w_i A eps tau ((v.F)^2/|F| - |F|) for the moving directions and
 * + A eps tau w_0 |F| for the rest one; it is zero when |F| = 0.           */
static void feq_dev(double drho, const double u[3], double eps, double tau, double A,
                    const double F[3], double out[NQ])
{
    double rho = 1.0 + drho;
    double uu = u[0] * u[0] + u[1] * u[1] + u[2] * u[2];
    double Fn = sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]);
    for (int q = 0; q < NQ; ++q) {
        double vu = VEL[q][0] * u[0] + VEL[q][1] * u[1] + VEL[q][2] * u[2];
        double st = 0.0;
        if (q == 0) {
            out[q] = WGT[q] * drho + WGT[q] * rho * (-1.5 / eps * uu);
            if (Fn > 0.0) st = A * eps * tau * WGT[q] * Fn;
        } else {
            out[q] = WGT[q] * drho + WGT[q] * rho * (3.0 * vu + 4.5 / eps * vu * vu - 1.5 / eps * uu);
            if (Fn > 0.0) {
                double vF = VEL[q][0] * F[0] + VEL[q][1] * F[1] + VEL[q][2] * F[2];
                st = WGT[q] * A * eps * tau * (vF * vF / Fn - Fn);
            }
        }
        out[q] += st;
    }
}

/* Forcing terms of Eq. coeffforce1 with the weight w_i rho (Guo forcing).  */
static void force_terms(double rho, const double u[3], double eps, double tau,
                        const double Fx[3], double out[NQ])
{
    double pre = 1.0 - 1.0 / (2.0 * tau);
    double uF = u[0] * Fx[0] + u[1] * Fx[1] + u[2] * Fx[2];
    for (int q = 0; q < NQ; ++q) {
        double vu = VEL[q][0] * u[0] + VEL[q][1] * u[1] + VEL[q][2] * u[2];
        double vF = VEL[q][0] * Fx[0] + VEL[q][1] * Fx[1] + VEL[q][2] * Fx[2];
        if (q == 0)
            out[q] = WGT[q] * rho * pre * (-3.0 / eps * uF);
        else
            out[q] = WGT[q] * rho * pre * (3.0 * vF + 9.0 / eps * vu * vF - 3.0 / eps * uF);
    }
}

/* Solute equilibrium of Eq. equild: h^eq_i = w_i eps C (1 + 3 v_i . V*). */
static void heq(double epsC, const double vs[3], double out[NQ])
{
    for (int q = 0; q < NQ; ++q) {
        double vv = VEL[q][0] * vs[0] + VEL[q][1] * vs[1] + VEL[q][2] * vs[2];
        out[q] = (q == 0) ? WGT[q] * epsC : WGT[q] * epsC * (1.0 + 3.0 * vv);
    }
}

/* grad(eps)/eps by 3 Sum_i w_i eps(x+v_i) v_i / eps(x); a neighbour outside
 * the box or in a solid cell takes eps(x).                                 */
static void eps_gradient(const orc_state *s, int x, int y, int z, double g[3])
{
    long i0 = cidx(s, x, y, z);
    double e0 = s->eps[i0];
    g[0] = g[1] = g[2] = 0.0;
    for (int q = 1; q < NQ; ++q) {
        long j = neighbour(s, x, y, z, VEL[q][0], VEL[q][1], VEL[q][2]);
        double e = (j < 0 || s->type[j] == CELL_SOLID) ? e0 : s->eps[j];
        for (int a = 0; a < 3; ++a) g[a] += 3.0 * WGT[q] * e * VEL[q][a];
    }
    for (int a = 0; a < 3; ++a) g[a] /= e0;
}

/* colour gradient, Eq. macros: F = Sum_{i != 0} rho_1(x + v_i) v_i, over the
 * current colour field s->rho1 (solid cells hold their wall colour).     */
static void colour_gradient(const orc_state *s, int x, int y, int z, double F[3])
{
    F[0] = F[1] = F[2] = 0.0;
    for (int q = 1; q < NQ; ++q) {
        long j = neighbour(s, x, y, z, VEL[q][0], VEL[q][1], VEL[q][2]);
        double r = (j < 0) ? 0.0 : s->rho1[j];
        for (int a = 0; a < 3; ++a) F[a] += r * VEL[q][a];
    }
}

static double solute_D(const orc_params *p) { return (p->tau_d - 0.5) / 3.0; }

/* free surface with surface tension: the gradient of Eq. macros over the
 * liquid, F = Sum_{i != 0} lambda(x + v_i) v_i with the fill fraction of the
 * step's start (1 liquid, 0 gas, m / rho interface); a solid or out-of-box
 * neighbour takes lambda(x) (no wall normal).                               */
static void fs_gradient(const orc_state *s, int x, int y, int z, double F[3])
{
    long i0 = cidx(s, x, y, z);
    double l0 = s->lam[i0];
    F[0] = F[1] = F[2] = 0.0;
    for (int q = 1; q < NQ; ++q) {
        long j = neighbour(s, x, y, z, VEL[q][0], VEL[q][1], VEL[q][2]);
        double l = (j < 0 || s->type[j] == CELL_SOLID) ? l0 : s->lam[j];
        for (int a = 0; a < 3; ++a) F[a] += l * VEL[q][a];
    }
}

/* pulled (streamed) population q of lattice L at fluid cell (x,y,z):
 * f_q(x) = f~_q(x - v_q), or f~_{opp q}(x) when x - v_q is solid
 * (halfway bounce-back).                                                   */
static double pull(const orc_state *s, const double *L, int x, int y, int z, int q)
{
    long i0 = cidx(s, x, y, z);
    long j = neighbour(s, x, y, z, -VEL[q][0], -VEL[q][1], -VEL[q][2]);
    if (j < 0 || s->type[j] == CELL_SOLID) return L[(long)OPP[q] * s->n + i0];
    return L[(long)q * s->n + j];
}

/* ------------------------------------------------------------------------ */
/* Collision of one fluid cell from its streamed populations.  fin: f - w
 * deviations, hin: h (or g).  Writes post-collision values and the moments
 * (rho, V'[3], C) of this step.  t is the index of the step being computed. */
static void collide_cell(const orc_state *s, int x, int y, int z, double t,
                         const double fin[NQ], const double hin[NQ],
                         double fout[NQ], double hout[NQ], double mom[5])
{
    const orc_params *p = &s->p;
    long i0 = cidx(s, x, y, z);
    double eps = s->eps[i0];

    /* moments (Eqs. macros1, macros, all 19 directions) */
    double drho = 0.0, j[3] = {0.0, 0.0, 0.0};
    for (int q = 0; q < NQ; ++q) {
        drho += fin[q];
        for (int a = 0; a < 3; ++a) j[a] += fin[q] * VEL[q][a];
    }
    double rho = 1.0 + drho;
    double V[3] = {j[0] / rho, j[1] / rho, j[2] / rho};

    double C = 0.0, rho1 = 0.0;
    if (p->physics == PHYS_MISCIBLE) {
        double sh = 0.0;
        for (int q = 0; q < NQ; ++q) sh += hin[q];
        C = sh / eps;
    } else if (p->physics == PHYS_IMMISCIBLE) {
        for (int q = 0; q < NQ; ++q) rho1 += hin[q];
        C = rho1 / rho;
    }

    double nu = viscosity(p, C, t);
    double tau = 0.5 + 3.0 * nu;

    double Vp[3], Fext[3];
    if (p->full_tensor) {
        double kinv[6], ksq[6];
        for (int c = 0; c < 6; ++c) {
            kinv[c] = s->kinv[c * s->n + i0];
            ksq[c] = s->ksqrt[c * s->n + i0];
        }
        porous_velocity_full(p, eps, kinv, ksq, nu, V, Vp, Fext);
    } else {
        double kinv[3] = {s->kinv[i0], s->kinv[s->n + i0], s->kinv[2 * s->n + i0]};
        porous_velocity(p, eps, kinv, nu, V, Vp, Fext);
    }

    double F[3] = {0.0, 0.0, 0.0};
    if (p->physics == PHYS_IMMISCIBLE) colour_gradient(s, x, y, z, F);
    else if (p->physics == PHYS_FREESURF && p->A != 0.0) fs_gradient(s, x, y, z, F);

    double eq[NQ], T[NQ];
    feq_dev(drho, Vp, eps, tau, p->A, F, eq);
    force_terms(rho, Vp, eps, tau, Fext, T);
    for (int q = 0; q < NQ; ++q) fout[q] = fin[q] - (fin[q] - eq[q]) / tau + T[q];

    if (p->physics == PHYS_MISCIBLE) {
        double D = solute_D(p), vs[3] = {Vp[0], Vp[1], Vp[2]};
        if (p->eps_grad) {
            double g[3];
            eps_gradient(s, x, y, z, g);
            for (int a = 0; a < 3; ++a) vs[a] += D * g[a];
        }
        double he[NQ];
        heq(eps * C, vs, he);
        for (int q = 0; q < NQ; ++q) hout[q] = hin[q] - (hin[q] - he[q]) / p->tau_d;
    } else if (p->physics == PHYS_IMMISCIBLE) {
        double Fn = sqrt(F[0] * F[0] + F[1] * F[1] + F[2] * F[2]);
        for (int q = 0; q < NQ; ++q) {
            double ft = WGT[q] + fout[q];
            double rec = 0.0;
            if (q != 0 && Fn > 0.0) {
                double vF = VEL[q][0] * F[0] + VEL[q][1] * F[1] + VEL[q][2] * F[2];
                double vn = sqrt((double)(VEL[q][0] * VEL[q][0] + VEL[q][1] * VEL[q][1] + VEL[q][2] * VEL[q][2]));
                rec = p->beta * C * (1.0 - C) * rho * WGT[q] * vF / (vn * Fn);
            }
            hout[q] = C * ft + rec;
        }
    }
    mom[0] = rho;
    mom[1] = Vp[0];
    mom[2] = Vp[1];
    mom[3] = Vp[2];
    mom[4] = C;
}

/* Solutes beyond the first (the extension to several species that Sec. 2.2
 * prepares): each has its own lattice, relaxation time tau_d,k and reservoir
 * concentrations, and follows Eqs. equild and boltzeqD with the velocity V'
 * of the hydrodynamic lattice, exactly as the first solute; the viscosity
 * law reads the first solute's concentration.  From the streamed hin of
 * solute k (k >= 1) at a fluid cell: hout and C_k.                         */
static double solute_extra(const orc_state *s, int x, int y, int z, int k, const double Vp[3],
                           const double hin[NQ], double hout[NQ])
{
    const orc_params *p = &s->p;
    long i0 = cidx(s, x, y, z);
    double eps = s->eps[i0];
    double sh = 0.0;
    for (int q = 0; q < NQ; ++q) sh += hin[q];
    double C = sh / eps;
    double tau_d = p->tau_dx[k - 1];
    double D = (tau_d - 0.5) / 3.0, vs[3] = {Vp[0], Vp[1], Vp[2]};
    if (p->eps_grad) {
        double g[3];
        eps_gradient(s, x, y, z, g);
        for (int a = 0; a < 3; ++a) vs[a] += D * g[a];
    }
    double he[NQ];
    heq(eps * C, vs, he);
    for (int q = 0; q < NQ; ++q) hout[q] = hin[q] - (hin[q] - he[q]) / tau_d;
    return C;
}

/* fixed state of a reservoir cell: the equilibrium of (rho_bc, V' = 0, F = 0);
 * solute h = w eps C_bc; fluid-1 populations g = C_bc w rho_bc.            */
static void reservoir_state(const orc_state *s, long i, double fo[NQ], double ho[NQ], double mom[5])
{
    int f = s->tface[i];
    double rb = s->p.face_rho[f], cb = s->p.face_conc[f];
    for (int q = 0; q < NQ; ++q) {
        fo[q] = WGT[q] * (rb - 1.0);
        if (s->p.physics == PHYS_MISCIBLE) ho[q] = WGT[q] * s->eps[i] * cb;
        else if (s->p.physics == PHYS_IMMISCIBLE) ho[q] = cb * WGT[q] * rb;
        else ho[q] = 0.0;
    }
    mom[0] = rb;
    mom[1] = mom[2] = mom[3] = 0.0;
    mom[4] = (s->p.physics == PHYS_SINGLE) ? 0.0 : cb;
}

/* colour field of the current step: fluid cells Sum of streamed g, reservoir
 * cells C_bc rho_bc, solid cells their wall colour.                       */
static void colour_field(orc_state *s, int from_state)
{
    const double *G = s->h[s->cur];
    int nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = cidx(s, x, y, z);
                double r;
                if (s->type[i] == CELL_SOLID) r = wall_colour(s, s->tface[i]);
                else if (s->type[i] == CELL_RESERVOIR) r = s->p.face_conc[s->tface[i]] * s->p.face_rho[s->tface[i]];
                else if (from_state) {
                    r = 0.0;
                    for (int q = 0; q < NQ; ++q) r += pull(s, G, x, y, z, q);
                } else r = s->conc[i] * s->rho[i];
                s->rho1[i] = r;
            }
}

/* ------------------------------------------------------------------------ */
/* public API (ctypes) */

void orc_lattice(int *vel, double *w, int *opp)
{
    lattice_setup();
    for (int q = 0; q < NQ; ++q) {
        for (int a = 0; a < 3; ++a) vel[3 * q + a] = VEL[q][a];
        w[q] = WGT[q];
        if (opp) opp[q] = OPP[q];
    }
}

/* point functions for the identity tests (absolute populations) */
void orc_feq(double rho, const double u[3], double eps, double tau, double A, const double F[3], double out[NQ])
{
    lattice_setup();
    feq_dev(rho - 1.0, u, eps, tau, A, F, out);
    for (int q = 0; q < NQ; ++q) out[q] += WGT[q];
}

void orc_force(double rho, const double u[3], double eps, double tau, const double Fext[3], double out[NQ])
{
    lattice_setup();
    force_terms(rho, u, eps, tau, Fext, out);
}

void orc_heq(double epsC, const double vs[3], double out[NQ])
{
    lattice_setup();
    heq(epsC, vs, out);
}

double orc_viscosity(const orc_params *p, double C, double t) { return viscosity(p, C, t); }

void orc_porous_velocity(const orc_params *p, double eps, const double kinv[3], double nu,
                         const double V[3], double Vp[3], double Fext[3])
{
    porous_velocity(p, eps, kinv, nu, V, Vp, Fext);
}

/* number of OpenMP threads of the following calls (the CPU baseline times
 * the oracle with one thread and with all of them) */
void orc_set_threads(int n)
{
#ifdef _OPENMP
    if (n > 0) omp_set_num_threads(n);
#else
    (void)n;
#endif
}

/* full-tensor forms for the tests: K^-1/2 of one cell, and V', F^ext */
void orc_sym_sqrt(const double k[6], double out[6]) { sym_sqrt(k, out); }

void orc_porous_velocity_full(const orc_params *p, double eps, const double kinv[6], double nu,
                              const double V[3], double Vp[3], double Fext[3])
{
    double ksq[6];
    sym_sqrt(kinv, ksq);
    porous_velocity_full(p, eps, kinv, ksq, nu, V, Vp, Fext);
}

void orc_destroy(orc_state *s)
{
    if (!s) return;
    free(s->eps); free(s->kinv); free(s->ksqrt); free(s->type); free(s->tface);
    free(s->f[0]); free(s->f[1]); free(s->h[0]); free(s->h[1]);
    free(s->rho); free(s->vel); free(s->conc); free(s->vsnap); free(s->rho1);
    free(s->fst); free(s->mass); free(s->lam);
    free(s->hx[0]); free(s->hx[1]); free(s->concx);
    free(s);
}


/* ------------------------------------------------------------------------ */
/* Free-surface technique (Sec. 3; the method of the cited free-surface
 * reference, whose details the paper defers to):  a liquid penetrating
 * empty space.  Non-solid cells are liquid (full), gas (empty, no state) or
 * interface (liquid mass m, fill fraction lambda = m / rho).
 * Readings of the points the paper leaves open:
 *  - mass exchange (Eq. deltamass) only over links to liquid or interface
 *    neighbours: weight 1 to a liquid neighbour, (lambda(x) + lambda(y))/2 to
 *    an interface neighbour, 0 to a gas cell (the printed average applied to
 *    gas and liquid links would not conserve mass);
 *  - populations arriving from a gas cell (Eq. equilempty) use the
 *    equilibria at the gas density rho_A = 1 and the velocity of the
 *    receiving cell's own post-collision populations (its state at t);
 *  - conversion thresholds: m > (1 + kappa) rho -> liquid, m < -kappa rho ->
 *    gas, kappa = 1e-3; a cell that would empty next to one that fills stays
 *    interface; gas cells next to a new liquid cell become interface cells
 *    with the equilibrium of the mean density and velocity (rho and V' of
 *    the step) of their liquid / interface neighbours that do not empty, and
 *    m = 0; liquid cells next to a new gas cell
 *    become interface cells with m = rho;
 *  - the excess mass of a converted cell (m - rho, or m for a new gas cell)
 *    is shared equally among its neighbours that end the step as interface
 *    cells (mass is lost only if there is none, and counted). */
#define FS_KAPPA 1e-3
#define FS_RHO_A 1.0
enum { FS_NONE = 0, FS_TO_LIQ = 1, FS_TO_GAS = 2 };

static int fs_open(const orc_state *s, long j)
{
    return j >= 0 && s->type[j] != CELL_SOLID;
}

/* set up the cell classes and masses from the initial fill fraction c0 */
static int fs_init(orc_state *s, const double *c0, const double *rho0)
{
    long n = s->n;
    s->fst = calloc(n, 1);
    s->mass = calloc(n, sizeof(double));
    s->lam = calloc(n, sizeof(double));
    if (!s->fst || !s->mass || !s->lam) return -1;
    for (long i = 0; i < n; ++i) {
        if (s->type[i] != CELL_FLUID) continue;
        double l = c0[i];
        s->fst[i] = l >= 1.0 ? FS_LIQ : (l <= 0.0 ? FS_GAS : FS_IF);
    }
    /* a liquid cell next to a gas cell is an interface cell */
    int nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
    unsigned char *t2 = malloc(n);
    if (!t2) return -1;
    memcpy(t2, s->fst, n);
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = cidx(s, x, y, z);
                if (s->type[i] != CELL_FLUID || s->fst[i] != FS_LIQ) continue;
                for (int q = 1; q < NQ; ++q) {
                    long j = neighbour(s, x, y, z, VEL[q][0], VEL[q][1], VEL[q][2]);
                    if (fs_open(s, j) && s->fst[j] == FS_GAS) t2[i] = FS_IF;
                }
            }
    memcpy(s->fst, t2, n);
    free(t2);
    for (long i = 0; i < n; ++i) {
        if (s->type[i] != CELL_FLUID) continue;
        double l = c0[i] < 0.0 ? 0.0 : (c0[i] > 1.0 ? 1.0 : c0[i]);
        if (s->fst[i] == FS_GAS) {
            for (int q = 0; q < NQ; ++q) s->f[0][(long)q * n + i] = 0.0;
            s->rho[i] = 0.0;
            for (int a = 0; a < 3; ++a) s->vel[a * n + i] = 0.0;
            s->mass[i] = s->lam[i] = s->conc[i] = 0.0;
        } else {
            if (s->fst[i] == FS_LIQ) l = 1.0;
            s->mass[i] = l * rho0[i];
            s->lam[i] = l;
            s->conc[i] = l;
        }
    }
    return 0;
}

/* One free-surface step: stream the populations and the mass, collide,
 * then redefine the cell classes (flowchart of Sec. 4).                    */
static int fs_step(orc_state *s, double t)
{
    const orc_params *p = &s->p;
    long n = s->n;
    int nx = p->nx, ny = p->ny, nz = p->nz;
    const double *Fc = s->f[s->cur];
    double *Fn = s->f[1 - s->cur];
    double *mnew = malloc(sizeof(double) * n), *share = calloc(n, sizeof(double));
    unsigned char *flag = calloc(n, 1), *flag2 = calloc(n, 1), *nt = malloc(n);
    if (!mnew || !share || !flag || !flag2 || !nt) {
        free(mnew); free(share); free(flag); free(flag2); free(nt);
        return -1;
    }

    /* 1. stream (with the gas-side reconstruction), exchange mass, collide */
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = cidx(s, x, y, z);
                mnew[i] = 0.0;
                if (s->type[i] != CELL_FLUID) continue;
                if (s->fst[i] == FS_GAS) {
                    for (int q = 0; q < NQ; ++q) Fn[(long)q * n + i] = 0.0;
                    continue;
                }
                double own[NQ], fin[NQ], hin[NQ], fo[NQ], ho[NQ], mom[5];
                double orho = 1.0, oj[3] = {0.0, 0.0, 0.0};
                for (int q = 0; q < NQ; ++q) {
                    own[q] = Fc[(long)q * n + i];
                    orho += own[q];
                    for (int a = 0; a < 3; ++a) oj[a] += own[q] * VEL[q][a];
                    hin[q] = 0.0;
                }
                double ou[3] = {oj[0] / orho, oj[1] / orho, oj[2] / orho};
                double eqA[NQ], F0[3] = {0.0, 0.0, 0.0};
                feq_dev(FS_RHO_A - 1.0, ou, s->eps[i], 1.0, 0.0, F0, eqA);
                for (int q = 0; q < NQ; ++q) {
                    long j = neighbour(s, x, y, z, -VEL[q][0], -VEL[q][1], -VEL[q][2]);
                    if (!fs_open(s, j)) fin[q] = own[OPP[q]];
                    else if (s->fst[j] == FS_GAS) fin[q] = eqA[q] + eqA[OPP[q]] - own[OPP[q]];
                    else fin[q] = Fc[(long)q * n + j];
                }
                double m = s->mass[i];
                if (s->fst[i] == FS_IF) {
                    double dm = 0.0;
                    for (int q = 1; q < NQ; ++q) {
                        long j = neighbour(s, x, y, z, VEL[q][0], VEL[q][1], VEL[q][2]);
                        if (!fs_open(s, j) || s->fst[j] == FS_GAS) continue;
                        double flux = Fc[(long)OPP[q] * n + j] - own[q];
                        dm += s->fst[j] == FS_LIQ ? flux : flux * 0.5 * (s->lam[i] + s->lam[j]);
                    }
                    m += dm;
                }
                collide_cell(s, x, y, z, t, fin, hin, fo, ho, mom);
                for (int q = 0; q < NQ; ++q) Fn[(long)q * n + i] = fo[q];
                double rho = mom[0];
                if (s->fst[i] == FS_LIQ) m = rho;
                mnew[i] = m;
                s->rho[i] = rho;
                for (int a = 0; a < 3; ++a) s->vel[a * n + i] = mom[1 + a];
                if (s->fst[i] == FS_IF) {
                    if (m > (1.0 + FS_KAPPA) * rho) flag[i] = FS_TO_LIQ;
                    else if (m < -FS_KAPPA * rho) flag[i] = FS_TO_GAS;
                }
            }

    /* 2. conflicts and the new classes */
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = cidx(s, x, y, z);
                nt[i] = s->type[i] == CELL_FLUID ? s->fst[i] : FS_GAS;
                flag2[i] = flag[i];
                if (s->type[i] != CELL_FLUID) continue;
                int near_liq = 0;
                for (int q = 1; q < NQ; ++q) {
                    long j = neighbour(s, x, y, z, VEL[q][0], VEL[q][1], VEL[q][2]);
                    if (fs_open(s, j) && flag[j] == FS_TO_LIQ) near_liq = 1;
                }
                if (flag[i] == FS_TO_GAS && near_liq) flag2[i] = FS_NONE;
                if (s->fst[i] == FS_GAS && near_liq) nt[i] = FS_IF;
            }
    /* converting cells take their new class; a liquid cell next to a cell
     * that empties after all becomes an interface cell */
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = cidx(s, x, y, z);
                if (s->type[i] != CELL_FLUID) continue;
                if (flag2[i] == FS_TO_LIQ) nt[i] = FS_LIQ;
                else if (flag2[i] == FS_TO_GAS) nt[i] = FS_GAS;
                else if (s->fst[i] == FS_LIQ) {
                    int near_gas = 0;
                    for (int q = 1; q < NQ; ++q) {
                        long j = neighbour(s, x, y, z, VEL[q][0], VEL[q][1], VEL[q][2]);
                        if (fs_open(s, j) && flag2[j] == FS_TO_GAS) near_gas = 1;
                    }
                    nt[i] = near_gas ? FS_IF : FS_LIQ;
                }
            }

    /* 3. gas cells turned interface: equilibrium of the mean density and
     *    velocity (rho and V' of this step) of their liquid and interface
     *    neighbours that do not empty */
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = cidx(s, x, y, z);
                if (s->type[i] != CELL_FLUID || s->fst[i] != FS_GAS || nt[i] != FS_IF) continue;
                double rs = 0.0, us[3] = {0.0, 0.0, 0.0};
                int k = 0;
                for (int q = 1; q < NQ; ++q) {
                    long j = neighbour(s, x, y, z, VEL[q][0], VEL[q][1], VEL[q][2]);
                    if (!fs_open(s, j) || s->fst[j] == FS_GAS || flag2[j] == FS_TO_GAS) continue;
                    rs += s->rho[j];
                    for (int a = 0; a < 3; ++a) us[a] += s->vel[a * n + j];
                    ++k;
                }
                double ra = rs / k, ua[3] = {us[0] / k, us[1] / k, us[2] / k}, fo[NQ], F0[3] = {0.0, 0.0, 0.0};
                double tau = 0.5 + 3.0 * viscosity(p, 0.0, t);
                feq_dev(ra - 1.0, ua, s->eps[i], tau, 0.0, F0, fo);
                for (int q = 0; q < NQ; ++q) Fn[(long)q * n + i] = fo[q];
                s->rho[i] = ra;
                for (int a = 0; a < 3; ++a) s->vel[a * n + i] = ua[a];
                mnew[i] = 0.0;
            }

    /* 4. excess mass of the converted cells, shared among the neighbours that
     *    end the step as interface cells */
    double lost = 0.0;
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = cidx(s, x, y, z);
                if (s->type[i] != CELL_FLUID || flag2[i] == FS_NONE) continue;
                double ex = flag2[i] == FS_TO_LIQ ? mnew[i] - s->rho[i] : mnew[i];
                int k = 0;
                for (int q = 1; q < NQ; ++q) {
                    long j = neighbour(s, x, y, z, VEL[q][0], VEL[q][1], VEL[q][2]);
                    if (fs_open(s, j) && nt[j] == FS_IF && flag2[j] == FS_NONE) ++k;
                }
                share[i] = k > 0 ? ex / k : 0.0;
                if (k == 0) lost += ex;
            }
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = cidx(s, x, y, z);
                if (s->type[i] != CELL_FLUID) continue;
                double m = mnew[i];
                if (nt[i] == FS_IF) {
                    for (int q = 1; q < NQ; ++q) {
                        long j = neighbour(s, x, y, z, VEL[q][0], VEL[q][1], VEL[q][2]);
                        if (fs_open(s, j) && flag2[j] != FS_NONE) m += share[j];
                    }
                } else if (nt[i] == FS_LIQ) {
                    m = s->rho[i];
                } else {
                    m = 0.0;
                }
                s->mass[i] = m;
            }
    /* 5. new classes, fill fractions, moments of gas cells */
    for (long i = 0; i < n; ++i) {
        if (s->type[i] != CELL_FLUID) continue;
        s->fst[i] = nt[i];
        if (nt[i] == FS_GAS) {
            s->lam[i] = 0.0;
            s->rho[i] = 0.0;
            for (int a = 0; a < 3; ++a) s->vel[a * n + i] = 0.0;
            for (int q = 0; q < NQ; ++q) Fn[(long)q * n + i] = 0.0;
        } else {
            s->lam[i] = nt[i] == FS_LIQ ? 1.0 : s->mass[i] / s->rho[i];
        }
        s->conc[i] = s->lam[i];
    }
    s->fs_lost += lost;
    free(mnew); free(share); free(flag); free(flag2); free(nt);
    return 0;
}

/* Create the state and apply the initial conditions (flowchart, first three
 * boxes): f = f^eq(rho0, V' := V0, F, eps, tau(C0, 0)); h = h^eq(eps C0,
 * V0 + D grad(eps)/eps); g = C0 f.  Arrays are FP64, idx = x + nx (y + ny z);
 * kinv holds 3 planes (6 with full_tensor), vel0 3 planes; solid (may be NULL) marks obstacle cells,
 * which carry no state and reflect the populations that stream into them.
 * Returns NULL on allocation failure.                                      */
orc_state *orc_create(const orc_params *p, const double *eps, const double *kinv,
                      const double *rho0, const double *vel0, const double *c0,
                      const unsigned char *solid)
{
    lattice_setup();
    if (p->nspecies < 0 || p->nspecies > ORC_MAXSP || (p->nspecies > 1 && p->physics != PHYS_MISCIBLE)) return NULL;
    if (p->physics == PHYS_FREESURF)
        for (int f = 0; f < 6; ++f)
            if (p->face_kind[f] == FACE_RESERVOIR) return NULL;
    orc_state *s = (orc_state *)calloc(1, sizeof(orc_state));
    if (!s) return NULL;
    s->p = *p;
    s->n = (long)p->nx * p->ny * p->nz;
    long n = s->n;
    s->eps = malloc(sizeof(double) * n);
    const int nk = p->full_tensor ? 6 : 3;
    s->kinv = malloc(sizeof(double) * nk * n);
    s->ksqrt = p->full_tensor ? malloc(sizeof(double) * 6 * n) : NULL;
    s->type = malloc(n);
    s->tface = malloc(n);
    s->f[0] = calloc((size_t)NQ * n, sizeof(double));
    s->h[0] = calloc((size_t)NQ * n, sizeof(double));
    s->rho = calloc(n, sizeof(double));
    s->vel = calloc(3 * n, sizeof(double));
    s->conc = calloc(n, sizeof(double));
    s->vsnap = calloc(3 * n, sizeof(double));
    s->rho1 = calloc(n, sizeof(double));
    if (!s->eps || !s->kinv || (p->full_tensor && !s->ksqrt) || !s->type || !s->tface || !s->f[0] || !s->h[0] || !s->rho ||
        !s->vel || !s->conc || !s->vsnap || !s->rho1) { orc_destroy(s); return NULL; }
    s->nsx = (p->physics == PHYS_MISCIBLE && p->nspecies > 1) ? p->nspecies - 1 : 0;
    if (s->nsx) {
        s->hx[0] = calloc((size_t)s->nsx * NQ * n, sizeof(double));
        s->hx[1] = calloc((size_t)s->nsx * NQ * n, sizeof(double));
        s->concx = calloc((size_t)s->nsx * n, sizeof(double));
        if (!s->hx[0] || !s->hx[1] || !s->concx) { orc_destroy(s); return NULL; }
    }
    memcpy(s->eps, eps, sizeof(double) * n);
    memcpy(s->kinv, kinv, sizeof(double) * nk * n);
    if (p->full_tensor) {
        for (long i = 0; i < n; ++i) {
            double k[6], r[6];
            for (int c = 0; c < 6; ++c) k[c] = kinv[c * n + i];
            sym_sqrt(k, r);
            for (int c = 0; c < 6; ++c) s->ksqrt[c * n + i] = r[c];
        }
    }
    classify(s, solid);
    s->cur = 0;

    /* initial moments */
    for (long i = 0; i < n; ++i) {
        if (s->type[i] == CELL_FLUID) {
            s->rho[i] = rho0[i];
            for (int a = 0; a < 3; ++a) s->vel[a * n + i] = vel0[a * n + i];
            s->conc[i] = (p->physics == PHYS_SINGLE) ? 0.0 : c0[i];
        }
    }
    if (p->physics == PHYS_IMMISCIBLE) colour_field(s, 0);

    int nx = p->nx, ny = p->ny, nz = p->nz;
#pragma omp parallel for collapse(2) schedule(static)
    for (int z = 0; z < nz; ++z)
        for (int y = 0; y < ny; ++y)
            for (int x = 0; x < nx; ++x) {
                long i = cidx(s, x, y, z);
                double fo[NQ], ho[NQ], mom[5];
                if (s->type[i] == CELL_SOLID) continue;
                if (s->type[i] == CELL_RESERVOIR) {
                    reservoir_state(s, i, fo, ho, mom);
                    s->rho[i] = mom[0];
                    s->conc[i] = mom[4];
                } else {
                    double u[3] = {vel0[i], vel0[n + i], vel0[2 * n + i]};
                    double C = s->conc[i];
                    double tau = 0.5 + 3.0 * viscosity(p, C, 0.0);
                    double F[3] = {0.0, 0.0, 0.0};
                    if (p->physics == PHYS_IMMISCIBLE) colour_gradient(s, x, y, z, F);
                    feq_dev(rho0[i] - 1.0, u, eps[i], tau, p->A, F, fo);
                    if (p->physics == PHYS_MISCIBLE) {
                        double vs[3] = {u[0], u[1], u[2]};
                        if (p->eps_grad) {
                            double g[3];
                            eps_gradient(s, x, y, z, g);
                            for (int a = 0; a < 3; ++a) vs[a] += solute_D(p) * g[a];
                        }
                        heq(eps[i] * C, vs, ho);
                    } else if (p->physics == PHYS_IMMISCIBLE) {
                        for (int q = 0; q < NQ; ++q) ho[q] = C * (WGT[q] + fo[q]);
                    } else {
                        for (int q = 0; q < NQ; ++q) ho[q] = 0.0;
                    }
                }
                for (int q = 0; q < NQ; ++q) {
                    s->f[0][(long)q * n + i] = fo[q];
                    s->h[0][(long)q * n + i] = ho[q];
                }
            }
    /* solutes beyond the first: h = h^eq(eps C0_k, V0 + D_k grad(eps)/eps), c0
     * holding one plane per solute; reservoir cells w eps C_bc,k */
    for (int k = 1; k <= s->nsx; ++k) {
        double *H = s->hx[0] + (size_t)(k - 1) * NQ * n;
        double D = (p->tau_dx[k - 1] - 0.5) / 3.0;
#pragma omp parallel for collapse(2) schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    long i = cidx(s, x, y, z);
                    double ho[NQ], C = 0.0;
                    if (s->type[i] == CELL_SOLID) continue;
                    if (s->type[i] == CELL_RESERVOIR) {
                        C = p->face_concx[k - 1][s->tface[i]];
                        for (int q = 0; q < NQ; ++q) ho[q] = WGT[q] * s->eps[i] * C;
                    } else {
                        double vs[3] = {vel0[i], vel0[n + i], vel0[2 * n + i]};
                        C = c0[(size_t)k * n + i];
                        if (p->eps_grad) {
                            double g[3];
                            eps_gradient(s, x, y, z, g);
                            for (int a = 0; a < 3; ++a) vs[a] += D * g[a];
                        }
                        heq(eps[i] * C, vs, ho);
                    }
                    for (int q = 0; q < NQ; ++q) H[(long)q * n + i] = ho[q];
                    s->concx[(size_t)(k - 1) * n + i] = C;
                }
    }
    if (s->nsx) memcpy(s->hx[1], s->hx[0], sizeof(double) * (size_t)s->nsx * NQ * n);
    if (p->physics == PHYS_FREESURF && fs_init(s, c0, rho0) != 0) { orc_destroy(s); return NULL; }
    memcpy(s->vsnap, s->vel, sizeof(double) * 3 * n);
    s->step = 0;
    return s;
}

/* Advance nsteps steps (flowchart loop).  Returns 0, or -1 on allocation
 * failure.                                                                 */
int orc_step(orc_state *s, int nsteps)
{
    long n = s->n;
    if (!s->f[1]) {
        s->f[1] = calloc((size_t)NQ * n, sizeof(double));
        s->h[1] = calloc((size_t)NQ * n, sizeof(double));
        if (!s->f[1] || !s->h[1]) return -1;
        memcpy(s->f[1], s->f[0], sizeof(double) * NQ * n);
        memcpy(s->h[1], s->h[0], sizeof(double) * NQ * n);
    }
    int nx = s->p.nx, ny = s->p.ny, nz = s->p.nz;
    for (int it = 0; it < nsteps; ++it) {
        double t = (double)(s->step + 1);
        if (s->p.physics == PHYS_FREESURF) {
            if (fs_step(s, t) != 0) return -1;
            s->cur = 1 - s->cur;
            s->step += 1;
            continue;
        }
        const double *Fc = s->f[s->cur], *Hc = s->h[s->cur];
        double *Fn = s->f[1 - s->cur], *Hn = s->h[1 - s->cur];
        if (s->p.physics == PHYS_IMMISCIBLE) colour_field(s, 1);
#pragma omp parallel for collapse(2) schedule(static)
        for (int z = 0; z < nz; ++z)
            for (int y = 0; y < ny; ++y)
                for (int x = 0; x < nx; ++x) {
                    long i = cidx(s, x, y, z);
                    double fin[NQ], hin[NQ], fo[NQ], ho[NQ], mom[5];
                    if (s->type[i] == CELL_SOLID) continue;
                    if (s->type[i] == CELL_RESERVOIR) {
                        reservoir_state(s, i, fo, ho, mom);
                    } else {
                        for (int q = 0; q < NQ; ++q) {
                            fin[q] = pull(s, Fc, x, y, z, q);
                            hin[q] = (s->p.physics == PHYS_SINGLE) ? 0.0 : pull(s, Hc, x, y, z, q);
                        }
                        collide_cell(s, x, y, z, t, fin, hin, fo, ho, mom);
                    }
                    for (int q = 0; q < NQ; ++q) {
                        Fn[(long)q * n + i] = fo[q];
                        Hn[(long)q * n + i] = ho[q];
                    }
                    for (int k = 1; k <= s->nsx; ++k) {
                        const double *Xc = s->hx[s->cur] + (size_t)(k - 1) * NQ * n;
                        double *Xn = s->hx[1 - s->cur] + (size_t)(k - 1) * NQ * n;
                        double xin[NQ], xo[NQ], C;
                        if (s->type[i] == CELL_RESERVOIR) {
                            C = s->p.face_concx[k - 1][s->tface[i]];
                            for (int q = 0; q < NQ; ++q) xo[q] = WGT[q] * s->eps[i] * C;
                        } else {
                            for (int q = 0; q < NQ; ++q) xin[q] = pull(s, Xc, x, y, z, q);
                            C = solute_extra(s, x, y, z, k, mom + 1, xin, xo);
                        }
                        for (int q = 0; q < NQ; ++q) Xn[(long)q * n + i] = xo[q];
                        s->concx[(size_t)(k - 1) * n + i] = C;
                    }
                    s->rho[i] = mom[0];
                    s->vel[i] = mom[1];
                    s->vel[n + i] = mom[2];
                    s->vel[2 * n + i] = mom[3];
                    s->conc[i] = mom[4];
                }
        s->cur = 1 - s->cur;
        s->step += 1;
    }
    return 0;
}

long orc_steps_done(const orc_state *s) { return s->step; }

/* moments of the last step (before its collision); after 0 steps the initial
 * fields.  Solid cells read 0.  Any pointer may be NULL.                  */
void orc_moments(const orc_state *s, double *rho, double *vel, double *conc)
{
    long n = s->n;
    if (rho) memcpy(rho, s->rho, sizeof(double) * n);
    if (vel) memcpy(vel, s->vel, sizeof(double) * 3 * n);
    if (conc) memcpy(conc, s->conc, sizeof(double) * n);
}

/* Diagnostics over fluid cells (free surface: liquid and interface cells):
 * {Sum rho, Sum rho V'_x, _y, _z, Sum eps C (miscible) or Sum rho_1
 * (two-fluid) or Sum m (free surface) or 0, |V' - V'_snap|^2 / |V'|^2,
 * max |V'|, number of cells with a non-finite moment}.  The snapshot is
 * replaced by the current V'.                                              */
void orc_diag(orc_state *s, double out[8])
{
    long n = s->n;
    double acc[7] = {0, 0, 0, 0, 0, 0, 0}, vmax = 0.0, bad = 0.0;
    for (long i = 0; i < n; ++i) {
        if (s->type[i] != CELL_FLUID) continue;
        if (s->p.physics == PHYS_FREESURF && s->fst[i] == FS_GAS) continue;
        double r = s->rho[i], u[3] = {s->vel[i], s->vel[n + i], s->vel[2 * n + i]}, c = s->conc[i];
        if (!isfinite(r) || !isfinite(u[0]) || !isfinite(u[1]) || !isfinite(u[2]) || !isfinite(c)) { bad += 1.0; continue; }
        acc[0] += r;
        for (int a = 0; a < 3; ++a) acc[1 + a] += r * u[a];
        if (s->p.physics == PHYS_MISCIBLE) acc[4] += s->eps[i] * c;
        else if (s->p.physics == PHYS_IMMISCIBLE) acc[4] += c * r;
        else if (s->p.physics == PHYS_FREESURF) acc[4] += s->mass[i];
        double du = 0.0, uu = 0.0;
        for (int a = 0; a < 3; ++a) {
            double d = u[a] - s->vsnap[a * n + i];
            du += d * d;
            uu += u[a] * u[a];
        }
        acc[5] += du;
        acc[6] += uu;
        if (sqrt(uu) > vmax) vmax = sqrt(uu);
    }
    for (int k = 0; k < 5; ++k) out[k] = acc[k];
    out[5] = acc[6] > 0.0 ? acc[5] / acc[6] : 0.0;
    out[6] = vmax;
    out[7] = bad;
    memcpy(s->vsnap, s->vel, sizeof(double) * 3 * n);
}

/* current post-collision populations of lattice L (0: f as deviations
 * f - w, 1: h or g, 2..: the further solutes), 19 planes in this file's
 * direction order.                                                         */
void orc_get_state(const orc_state *s, int L, double *out)
{
    if (L >= 2) {
        memcpy(out, s->hx[s->cur] + (size_t)(L - 2) * NQ * s->n, sizeof(double) * NQ * s->n);
        return;
    }
    memcpy(out, L == 0 ? s->f[s->cur] : s->h[s->cur], sizeof(double) * NQ * s->n);
}

/* replace the post-collision populations and the completed-step count. */
void orc_set_state(orc_state *s, int L, const double *in, long step)
{
    memcpy(L == 0 ? s->f[s->cur] : s->h[s->cur], in, sizeof(double) * NQ * s->n);
    s->step = step;
}

/* One step for the listed cells only, from the current state, without
 * changing it: writes post-collision populations (19 per cell, this file's
 * order) and moments (5 per cell).  Non-fluid cells get their fixed state.
 * For the two-fluid model the colour field of the step is needed: it is
 * recomputed for the whole box first.                                      */
void orc_step_cells(orc_state *s, long ncells, const long *cells, double *fo_out,
                    double *ho_out, double *mom_out)
{
    if (s->p.physics == PHYS_FREESURF) return;   /* the class update is not local */
    double t = (double)(s->step + 1);
    const double *Fc = s->f[s->cur], *Hc = s->h[s->cur];
    if (s->p.physics == PHYS_IMMISCIBLE) colour_field(s, 1);
#pragma omp parallel for schedule(static)
    for (long k = 0; k < ncells; ++k) {
        long i = cells[k];
        int x = (int)(i % s->p.nx), y = (int)((i / s->p.nx) % s->p.ny), z = (int)(i / ((long)s->p.nx * s->p.ny));
        double fin[NQ], hin[NQ], fo[NQ], ho[NQ], mom[5];
        if (s->type[i] == CELL_SOLID) {
            for (int q = 0; q < NQ; ++q) fo[q] = ho[q] = 0.0;
            for (int a = 0; a < 5; ++a) mom[a] = 0.0;
        } else if (s->type[i] == CELL_RESERVOIR) {
            reservoir_state(s, i, fo, ho, mom);
        } else {
            for (int q = 0; q < NQ; ++q) {
                fin[q] = pull(s, Fc, x, y, z, q);
                hin[q] = (s->p.physics == PHYS_SINGLE) ? 0.0 : pull(s, Hc, x, y, z, q);
            }
            collide_cell(s, x, y, z, t, fin, hin, fo, ho, mom);
        }
        for (int q = 0; q < NQ; ++q) {
            fo_out[k * NQ + q] = fo[q];
            ho_out[k * NQ + q] = ho[q];
        }
        for (int a = 0; a < 5; ++a) mom_out[k * 5 + a] = mom[a];
    }
}

/* cell classes (0 fluid, 1 solid, 2 reservoir) */
void orc_cell_types(const orc_state *s, unsigned char *out) { memcpy(out, s->type, s->n); }

/* concentration of solute k (0: the first) of the last step into out (ncell). */
int orc_species_conc(const orc_state *s, int k, double *out)
{
    if (k == 0) { memcpy(out, s->conc, sizeof(double) * s->n); return 0; }
    if (k < 0 || k > s->nsx) return -1;
    memcpy(out, s->concx + (size_t)(k - 1) * s->n, sizeof(double) * s->n);
    return 0;
}

/* Sum over fluid cells of eps C_k for every solute k (the conserved solute
 * masses of Eq. diffusionporous), into out[nspecies]. */
int orc_species_totals(const orc_state *s, double *out)
{
    int ns = 1 + s->nsx;
    for (int k = 0; k < ns; ++k) {
        const double *C = k == 0 ? s->conc : s->concx + (size_t)(k - 1) * s->n;
        double acc = 0.0;
        for (long i = 0; i < s->n; ++i)
            if (s->type[i] == CELL_FLUID) acc += s->eps[i] * C[i];
        out[k] = acc;
    }
    return ns;
}

/* free surface: per cell class (0 gas, 1 interface, 2 liquid; solid cells 0)
 * and liquid mass m; the total excess mass that found no interface cell to
 * take it.  Returns -1 for the other physics.                             */
double orc_fs_state(const orc_state *s, unsigned char *cls, double *mass)
{
    if (s->p.physics != PHYS_FREESURF) return -1.0;
    for (long i = 0; i < s->n; ++i) {
        if (cls) cls[i] = s->type[i] == CELL_FLUID ? s->fst[i] : FS_GAS;
        if (mass) mass[i] = s->type[i] == CELL_FLUID ? s->mass[i] : 0.0;
    }
    return s->fs_lost;
}

/* free surface: replace the cell classes (0 gas, 1 interface, 2 liquid; the
 * entries of non-fluid cells are ignored), the liquid masses m and the fill
 * fractions lambda of the current state, to continue from a state exported
 * elsewhere (the populations are replaced with orc_set_state).  Gas cells
 * get zero populations and moments, as this file's own steps leave them.
 * Returns -1 for the other physics.                                        */
int orc_fs_set_state(orc_state *s, const unsigned char *cls, const double *mass, const double *lam)
{
    if (s->p.physics != PHYS_FREESURF) return -1;
    long n = s->n;
    for (long i = 0; i < n; ++i) {
        if (s->type[i] != CELL_FLUID) continue;
        s->fst[i] = cls[i];
        s->mass[i] = mass[i];
        s->lam[i] = lam[i];
        s->conc[i] = lam[i];
        if (cls[i] == FS_GAS) {
            for (int q = 0; q < NQ; ++q) s->f[s->cur][(long)q * n + i] = 0.0;
            s->rho[i] = 0.0;
            for (int a = 0; a < 3; ++a) s->vel[a * n + i] = 0.0;
        }
    }
    return 0;
}
