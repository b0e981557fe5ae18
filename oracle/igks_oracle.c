/*
 * igks_oracle.c - plain, slow FP64 CPU oracle of the implicit gas-kinetic
 * scheme (IGKS) of Pan, Zhong & Zhuo, "An Implicit Gas-Kinetic Scheme for
 * Turbulent Flow on Unstructured Hybrid Mesh" (arXiv 1709.00803).
 *
 * TEST INFRASTRUCTURE.  Only the tests, the package smoke check and the
 * benchmark's CPU-baseline leg load this library.  It shares no code,
 * header or table with the GPU library and is never called by it.
 *
 * Style: every step follows the paper's order and notation, with generic
 * building blocks (velocity-space polynomials integrated against
 * half/full Maxwellians, 4x4 moment matrices solved by Gaussian elimination
 * with partial pivoting, sequential Gauss-Seidel in cell-index order).
 * Nothing is fused, blocked or reordered for speed.
 *
 * Citations name the paper's section and equation.  Points where the paper
 * is silent, and the reading taken there, are marked "reading:".
 *
 * Threads: the per-cell and per-face loops of a residual evaluation may run
 * on several OpenMP threads (oigks_set_threads; one by default).  Each
 * thread writes only its own cells' or faces' entries, the face results are
 * summed into the cells afterwards in face order on one thread, and the
 * Gauss-Seidel sweeps stay sequential, so the results do not depend on the
 * thread count, bit for bit.
 */
#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#define EXPORT __attribute__((visibility("default")))

/* Sec. 2.1 after Eq.2: K = 3 internal degrees of freedom (2D diatomic gas);
 * gamma = (K+4)/(K+2). */
#define KDOF 3
static const double GAMMA = (KDOF + 4.0) / (KDOF + 2.0);

enum { BC_FREESTREAM = 1, BC_SYMMETRY = 2, BC_WALL = 3, BC_OUTFLOW = 4, BC_FARFIELD = 5, BC_MOVING_WALL = 6 };

/* Spalart-Allmaras constants (standard SA, "noft2" variant).  The paper
 * defers the model's constants to its Ref. (Moro et al.); reading: the
 * standard published values. */
static const double SA_CB1 = 0.1355, SA_CB2 = 0.622, SA_SIGMA = 2.0 / 3.0, SA_KAPPA = 0.41;
static const double SA_CW2 = 0.3, SA_CW3 = 2.0, SA_CV1 = 7.1;
static const double SA_C2 = 0.7, SA_C3 = 0.9; /* S-tilde clip (Allmaras 2012) */
static double sa_cw1(void) { return SA_CB1 / (SA_KAPPA * SA_KAPPA) + (1.0 + SA_CB2) / SA_SIGMA; }

/* Sutherland constant relative to the 288.15 K free stream. */
static const double SUTH_S = 110.4 / 288.15;

typedef struct {
    int limiter;        /* 0: off, 1: Eq.9 limiter */
    double cfl_init;    /* initial implicit CFL (Eq.25 start) */
    double cfl_min, cfl_max;
    int cfl_mode;       /* 0: Eq.25 (SER), 1: fixed */
    double cfl_flux;    /* delta_CFL0 of Eq.23 */
    int visc_sr;        /* viscous term in the LU-SGS spectral radius */
    int mu_law;         /* 0: Sutherland, 1: constant */
    int scheme;         /* 0: implicit LU-SGS (Eq.18-22); 1: explicit Eq.15 with local time steps */
    double wall_temp;   /* 0: adiabatic no-slip walls (Sec. 2.5); > 0: isothermal walls at this
                           multiple of the free-stream temperature */
    double limiter_freeze; /* > 0: once the density residual has dropped to this fraction of its
                              first value, the limiter factors of Eq.9 are held at their values of
                              that iteration (0: never) */
    int tau_jump;       /* 1: add dt |p_l - p_r| / (p_l + p_r) to the collision time of Eq.34 */
    int lusgs_op;       /* dissipation of the LU-SGS operator: 0 the scalar spectral radius of Eq.20
                           (lambda_ij I); 1 the first-order Roe matrix |A_ij| (Eq.18), except on
                           faces between sweep blocks, which keep lambda_ij I; 2 the same with the
                           kinetic wave magnitudes (roe_abs) */
} oigks_options;

typedef struct {
    int iteration;
    double res_l2;      /* ||M_rho||_2 of the last residual evaluation */
    double res_drop;    /* res_l2 / the largest res_l2 so far */
    double res_inf;     /* ||M||_inf over cells and the 4 flow components */
    double eq40;        /* max_i |dW_i| / |W_i| of the last update (Eq.40) */
    double cfl;         /* implicit CFL used by the last update */
    double dt_flux;     /* Eq.23 time step used inside the flux */
    double sa_l2;       /* ||R_SA||_2 */
} oigks_residual;

typedef struct oigks_ctx {
    oigks_options opt;
    char err[256];
    /* mesh */
    int nn, nc, nf, nbf;
    double *x, *y;
    int *cptr, *cnod;            /* counter-clockwise vertex lists */
    int *fL, *fR, *ftag;         /* fR = -1 on boundary faces; ftag = input tag (0 interior) */
    int *fa, *fb;                /* end nodes of each face (counter-clockwise for the owner) */
    int *fbc;                    /* boundary type in use (FARFIELD resolved) */
    int *fbidx;                  /* input boundary-edge index of a boundary face, -1 interior */
    int *wall_faces;             /* WALL faces in the order of the input boundary edges */
    double *fnx, *fny, *flen, *fxm, *fym;
    double *area, *xc, *yc, *dwall;
    int *cfp, *cff;              /* cell -> face lists */
    int *sblk;                   /* sweep block of each cell (NULL: the whole mesh is one block) */
    int block_passes;            /* 1, or 2: a second block pass with the cross-block terms of the first */
    double *dW1;                 /* the first pass's increments (two passes) */
    int nwall;                   /* number of WALL faces */
    /* flow parameters */
    int have_flow, sa;
    double mach, alpha, re, nut_ratio;
    double Winf[5], lam_inf, mu_inf, p_inf;
    /* state */
    double *W;                   /* 5 per cell, W[5*i+k]: rho, rhoU, rhoV, rhoE, nu-tilde */
    /* work arrays */
    double *M;                   /* 5 per cell: flow residual (Eq.16) and SA residual (Eq.27 rhs) */
    double *gx, *gy;             /* 4 per cell, limited gradients */
    double *ugx, *ugy;           /* 4 per cell, unlimited gradients */
    double *lamc, *vort, *dtimp;
    double *ff;                  /* 4 per face: Fbar * S, global frame, owner -> neighbour */
    double *flam;                /* per face: lambda_ij (spectral radius) */
    double *fabsA;               /* per face (lusgs_op 1): |A_ij| + lambda_visc I, 16 values row by row */
    double *Dm;                  /* per cell (lusgs_op 1): the 4x4 diagonal block of Eq.20 */
    double *D, *Dsa;
    double *dW;                  /* 5 per cell */
    double *Wg;                  /* 5 per face: ghost (cell-centre) state, boundary faces */
    double *phi;                 /* 4 per cell: the last computed limiter factors */
    double *fsa;                 /* 2 per face: the face's SA residual terms of owner and neighbour */
    double *fsag;                /* 2 per face: the magnitudes of those terms' parts (|F_inv| + |F_vis| + |F_ad|) S */
    double *sasrc;               /* per cell: Omega Sr, the SA source part of the right-hand side */
    int threads;                 /* OpenMP threads of the per-cell and per-face loops */
    int phi_frozen;              /* the limiter factors are held (limiter_freeze) */
    double dt_flux;
    /* iteration scalars */
    int iter;
    double cfl, res_inf_prev, res0;
    oigks_residual last;
} oigks_ctx;

static void seterr(oigks_ctx *c, const char *m) { snprintf(c->err, sizeof c->err, "%s", m); }

/* ======================================================================
 * Velocity-space polynomials and Maxwellian moments (Sec. 2.1, Eq.2,
 * and the slope expansion and moment relations between Eq.4 and Eq.5).
 * A polynomial is a list of monomials c * u^pu v^pv (xi^2)^px.
 * ==================================================================== */
#define PMAX 64
typedef struct { double c; int pu, pv, px; } mono;
typedef struct { int n; mono m[PMAX]; } poly;

static void p_zero(poly *p) { p->n = 0; }
static void p_add_mono(poly *p, double c, int pu, int pv, int px)
{
    for (int i = 0; i < p->n; i++)
        if (p->m[i].pu == pu && p->m[i].pv == pv && p->m[i].px == px) { p->m[i].c += c; return; }
    if (p->n >= PMAX) { fprintf(stderr, "oracle: polynomial overflow\n"); abort(); }
    p->m[p->n].c = c; p->m[p->n].pu = pu; p->m[p->n].pv = pv; p->m[p->n].px = px; p->n++;
}
static void p_mul(const poly *a, const poly *b, poly *out)
{
    poly r; p_zero(&r);
    for (int i = 0; i < a->n; i++)
        for (int j = 0; j < b->n; j++)
            p_add_mono(&r, a->m[i].c * b->m[j].c, a->m[i].pu + b->m[j].pu,
                       a->m[i].pv + b->m[j].pv, a->m[i].px + b->m[j].px);
    *out = r;
}
static void p_axpy(double s, const poly *a, poly *y)
{
    for (int i = 0; i < a->n; i++) p_add_mono(y, s * a->m[i].c, a->m[i].pu, a->m[i].pv, a->m[i].px);
}
/* collision invariants psi = (1, u, v, (u^2+v^2+xi^2)/2) (Sec. 2.1, the moment relations after Eq.4) */
static void p_psi(int i, poly *p)
{
    p_zero(p);
    if (i == 0) p_add_mono(p, 1.0, 0, 0, 0);
    else if (i == 1) p_add_mono(p, 1.0, 1, 0, 0);
    else if (i == 2) p_add_mono(p, 1.0, 0, 1, 0);
    else { p_add_mono(p, 0.5, 2, 0, 0); p_add_mono(p, 0.5, 0, 2, 0); p_add_mono(p, 0.5, 0, 0, 1); }
}
/* Taylor-coefficient form a = a1 + a2 u + a3 v + a4 (u^2+v^2+xi^2)/2 (Sec. 2.1, the
 * slope expansion after Eq.4) */
static void p_coef(const double a[4], poly *p)
{
    p_zero(p);
    p_add_mono(p, a[0], 0, 0, 0);
    p_add_mono(p, a[1], 1, 0, 0);
    p_add_mono(p, a[2], 0, 1, 0);
    p_add_mono(p, 0.5 * a[3], 2, 0, 0);
    p_add_mono(p, 0.5 * a[3], 0, 2, 0);
    p_add_mono(p, 0.5 * a[3], 0, 0, 1);
}
static void p_u(poly *p) { p_zero(p); p_add_mono(p, 1.0, 1, 0, 0); }
static void p_v(poly *p) { p_zero(p); p_add_mono(p, 1.0, 0, 1, 0); }

/* Normalised moments <u^k> of exp(-lam (u-U)^2) (sqrt(lam/pi) weight):
 * kind 0 = whole line, +1 = u > 0 half, -1 = u < 0 half.  Whole line:
 * <1> = 1, <u> = U; half lines: <1> = erfc(-/+ sqrt(lam) U)/2,
 * <u> = U<1> +/- exp(-lam U^2)/(2 sqrt(pi lam)); all: the recursion
 * <u^(k+2)> = U <u^(k+1)> + (k+1)/(2 lam) <u^k> (integration by parts). */
#define MOMN 14
typedef struct { double u[MOMN], v[MOMN], x[4]; } moms;

static void mom_line(double U, double lam, int kind, double *m)
{
    if (kind == 0) { m[0] = 1.0; m[1] = U; }
    else if (kind > 0) {
        m[0] = 0.5 * erfc(-sqrt(lam) * U);
        m[1] = U * m[0] + exp(-lam * U * U) / (2.0 * sqrt(M_PI * lam));
    } else {
        m[0] = 0.5 * erfc(sqrt(lam) * U);
        m[1] = U * m[0] - exp(-lam * U * U) / (2.0 * sqrt(M_PI * lam));
    }
    for (int k = 0; k + 2 < MOMN; k++) m[k + 2] = U * m[k + 1] + (k + 1) / (2.0 * lam) * m[k];
}
/* <(xi^2)^k> over K internal dimensions: 1, K/(2 lam), K(K+2)/(4 lam^2), ... */
static void mom_xi(double lam, double *x)
{
    x[0] = 1.0;
    for (int k = 1; k < 4; k++) x[k] = x[k - 1] * (KDOF + 2.0 * (k - 1)) / (2.0 * lam);
}
static void mk_moms(double U, double V, double lam, int ukind, moms *m)
{
    mom_line(U, lam, ukind, m->u);
    mom_line(V, lam, 0, m->v);
    mom_xi(lam, m->x);
}
/* vector <p psi>, psi = (1, u, v, (u^2 + v^2 + xi^2)/2): each monomial is
 * shifted by the exponents of the invariant it is multiplied with */
static void p_int_psi(const poly *p, const moms *m, double out[4])
{
    out[0] = out[1] = out[2] = out[3] = 0.0;
    for (int i = 0; i < p->n; i++) {
        const mono *t = &p->m[i];
        if (t->pu + 2 >= MOMN || t->pv + 2 >= MOMN || t->px + 1 >= 4) { fprintf(stderr, "oracle: moment order\n"); abort(); }
        const double *mu = m->u + t->pu, *mv = m->v + t->pv, *mx = m->x + t->px;
        out[0] += t->c * mu[0] * mv[0] * mx[0];
        out[1] += t->c * mu[1] * mv[0] * mx[0];
        out[2] += t->c * mu[0] * mv[1] * mx[0];
        out[3] += 0.5 * t->c * (mu[2] * mv[0] * mx[0] + mu[0] * mv[2] * mx[0] + mu[0] * mv[0] * mx[1]);
    }
}
/* moment matrix M_ij = <psi_i psi_j> (left side of the Sec. 2.1 moment
 * relations after Eq.4, divided by rho) */
static void moment_matrix(const moms *m, double M[16])
{
    for (int j = 0; j < 4; j++) {
        poly b; double col[4];
        p_psi(j, &b);
        p_int_psi(&b, m, col);
        for (int i = 0; i < 4; i++) M[4 * i + j] = col[i];
    }
}
/* Gaussian elimination with partial pivoting (the paper solves its moment
 * systems "by the Gaussian elimination", Sec. 2.1 after Eq.12). */
static int gauss4(const double Min[16], const double b[4], double x[4])
{
    double A[4][5];
    for (int i = 0; i < 4; i++) { for (int j = 0; j < 4; j++) A[i][j] = Min[4 * i + j]; A[i][4] = b[i]; }
    for (int k = 0; k < 4; k++) {
        int piv = k;
        for (int i = k + 1; i < 4; i++) if (fabs(A[i][k]) > fabs(A[piv][k])) piv = i;
        if (A[piv][k] == 0.0) return -1;
        if (piv != k) for (int j = 0; j < 5; j++) { double t = A[k][j]; A[k][j] = A[piv][j]; A[piv][j] = t; }
        for (int i = k + 1; i < 4; i++) {
            double f = A[i][k] / A[k][k];
            for (int j = k; j < 5; j++) A[i][j] -= f * A[k][j];
        }
    }
    for (int i = 3; i >= 0; i--) {
        double s = A[i][4];
        for (int j = i + 1; j < 4; j++) s -= A[i][j] * x[j];
        x[i] = s / A[i][i];
    }
    return 0;
}
/* Sec. 2.1 moment relations (after Eq.4): integral of g a psi = dW  ->  M(g) a = dW / rho */
static void solve_slope(const moms *full, double rho, const double dW[4], double a[4])
{
    double M[16], b[4];
    moment_matrix(full, M);
    for (int i = 0; i < 4; i++) b[i] = dW[i] / rho;
    gauss4(M, b, a);
}

/* primitive quantities of a conservative state (Eq.2: rho E = rho (U^2 + V^2
 * + (K+2)/(2 lam)) / 2) */
static double lam_of(const double W[4])
{
    double r = W[0], U = W[1] / r, V = W[2] / r;
    return (KDOF + 2.0) * r / (4.0 * (W[3] - 0.5 * r * (U * U + V * V)));
}

/* ======================================================================
 * GKS interface flux (Sec. 2.1, Eq.4-5, Eq.11-14), in the face frame
 * (x along the unit normal from the left to the right cell, y along the
 * tangent).  Inputs are the reconstructed interface states W^l, W^r, their
 * normal and tangential derivatives, the left/right cell-centre states and
 * the normal distances from the cell centres to the face.
 * ==================================================================== */
typedef struct {
    double W0[4], lam0;
    double aln[4], alt[4], arn[4], art[4];   /* a_n^l, a_t^l, a_n^r, a_t^r (Eq.4) */
    double abnl[4], abnr[4], abt[4];         /* abar_n^l, abar_n^r, abar_t (Eq.5) */
    double Al[4], Ar[4], Ab[4];              /* A^l, A^r (Eq.11), Abar (Eq.12) */
    double T[6];                             /* time integrals of the six Eq.13 factors */
    double F[4];                             /* Eq.14, integrated over [0, dt] */
} face_detail;

static void gks_core(const double Wl[4], const double Gln[4], const double Glt[4],
                     const double Wr[4], const double Grn[4], const double Grt[4],
                     const double Wlc[4], const double Wrc[4], double dl, double dr,
                     double dt, double tau, face_detail *o)
{
    double rl = Wl[0], Ul = Wl[1] / rl, Vl = Wl[2] / rl, laml = lam_of(Wl);
    double rr = Wr[0], Ur = Wr[1] / rr, Vr = Wr[2] / rr, lamr = lam_of(Wr);
    moms mlp, mrm, mlf, mrf;
    mk_moms(Ul, Vl, laml, +1, &mlp);   /* g^l on u > 0 */
    mk_moms(Ur, Vr, lamr, -1, &mrm);   /* g^r on u < 0 */
    mk_moms(Ul, Vl, laml, 0, &mlf);
    mk_moms(Ur, Vr, lamr, 0, &mrf);

    /* reading (the paper defers to Xu 2001): the interface equilibrium g0
     * carries the conservative moments of H[u] g^l + (1 - H[u]) g^r. */
    poly one; p_zero(&one); p_add_mono(&one, 1.0, 0, 0, 0);
    double sl[4], sr[4];
    p_int_psi(&one, &mlp, sl);
    p_int_psi(&one, &mrm, sr);
    for (int i = 0; i < 4; i++) o->W0[i] = rl * sl[i] + rr * sr[i];
    double r0 = o->W0[0], U0 = o->W0[1] / r0, V0 = o->W0[2] / r0, lam0 = lam_of(o->W0);
    o->lam0 = lam0;
    moms m0f, m0p, m0m;
    mk_moms(U0, V0, lam0, 0, &m0f);
    mk_moms(U0, V0, lam0, +1, &m0p);
    mk_moms(U0, V0, lam0, -1, &m0m);

    /* Eq.4 slopes from the reconstructed derivatives (the Sec. 2.1 moment relations) */
    solve_slope(&mlf, rl, Gln, o->aln);
    solve_slope(&mlf, rl, Glt, o->alt);
    solve_slope(&mrf, rr, Grn, o->arn);
    solve_slope(&mrf, rr, Grt, o->art);
    /* Eq.5 slopes of the equilibrium part.  reading: one-sided differences
     * between W0 and the two cell-centre states for abar_n^l, abar_n^r; the
     * average of the two reconstructed tangential derivatives for abar_t. */
    double d[4];
    for (int i = 0; i < 4; i++) d[i] = (o->W0[i] - Wlc[i]) / dl;
    solve_slope(&m0f, r0, d, o->abnl);
    for (int i = 0; i < 4; i++) d[i] = (Wrc[i] - o->W0[i]) / dr;
    solve_slope(&m0f, r0, d, o->abnr);
    for (int i = 0; i < 4; i++) d[i] = 0.5 * (Glt[i] + Grt[i]);
    solve_slope(&m0f, r0, d, o->abt);

    /* Eq.11: <(a_n u + a_t v + A) psi>_g = 0 on each side (whole space) */
    poly pu, pv, pa, pb, q, t1;
    p_u(&pu); p_v(&pv);
    double Ml[16], Mr[16], M0[16], rhs[4];
    moment_matrix(&mlf, Ml); moment_matrix(&mrf, Mr); moment_matrix(&m0f, M0);
    p_coef(o->aln, &pa); p_mul(&pu, &pa, &q);
    p_coef(o->alt, &pb); p_mul(&pv, &pb, &t1); p_axpy(1.0, &t1, &q);
    p_int_psi(&q, &mlf, rhs); for (int i = 0; i < 4; i++) rhs[i] = -rhs[i];
    gauss4(Ml, rhs, o->Al);
    p_coef(o->arn, &pa); p_mul(&pu, &pa, &q);
    p_coef(o->art, &pb); p_mul(&pv, &pb, &t1); p_axpy(1.0, &t1, &q);
    p_int_psi(&q, &mrf, rhs); for (int i = 0; i < 4; i++) rhs[i] = -rhs[i];
    gauss4(Mr, rhs, o->Ar);

    /* time integrals over [0, dt] of the six factors of Eq.13:
     * c1 = 1-e, c2 = tau(-1+e) + t e, c3 = t - tau + tau e, c4 = e,
     * c5 = -(t+tau) e, c6 = -tau e, with e = exp(-t/tau). */
    double eta = exp(-dt / tau), ome = -expm1(-dt / tau);   /* 1 - eta */
    o->T[0] = dt - tau * ome;
    o->T[1] = -tau * dt * (1.0 + eta) + 2.0 * tau * tau * ome;
    o->T[2] = 0.5 * dt * dt - tau * dt + tau * tau * ome;
    o->T[3] = tau * ome;
    o->T[4] = tau * dt * eta - 2.0 * tau * tau * ome;
    o->T[5] = -tau * tau * ome;

    /* Eq.12: the integral over [0, dt] of psi (f - g) vanishes, with
     * g = g0 (1 + Abar t) at the interface.  The g0 terms of f integrate to
     * (T1 + T4) W0 = dt W0, cancelling dt W0 from g, which leaves
     * T2 Q2 + T3 rho0 M0 Abar + T5 Q5 + T6 Q6 = (dt^2/2) rho0 M0 Abar. */
    double Q2[4], Q5[4], Q6[4], a[4], b[4], cc[4];
    p_coef(o->abnl, &pa); p_mul(&pu, &pa, &q); p_int_psi(&q, &m0p, a);
    p_coef(o->abnr, &pa); p_mul(&pu, &pa, &q); p_int_psi(&q, &m0m, b);
    p_coef(o->abt, &pa); p_mul(&pv, &pa, &q); p_int_psi(&q, &m0f, cc);
    for (int i = 0; i < 4; i++) Q2[i] = r0 * (a[i] + b[i] + cc[i]);
    p_coef(o->aln, &pa); p_mul(&pu, &pa, &q); p_coef(o->alt, &pb); p_mul(&pv, &pb, &t1); p_axpy(1.0, &t1, &q);
    p_int_psi(&q, &mlp, a);
    p_coef(o->arn, &pa); p_mul(&pu, &pa, &q); p_coef(o->art, &pb); p_mul(&pv, &pb, &t1); p_axpy(1.0, &t1, &q);
    p_int_psi(&q, &mrm, b);
    for (int i = 0; i < 4; i++) Q5[i] = rl * a[i] + rr * b[i];
    p_coef(o->Al, &pa); p_int_psi(&pa, &mlp, a);
    p_coef(o->Ar, &pa); p_int_psi(&pa, &mrm, b);
    for (int i = 0; i < 4; i++) Q6[i] = rl * a[i] + rr * b[i];
    double lhs = 0.5 * dt * dt - o->T[2];
    double MA[16];
    for (int i = 0; i < 16; i++) MA[i] = r0 * M0[i] * lhs;
    for (int i = 0; i < 4; i++) rhs[i] = o->T[1] * Q2[i] + o->T[4] * Q5[i] + o->T[5] * Q6[i];
    gauss4(MA, rhs, o->Ab);

    /* Eq.14: F = integral over [0, dt] and velocity space of u psi f_cf,
     * with f_cf from Eq.13 term by term. */
    double F[4] = {0, 0, 0, 0}, v4[4], w4[4];
    /* c1 g0 */
    p_int_psi(&pu, &m0f, v4);
    for (int i = 0; i < 4; i++) F[i] += o->T[0] * r0 * v4[i];
    /* c2 ((abar_n^l H + abar_n^r (1-H)) u + abar_t v) g0 */
    p_coef(o->abnl, &pa); p_mul(&pu, &pa, &q); p_mul(&pu, &q, &t1); p_int_psi(&t1, &m0p, v4);
    p_coef(o->abnr, &pa); p_mul(&pu, &pa, &q); p_mul(&pu, &q, &t1); p_int_psi(&t1, &m0m, w4);
    for (int i = 0; i < 4; i++) F[i] += o->T[1] * r0 * (v4[i] + w4[i]);
    p_coef(o->abt, &pa); p_mul(&pv, &pa, &q); p_mul(&pu, &q, &t1); p_int_psi(&t1, &m0f, v4);
    for (int i = 0; i < 4; i++) F[i] += o->T[1] * r0 * v4[i];
    /* c3 Abar g0 */
    p_coef(o->Ab, &pa); p_mul(&pu, &pa, &q); p_int_psi(&q, &m0f, v4);
    for (int i = 0; i < 4; i++) F[i] += o->T[2] * r0 * v4[i];
    /* c4 (H g^l + (1-H) g^r) */
    p_int_psi(&pu, &mlp, v4); p_int_psi(&pu, &mrm, w4);
    for (int i = 0; i < 4; i++) F[i] += o->T[3] * (rl * v4[i] + rr * w4[i]);
    /* c5 ((u a_n^l + v a_t^l) H g^l + (u a_n^r + v a_t^r)(1-H) g^r) */
    p_coef(o->aln, &pa); p_mul(&pu, &pa, &q); p_coef(o->alt, &pb); p_mul(&pv, &pb, &t1); p_axpy(1.0, &t1, &q);
    p_mul(&pu, &q, &t1); p_int_psi(&t1, &mlp, v4);
    p_coef(o->arn, &pa); p_mul(&pu, &pa, &q); p_coef(o->art, &pb); p_mul(&pv, &pb, &t1); p_axpy(1.0, &t1, &q);
    p_mul(&pu, &q, &t1); p_int_psi(&t1, &mrm, w4);
    for (int i = 0; i < 4; i++) F[i] += o->T[4] * (rl * v4[i] + rr * w4[i]);
    /* c6 (A^l H g^l + A^r (1-H) g^r) */
    p_coef(o->Al, &pa); p_mul(&pu, &pa, &q); p_int_psi(&q, &mlp, v4);
    p_coef(o->Ar, &pa); p_mul(&pu, &pa, &q); p_int_psi(&q, &mrm, w4);
    for (int i = 0; i < 4; i++) F[i] += o->T[5] * (rl * v4[i] + rr * w4[i]);
    for (int i = 0; i < 4; i++) o->F[i] = F[i];
}

/* ======================================================================
 * Viscosity, collision time (Eq.33-34) and the SA model (Eq.26-32)
 * ==================================================================== */
static double mu_lam(const oigks_ctx *c, double lam)
{
    if (c->opt.mu_law == 1) return c->mu_inf;
    double th = c->lam_inf / lam;   /* T / T_inf (Eq.2: lam = m / (2 R T)) */
    return c->mu_inf * pow(th, 1.5) * (1.0 + SUTH_S) / (th + SUTH_S);
}
static double sa_fv1(double chi) { double c3 = chi * chi * chi; return c3 / (c3 + SA_CV1 * SA_CV1 * SA_CV1); }

/* Eq.34: tau = (mu_l + mu_t) / p at the interface equilibrium state, with
 * mu_t = rho nu_t = rho nu-tilde f_v1.  reading: nu-tilde at the face is the
 * average of the two cell-centre values, clipped at zero. */
static double collision_time(const oigks_ctx *c, double rho0, double lam0, double nut_f)
{
    double mul = mu_lam(c, lam0), mut = 0.0;
    if (c->sa && nut_f > 0.0) mut = rho0 * nut_f * sa_fv1(nut_f * rho0 / mul);
    double p0 = rho0 / (2.0 * lam0);
    return (mul + mut) / p0;
}

/* Eq.28a source S_r = c_b1 S~ nu~ - c_w1 f_w (nu~/d)^2 and the pieces the
 * implicit diagonal of Eq.32 uses.  out: Sr, S~, f_w, max(0, -dSr/dnu~). */
static void sa_source(double nut, double nu, double d, double omega, double out[4])
{
    double k2d2 = SA_KAPPA * SA_KAPPA * d * d;
    double chi = nut / nu;
    double fv1 = sa_fv1(chi);
    double fv2 = 1.0 - chi / (1.0 + chi * fv1);
    double Sb = nut * fv2 / k2d2;
    double St;
    if (Sb >= -SA_C2 * omega) St = omega + Sb;
    else St = omega + omega * (SA_C2 * SA_C2 * omega + SA_C3 * Sb) / ((SA_C3 - 2.0 * SA_C2) * omega - Sb);
    double r = (St > 0.0) ? nut / (St * k2d2) : 10.0;
    if (r > 10.0) r = 10.0;
    double g = r + SA_CW2 * (pow(r, 6) - r);
    double c6 = pow(SA_CW3, 6);
    double fw = g * pow((1.0 + c6) / (pow(g, 6) + c6), 1.0 / 6.0);
    double cw1 = sa_cw1();
    out[0] = SA_CB1 * St * nut - cw1 * fw * (nut / d) * (nut / d);
    out[1] = St;
    out[2] = fw;
    double jd = 2.0 * cw1 * fw * nut / (d * d) - SA_CB1 * St;
    out[3] = jd > 0.0 ? jd : 0.0;
}

/* ======================================================================
 * Mesh ingest (Sec. 2.4: node coordinates + per-cell vertex lists) and
 * geometry; ghost cells per the ghost-cell method (Sec. 2.5).
 * ==================================================================== */
typedef struct { long long key; int cell, loc; } edge_rec;
static int cmp_edge(const void *a, const void *b)
{
    const edge_rec *x = a, *y = b;
    if (x->key != y->key) return x->key < y->key ? -1 : 1;
    if (x->cell != y->cell) return x->cell < y->cell ? -1 : 1;
    return x->loc - y->loc;
}
typedef struct { long long key; int idx; } bkey;
static int cmp_bkey(const void *a, const void *b)
{
    const bkey *x = a, *y = b;
    return x->key < y->key ? -1 : (x->key > y->key ? 1 : 0);
}

static void free_mesh(oigks_ctx *c)
{
    void *ps[] = {c->x, c->y, c->cptr, c->cnod, c->fL, c->fR, c->ftag, c->fa, c->fb, c->fbc, c->fbidx, c->wall_faces, c->fnx, c->fny, c->flen,
                  c->fxm, c->fym, c->area, c->xc, c->yc, c->dwall, c->cfp, c->cff, c->W, c->M, c->gx,
                  c->gy, c->ugx, c->ugy, c->lamc, c->vort, c->dtimp, c->ff, c->flam, c->D, c->Dsa,
                  c->dW, c->Wg, c->phi, c->fsa, c->fsag, c->sasrc, c->fabsA, c->Dm};
    for (size_t i = 0; i < sizeof ps / sizeof ps[0]; i++) free(ps[i]);
    free(c->sblk);
    c->sblk = NULL;
    free(c->dW1);
    c->dW1 = NULL;
    c->x = c->y = NULL; c->cptr = c->cnod = NULL; c->fa = c->fb = NULL; c->fL = c->fR = c->ftag = c->fbc = c->fbidx = c->wall_faces = NULL;
    c->fnx = c->fny = c->flen = c->fxm = c->fym = NULL; c->area = c->xc = c->yc = c->dwall = NULL;
    c->cfp = c->cff = NULL; c->W = c->M = c->gx = c->gy = c->ugx = c->ugy = NULL;
    c->lamc = c->vort = c->dtimp = c->ff = c->flam = c->D = c->Dsa = c->dW = c->Wg = c->phi = c->fsa = NULL;
    c->fsag = c->sasrc = c->fabsA = c->Dm = NULL;
}

EXPORT void oigks_default_options(oigks_options *o)
{
    o->limiter = 0; o->cfl_init = 1000.0; o->cfl_min = 1.0; o->cfl_max = 1e6; o->cfl_mode = 0; o->scheme = 0;
    o->cfl_flux = 1.0; o->visc_sr = 1; o->mu_law = 0; o->wall_temp = 0.0; o->limiter_freeze = 0.0; o->tau_jump = 0;
    o->lusgs_op = 0;
}

EXPORT int oigks_create(oigks_ctx **out, const oigks_options *opt)
{
    oigks_ctx *c = calloc(1, sizeof *c);
    if (!c) return -3;
    if (opt) c->opt = *opt; else oigks_default_options(&c->opt);
    c->threads = 1;
    *out = c;
    if (!(c->opt.wall_temp >= 0.0) || !isfinite(c->opt.wall_temp)) { seterr(c, "wall_temp must be >= 0"); return -1; }
    if (c->opt.tau_jump < 0 || c->opt.tau_jump > 1) { seterr(c, "tau_jump must be 0 or 1"); return -1; }
    if (c->opt.lusgs_op < 0 || c->opt.lusgs_op > 2) { seterr(c, "lusgs_op must be 0, 1 or 2"); return -1; }
    if (!(c->opt.limiter_freeze >= 0.0) || !(c->opt.limiter_freeze < 1.0)) {
        seterr(c, "limiter_freeze must be in [0, 1)");
        return -1;
    }
    return 0;
}
EXPORT void oigks_destroy(oigks_ctx *c) { if (c) { free_mesh(c); free(c); } }
EXPORT const char *oigks_last_error(const oigks_ctx *c) { return c ? c->err : "null context"; }

/* point-to-segment distance */
static double seg_dist(double px, double py, double ax, double ay, double bx, double by)
{
    double ex = bx - ax, ey = by - ay, t = ((px - ax) * ex + (py - ay) * ey) / (ex * ex + ey * ey);
    if (t < 0) t = 0; if (t > 1) t = 1;
    double dx = px - ax - t * ex, dy = py - ay - t * ey;
    return sqrt(dx * dx + dy * dy);
}

EXPORT int oigks_mesh_upload(oigks_ctx *c, int n_nodes, const double *xy, int n_cells,
                             const int *cell_ptr, const int *cell_nodes, int n_bfaces,
                             const int *bface_nodes, const int *bface_tag)
{
    free_mesh(c);
    c->have_flow = 0;
    c->nn = n_nodes; c->nc = n_cells;
    c->x = malloc(sizeof(double) * n_nodes); c->y = malloc(sizeof(double) * n_nodes);
    for (int i = 0; i < n_nodes; i++) { c->x[i] = xy[2 * i]; c->y[i] = xy[2 * i + 1]; }
    c->cptr = malloc(sizeof(int) * (n_cells + 1));
    memcpy(c->cptr, cell_ptr, sizeof(int) * (n_cells + 1));
    int nv = cell_ptr[n_cells];
    c->cnod = malloc(sizeof(int) * nv);
    memcpy(c->cnod, cell_nodes, sizeof(int) * nv);
    /* orient counter-clockwise, area and area centroid (shoelace) */
    c->area = malloc(sizeof(double) * n_cells); c->xc = malloc(sizeof(double) * n_cells);
    c->yc = malloc(sizeof(double) * n_cells);
    for (int i = 0; i < n_cells; i++) {
        int p0 = c->cptr[i], k = c->cptr[i + 1] - p0;
        if (k < 3) { seterr(c, "cell with fewer than 3 nodes"); return -2; }
        /* shoelace area and area centroid, with coordinates taken relative
         * to the cell's first vertex (the same formula; it keeps small cells
         * far from the origin free of cancellation) */
        double a = 0, sx = 0, sy = 0;
        double ox = c->x[c->cnod[p0]], oy = c->y[c->cnod[p0]];
        for (int j = 0; j < k; j++) {
            int n1 = c->cnod[p0 + j], n2 = c->cnod[p0 + (j + 1) % k];
            double x1 = c->x[n1] - ox, y1 = c->y[n1] - oy, x2 = c->x[n2] - ox, y2 = c->y[n2] - oy;
            double cr = x1 * y2 - x2 * y1;
            a += cr; sx += (x1 + x2) * cr; sy += (y1 + y2) * cr;
        }
        if (a < 0) {   /* reverse */
            for (int j = 0; j < k / 2; j++) { int t = c->cnod[p0 + j]; c->cnod[p0 + j] = c->cnod[p0 + k - 1 - j]; c->cnod[p0 + k - 1 - j] = t; }
            a = -a; sx = -sx; sy = -sy;
        }
        if (!(a > 0)) { seterr(c, "degenerate cell"); return -2; }
        c->area[i] = 0.5 * a; c->xc[i] = ox + sx / (3.0 * a); c->yc[i] = oy + sy / (3.0 * a);
        /* convexity (Sec. 2.4 cells are convex polygons; reading: a vertex
         * where the counter-clockwise boundary turns clockwise by more than
         * asin(0.1), about 5.7 degrees, makes the cell non-convex, while the
         * slight reflex turn of a hanging node on a curved edge is accepted),
         * and every face must see the centroid on its inner side, since the
         * centroid-to-face distance d of Eq.5 divides */
        for (int j = 0; j < k; j++) {
            int nm = c->cnod[p0 + (j + k - 1) % k], n0 = c->cnod[p0 + j], np = c->cnod[p0 + (j + 1) % k];
            double e1x = c->x[n0] - c->x[nm], e1y = c->y[n0] - c->y[nm];
            double e2x = c->x[np] - c->x[n0], e2y = c->y[np] - c->y[n0];
            double turn = (e1x * e2y - e1y * e2x) / (sqrt(e1x * e1x + e1y * e1y) * sqrt(e2x * e2x + e2y * e2y));
            if (!(turn >= -0.1)) { seterr(c, "non-convex cell"); return -2; }
            double ax = c->x[n0] - c->xc[i], ay = c->y[n0] - c->yc[i];
            double bx = c->x[np] - c->xc[i], by = c->y[np] - c->yc[i];
            if (!(ax * by - ay * bx > 0)) { seterr(c, "cell centroid outside a face's half plane"); return -2; }
        }
    }
    /* edges: sort (min node, max node) keys and pair them */
    edge_rec *E = malloc(sizeof(edge_rec) * nv);
    for (int i = 0; i < n_cells; i++) {
        int p0 = c->cptr[i], k = c->cptr[i + 1] - p0;
        for (int j = 0; j < k; j++) {
            int a = c->cnod[p0 + j], b = c->cnod[p0 + (j + 1) % k];
            long long lo = a < b ? a : b, hi = a < b ? b : a;
            E[p0 + j].key = lo * (long long)(n_nodes + 1) + hi; E[p0 + j].cell = i; E[p0 + j].loc = j;
        }
    }
    qsort(E, nv, sizeof(edge_rec), cmp_edge);
    int nf = 0;
    for (int i = 0; i < nv;) {
        int j = i + 1;
        while (j < nv && E[j].key == E[i].key) j++;
        if (j - i > 2) { free(E); seterr(c, "edge shared by more than two cells"); return -2; }
        nf++; i = j;
    }
    c->nf = nf;
    c->fL = malloc(sizeof(int) * nf); c->fR = malloc(sizeof(int) * nf); c->ftag = calloc(nf, sizeof(int));
    c->fa = malloc(sizeof(int) * nf); c->fb = malloc(sizeof(int) * nf);
    c->fbc = calloc(nf, sizeof(int));
    c->fbidx = malloc(sizeof(int) * nf);
    c->fnx = malloc(sizeof(double) * nf); c->fny = malloc(sizeof(double) * nf);
    c->flen = malloc(sizeof(double) * nf); c->fxm = malloc(sizeof(double) * nf); c->fym = malloc(sizeof(double) * nf);
    bkey *BK = malloc(sizeof(bkey) * (n_bfaces > 0 ? n_bfaces : 1));
    for (int b = 0; b < n_bfaces; b++) {
        long long a = bface_nodes[2 * b], d = bface_nodes[2 * b + 1];
        long long lo = a < d ? a : d, hi = a < d ? d : a;
        BK[b].key = lo * (long long)(n_nodes + 1) + hi; BK[b].idx = b;
    }
    qsort(BK, n_bfaces, sizeof(bkey), cmp_bkey);
    int *bused = calloc(n_bfaces > 0 ? n_bfaces : 1, sizeof(int));
    int f = 0, nbf = 0, nwall = 0;
    for (int i = 0; i < nv;) {
        int j = i + 1;
        while (j < nv && E[j].key == E[i].key) j++;
        /* owner = the lower cell index; the normal points owner -> neighbour */
        int ow = E[i].cell, lo_ = E[i].loc;
        int p0 = c->cptr[ow], k = c->cptr[ow + 1] - p0;
        int a = c->cnod[p0 + lo_], b = c->cnod[p0 + (lo_ + 1) % k];
        double dx = c->x[b] - c->x[a], dy = c->y[b] - c->y[a], L = sqrt(dx * dx + dy * dy);
        c->fL[f] = ow;
        c->fa[f] = a; c->fb[f] = b;
        c->fbidx[f] = -1;
        c->fnx[f] = dy / L; c->fny[f] = -dx / L; c->flen[f] = L;   /* outward normal of a CCW edge */
        c->fxm[f] = 0.5 * (c->x[a] + c->x[b]); c->fym[f] = 0.5 * (c->y[a] + c->y[b]);
        if (j - i == 2) {
            c->fR[f] = E[i + 1].cell;
        } else {
            c->fR[f] = -1; nbf++;
            bkey q = {E[i].key, 0};
            bkey *hit = bsearch(&q, BK, n_bfaces, sizeof(bkey), cmp_bkey);
            if (!hit) { free(E); free(BK); free(bused); seterr(c, "unmatched boundary edge"); return -2; }
            int tag = bface_tag[hit->idx];
            if (tag < 1 || tag > 6) { free(E); free(BK); free(bused); seterr(c, "bad boundary tag"); return -2; }
            c->ftag[f] = tag; bused[hit - BK] = 1; c->fbidx[f] = hit->idx;
            if (tag == BC_WALL) nwall++;
        }
        f++; i = j;
    }
    for (int b = 0; b < n_bfaces; b++)
        if (!bused[b]) { free(E); free(BK); free(bused); seterr(c, "boundary edge not on the mesh boundary"); return -2; }
    free(E); free(BK); free(bused);
    c->nbf = nbf; c->nwall = nwall;
    {   /* wall faces ordered by their input boundary-edge index */
        int *slot = malloc(sizeof(int) * (n_bfaces > 0 ? n_bfaces : 1));
        for (int b = 0; b < n_bfaces; b++) slot[b] = -1;
        for (int q = 0; q < nf; q++) if (c->ftag[q] == BC_WALL) slot[c->fbidx[q]] = q;
        c->wall_faces = malloc(sizeof(int) * (nwall > 0 ? nwall : 1));
        int w = 0;
        for (int b = 0; b < n_bfaces; b++) if (slot[b] >= 0) c->wall_faces[w++] = slot[b];
        free(slot);
    }
    /* cell -> face lists */
    c->cfp = calloc(n_cells + 1, sizeof(int));
    for (int q = 0; q < nf; q++) { c->cfp[c->fL[q] + 1]++; if (c->fR[q] >= 0) c->cfp[c->fR[q] + 1]++; }
    for (int i = 0; i < n_cells; i++) c->cfp[i + 1] += c->cfp[i];
    c->cff = malloc(sizeof(int) * c->cfp[n_cells]);
    int *fill = calloc(n_cells, sizeof(int));
    for (int q = 0; q < nf; q++) {
        c->cff[c->cfp[c->fL[q]] + fill[c->fL[q]]++] = q;
        if (c->fR[q] >= 0) c->cff[c->cfp[c->fR[q]] + fill[c->fR[q]]++] = q;
    }
    free(fill);
    /* wall distance: exact distance from each centroid to the closest wall
     * edge, the segment between the edge's two nodes */
    c->dwall = malloc(sizeof(double) * n_cells);
#pragma omp parallel for num_threads(c->threads) schedule(static)
    for (int i = 0; i < n_cells; i++) {
        double best = 1e300;
        for (int w = 0; w < c->nwall; w++) {
            int q = c->wall_faces[w];
            double dd = seg_dist(c->xc[i], c->yc[i], c->x[c->fa[q]], c->y[c->fa[q]], c->x[c->fb[q]], c->y[c->fb[q]]);
            if (dd < best) best = dd;
        }
        c->dwall[i] = best;
    }
    int n4 = 4 * n_cells;
    c->W = calloc(5 * n_cells, sizeof(double)); c->M = calloc(5 * n_cells, sizeof(double));
    c->gx = calloc(n4, sizeof(double)); c->gy = calloc(n4, sizeof(double));
    c->ugx = calloc(n4, sizeof(double)); c->ugy = calloc(n4, sizeof(double));
    c->lamc = calloc(n_cells, sizeof(double)); c->vort = calloc(n_cells, sizeof(double));
    c->dtimp = calloc(n_cells, sizeof(double));
    c->ff = calloc(4 * nf, sizeof(double)); c->flam = calloc(nf, sizeof(double));
    if (c->opt.lusgs_op) { c->fabsA = calloc(16 * (size_t)nf, sizeof(double)); c->Dm = calloc(16 * (size_t)n_cells, sizeof(double)); }
    c->D = calloc(n_cells, sizeof(double)); c->Dsa = calloc(n_cells, sizeof(double));
    c->dW = calloc(5 * n_cells, sizeof(double)); c->Wg = calloc(5 * nf, sizeof(double));
    c->phi = calloc(n4, sizeof(double));
    c->fsa = calloc(2 * nf, sizeof(double));
    c->fsag = calloc(2 * nf, sizeof(double));
    c->sasrc = calloc(n_cells, sizeof(double));
    return 0;
}

/* ======================================================================
 * Boundary conditions (Sec. 2.5): ghost values and ghost increments
 * ==================================================================== */
/* Cell-centre ghost of an isothermal no-slip wall (reading): the interior
 * pressure, the temperature mirrored about the wall's, RT_g = 2 RT_w - RT_i
 * (at least RT_w / 2), the no-slip ghost velocity (ux, uy), nu-tilde
 * negated.  It serves the least-squares stencil, the limiter bounds, the
 * spectral radius and the SA face terms; the face flux reflects the
 * interior states instead (see residual()). */
static void iso_ghost(const oigks_ctx *c, const double *Wi, double ux, double uy, double *Wg)
{
    const double tw = c->opt.wall_temp * c->p_inf / c->Winf[0];
    const double r = Wi[0];
    const double p = (GAMMA - 1.0) * (Wi[3] - 0.5 * (Wi[1] * Wi[1] + Wi[2] * Wi[2]) / r);
    double tg = 2.0 * tw - p / r;
    if (tg < 0.5 * tw) tg = 0.5 * tw;
    const double rg = p / tg;
    Wg[0] = rg;
    Wg[1] = rg * ux;
    Wg[2] = rg * uy;
    Wg[3] = p / (GAMMA - 1.0) + 0.5 * rg * (ux * ux + uy * uy);
    Wg[4] = -Wi[4];
}

static void ghost_state(const oigks_ctx *c, int bc, const double *Wi, double nx, double ny, double *Wg)
{
    if (bc == BC_FREESTREAM) { for (int k = 0; k < 5; k++) Wg[k] = c->Winf[k]; return; }
    double r = Wi[0], mx = Wi[1], my = Wi[2];
    if (bc == BC_SYMMETRY) {            /* (rho V_n)_-1 = -(rho V_n)_1, others copied */
        double mn = mx * nx + my * ny;
        Wg[0] = r; Wg[1] = mx - 2.0 * mn * nx; Wg[2] = my - 2.0 * mn * ny; Wg[3] = Wi[3]; Wg[4] = Wi[4];
        return;
    }
    if (bc == BC_WALL && c->opt.wall_temp > 0.0) { iso_ghost(c, Wi, -mx / r, -my / r, Wg); return; }
    if (bc == BC_WALL) {                /* momentum and nu-tilde negated */
        Wg[0] = r; Wg[1] = -mx; Wg[2] = -my; Wg[3] = Wi[3]; Wg[4] = -Wi[4];
        return;
    }
    if (bc == BC_MOVING_WALL) {
        /* reading: a no-slip wall moving with the tangential part V_w of the
         * free-stream velocity.  The ghost keeps the interior density and
         * temperature and takes the velocity 2 V_w - V_i, so that the face
         * average is V_w; V_w = 0 gives the rule above. */
        double tx = -ny, ty = nx, vt = (c->Winf[1] * tx + c->Winf[2] * ty) / c->Winf[0];
        double vwx = vt * tx, vwy = vt * ty;
        if (c->opt.wall_temp > 0.0) { iso_ghost(c, Wi, 2.0 * vwx - mx / r, 2.0 * vwy - my / r, Wg); return; }
        Wg[0] = r;
        Wg[1] = 2.0 * vwx * r - mx;
        Wg[2] = 2.0 * vwy * r - my;
        Wg[3] = Wi[3] + 2.0 * r * (vwx * vwx + vwy * vwy) - 2.0 * (vwx * mx + vwy * my);
        Wg[4] = -Wi[4];
        return;
    }
    /* BC_OUTFLOW: Riemann invariants R+ (inside) and R- (free stream) along
     * the outward normal; U_b = (R+ + R-)/2, rho_b = rho_i, (rho E)_b from
     * U_b, the inside tangential velocity and lam_i; nu-tilde copied.
     * reading: the printed c_b is never used by the rule for rho_b and
     * (rho E)_b, so it is not needed; the rule is applied for either sign
     * of U_b (a switch to the free-stream state on backflow would make the
     * residual discontinuous). */
    double U = mx / r, V = my / r, lam = lam_of(Wi);
    double ci = sqrt(GAMMA / (2.0 * lam));
    double Ui = U * nx + V * ny;
    double Uo = (c->Winf[1] * nx + c->Winf[2] * ny) / c->Winf[0];
    double co = sqrt(GAMMA / (2.0 * c->lam_inf));
    double Rp = Ui + 2.0 * ci / (GAMMA - 1.0), Rm = Uo - 2.0 * co / (GAMMA - 1.0);
    double Ub = 0.5 * (Rp + Rm);
    double Vt = -U * ny + V * nx;
    Wg[0] = r;
    Wg[1] = r * (Ub * nx - Vt * ny);
    Wg[2] = r * (Ub * ny + Vt * nx);
    Wg[3] = 0.5 * r * (Ub * Ub + Vt * Vt + (KDOF + 2.0) / (2.0 * lam));
    Wg[4] = Wi[4];
}
/* increments of the ghost values for the implicit sweep (Sec. 2.5) */
static void ghost_incr(const oigks_ctx *c, int bc, const double *dWi, double nx, double ny, double *dWg)
{
    if (bc == BC_MOVING_WALL) {         /* the linear map of the moving-wall ghost state */
        double tx = -ny, ty = nx, vt = (c->Winf[1] * tx + c->Winf[2] * ty) / c->Winf[0];
        double vwx = vt * tx, vwy = vt * ty;
        dWg[0] = dWi[0];
        dWg[1] = 2.0 * vwx * dWi[0] - dWi[1];
        dWg[2] = 2.0 * vwy * dWi[0] - dWi[2];
        dWg[3] = dWi[3] + 2.0 * (vwx * vwx + vwy * vwy) * dWi[0] - 2.0 * (vwx * dWi[1] + vwy * dWi[2]);
        dWg[4] = -dWi[4];
        return;
    }
    if (bc == BC_SYMMETRY) {
        double mn = dWi[1] * nx + dWi[2] * ny;
        dWg[0] = dWi[0]; dWg[1] = dWi[1] - 2.0 * mn * nx; dWg[2] = dWi[2] - 2.0 * mn * ny;
        dWg[3] = dWi[3]; dWg[4] = dWi[4];
    } else if (bc == BC_WALL) {
        dWg[0] = dWi[0]; dWg[1] = -dWi[1]; dWg[2] = -dWi[2]; dWg[3] = dWi[3]; dWg[4] = -dWi[4];
    } else {
        for (int k = 0; k < 5; k++) dWg[k] = 0.0;
    }
}

EXPORT int oigks_set_freestream(oigks_ctx *c, double mach, double alpha_deg, double reynolds, double nut_ratio)
{
    if (!c->cptr) { seterr(c, "no mesh"); return -1; }
    if (!(mach > 0) || !(reynolds > 0)) { seterr(c, "mach and reynolds must be positive"); return -1; }
    c->mach = mach; c->alpha = alpha_deg * M_PI / 180.0; c->re = reynolds; c->nut_ratio = nut_ratio;
    c->sa = nut_ratio >= 0.0;
    /* non-dimensionalisation: rho_inf = 1, |V_inf| = 1, reference length 1 */
    c->p_inf = 1.0 / (GAMMA * mach * mach);
    c->lam_inf = 1.0 / (2.0 * c->p_inf);
    c->mu_inf = 1.0 / reynolds;
    c->Winf[0] = 1.0; c->Winf[1] = cos(c->alpha); c->Winf[2] = sin(c->alpha);
    c->Winf[3] = c->p_inf / (GAMMA - 1.0) + 0.5;
    c->Winf[4] = c->sa ? nut_ratio * c->mu_inf : 0.0;
    for (int f = 0; f < c->nf; f++) {
        int t = c->ftag[f];
        if (t == BC_FARFIELD) t = (c->Winf[1] * c->fnx[f] + c->Winf[2] * c->fny[f] < 0.0) ? BC_FREESTREAM : BC_OUTFLOW;
        c->fbc[f] = t;
    }
    for (int i = 0; i < c->nc; i++) for (int k = 0; k < 5; k++) c->W[5 * i + k] = c->Winf[k];
    c->iter = 0; c->cfl = c->opt.cfl_init; c->res_inf_prev = 0.0; c->res0 = 0.0;
    c->phi_frozen = 0;
    memset(&c->last, 0, sizeof c->last);
    c->have_flow = 1;
    return 0;
}

/* ghost centroid: the owner centroid reflected in the face line */
static void ghost_centroid(const oigks_ctx *c, int f, double *gx, double *gy)
{
    int i = c->fL[f];
    double dn = (c->fxm[f] - c->xc[i]) * c->fnx[f] + (c->fym[f] - c->yc[i]) * c->fny[f];
    *gx = c->xc[i] + 2.0 * dn * c->fnx[f];
    *gy = c->yc[i] + 2.0 * dn * c->fny[f];
}

/* ======================================================================
 * Residual evaluation: Eq.6-10 (reconstruction), Eq.14 (flux), Eq.16
 * (residual M), Eq.21/23 (spectral radius and dt), Eq.27-30 (SA).
 * ==================================================================== */
static double sound(const double *W) { return sqrt(GAMMA / (2.0 * lam_of(W))); }

/* Entropy fix of the Roe dissipation (reading: the paper gives none): each
 * eigenvalue's magnitude is held at least at this fraction of the
 * Roe-averaged sound speed. */
static const double ROE_DELTA = 0.1;

/* |A| = R |Lambda| L of the Euler flux Jacobian in direction n at the Roe
 * average of the states Wl, Wr (the first-order Roe scheme's dissipation
 * matrix, Eq.18), plus vis times the identity (the viscous part of the
 * spectral radius).  Written out as the product of the right eigenvectors,
 * the eigenvalue magnitudes and the left eigenvectors of the conservative
 * variables (rho, rho u, rho v, rho E).  The magnitudes of the eigenvalues
 * s = q - c, q, q, q + c: kin 0, |s| limited below by ROE_DELTA c; kin 1
 * (reading: the dissipation a wave of speed s gets when its particles'
 * normal velocities spread as a Maxwellian of temperature RT = c^2 / gamma
 * about s and are split by sign at the interface, as in the collisionless
 * part of the kinetic flux, Eq.13 with tau >> dt), the mean of |u| for
 * u ~ N(s, RT): s erf(s / sqrt(2RT)) + sqrt(2RT / pi) exp(-s^2 / (2RT)),
 * which is at least |s| and sqrt(2RT / pi) at s = 0. */
static void roe_abs(const double *Wl, const double *Wr, double nx, double ny, double vis, int kin, double *A)
{
    const double b = GAMMA - 1.0;
    double rl = Wl[0], rr = Wr[0];
    double ul = Wl[1] / rl, vl = Wl[2] / rl, ur = Wr[1] / rr, vr = Wr[2] / rr;
    double pl = b * (Wl[3] - 0.5 * rl * (ul * ul + vl * vl)), pr = b * (Wr[3] - 0.5 * rr * (ur * ur + vr * vr));
    double Hl = (Wl[3] + pl) / rl, Hr = (Wr[3] + pr) / rr;
    double sl = sqrt(rl), sr = sqrt(rr);
    double u = (sl * ul + sr * ur) / (sl + sr), v = (sl * vl + sr * vr) / (sl + sr), H = (sl * Hl + sr * Hr) / (sl + sr);
    double k = 0.5 * (u * u + v * v), c2 = b * (H - k), c = sqrt(c2);
    double q = u * nx + v * ny, qt = -u * ny + v * nx;
    double lm[4] = {q - c, q, q, q + c};
    const double rt2 = 2.0 * c2 / GAMMA;   /* 2RT */
    for (int m = 0; m < 4; m++) {
        const double sv = lm[m];
        if (kin) lm[m] = sv * erf(sv / sqrt(rt2)) + sqrt(rt2 / M_PI) * exp(-sv * sv / rt2);
        else lm[m] = fabs(sv) < ROE_DELTA * c ? ROE_DELTA * c : fabs(sv);
    }
    double R[4][4] = {{1.0, 1.0, 0.0, 1.0},
                      {u - c * nx, u, -ny, u + c * nx},
                      {v - c * ny, v, nx, v + c * ny},
                      {H - q * c, k, qt, H + q * c}};
    double L[4][4] = {{0.5 * (b * k / c2 + q / c), -0.5 * (b * u / c2 + nx / c), -0.5 * (b * v / c2 + ny / c), 0.5 * b / c2},
                      {1.0 - b * k / c2, b * u / c2, b * v / c2, -b / c2},
                      {-qt, -ny, nx, 0.0},
                      {0.5 * (b * k / c2 - q / c), -0.5 * (b * u / c2 - nx / c), -0.5 * (b * v / c2 - ny / c), 0.5 * b / c2}};
    for (int a = 0; a < 4; a++)
        for (int d = 0; d < 4; d++) {
            double s = 0.0;
            for (int m = 0; m < 4; m++) s += R[a][m] * lm[m] * L[m][d];
            A[4 * a + d] = s + (a == d ? vis : 0.0);
        }
}

static int residual(oigks_ctx *c)
{
    int nc = c->nc, nf = c->nf;
    double *W = c->W;
    const int nt = c->threads;
    /* ghost cell-centre states */
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int f = 0; f < nf; f++)
        if (c->fR[f] < 0) ghost_state(c, c->fbc[f], &W[5 * c->fL[f]], c->fnx[f], c->fny[f], &c->Wg[5 * f]);
    /* Eq.21: (Lambda_c)_i = sum_faces (|V_i . n| + C_i) S; Eq.23 dt = min */
    double dtmin = 1e300;
#pragma omp parallel for num_threads(nt) schedule(static) reduction(min : dtmin)
    for (int i = 0; i < nc; i++) {
        const double *Wi = &W[5 * i];
        double U = Wi[1] / Wi[0], V = Wi[2] / Wi[0], ci = sound(Wi), s = 0.0;
        for (int q = c->cfp[i]; q < c->cfp[i + 1]; q++) {
            int f = c->cff[q];
            s += (fabs(U * c->fnx[f] + V * c->fny[f]) + ci) * c->flen[f];
        }
        c->lamc[i] = s;
        double dt = c->opt.cfl_flux * c->area[i] / s;
        if (dt < dtmin) dtmin = dt;
    }
    c->dt_flux = dtmin;
    /* Eq.6-7: unweighted least squares over the face neighbours, ghost cells
     * at the reflected centroids included; 2x2 normal equations by Cramer. */
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int i = 0; i < nc; i++) {
        double a11 = 0, a12 = 0, a22 = 0, b1[4] = {0}, b2[4] = {0};
        for (int q = c->cfp[i]; q < c->cfp[i + 1]; q++) {
            int f = c->cff[q];
            double xj, yj; const double *Wj;
            if (c->fR[f] < 0) { ghost_centroid(c, f, &xj, &yj); Wj = &c->Wg[5 * f]; }
            else { int j = c->fL[f] == i ? c->fR[f] : c->fL[f]; xj = c->xc[j]; yj = c->yc[j]; Wj = &W[5 * j]; }
            double dx = xj - c->xc[i], dy = yj - c->yc[i];
            a11 += dx * dx; a12 += dx * dy; a22 += dy * dy;
            for (int k = 0; k < 4; k++) { double dw = Wj[k] - W[5 * i + k]; b1[k] += dx * dw; b2[k] += dy * dw; }
        }
        double det = a11 * a22 - a12 * a12;
        for (int k = 0; k < 4; k++) {
            c->ugx[4 * i + k] = (b1[k] * a22 - b2[k] * a12) / det;
            c->ugy[4 * i + k] = (a11 * b2[k] - a12 * b1[k]) / det;
        }
    }
    /* Eq.9-10 limiter, per cell and variable */
#pragma omp parallel for num_threads(nt) schedule(static)
    for (int i = 0; i < nc; i++) {
        for (int k = 0; k < 4; k++) {
            double phi = 1.0;
            if (c->opt.limiter && c->phi_frozen) {
                phi = c->phi[4 * i + k];
            } else if (c->opt.limiter) {
                double wc = W[5 * i + k], wmax = wc, wmin = wc;
                for (int q = c->cfp[i]; q < c->cfp[i + 1]; q++) {
                    int f = c->cff[q];
                    double wj = (c->fR[f] < 0) ? c->Wg[5 * f + k]
                                               : W[5 * (c->fL[f] == i ? c->fR[f] : c->fL[f]) + k];
                    if (wj > wmax) wmax = wj;
                    if (wj < wmin) wmin = wj;
                }
                double nmax = -1e300, nmin = 1e300;
                for (int p = c->cptr[i]; p < c->cptr[i + 1]; p++) {
                    int v = c->cnod[p];
                    double wv = wc + c->ugx[4 * i + k] * (c->x[v] - c->xc[i]) + c->ugy[4 * i + k] * (c->y[v] - c->yc[i]);
                    if (wv > nmax) nmax = wv;
                    if (wv < nmin) nmin = wv;
                }
                if (nmax > wc) { double r = (wmax - wc) / (nmax - wc); if (r < phi) phi = r; }
                if (nmin < wc) { double r = (wmin - wc) / (nmin - wc); if (r < phi) phi = r; }
                c->phi[4 * i + k] = phi;
            }
            c->gx[4 * i + k] = phi * c->ugx[4 * i + k];
            c->gy[4 * i + k] = phi * c->ugy[4 * i + k];
        }
        /* vorticity |dV/dx - dU/dy| from the unlimited gradients */
        double r = W[5 * i], U = W[5 * i + 1] / r, V = W[5 * i + 2] / r;
        double dUdy = (c->ugy[4 * i + 1] - U * c->ugy[4 * i + 0]) / r;
        double dVdx = (c->ugx[4 * i + 2] - V * c->ugx[4 * i + 0]) / r;
        c->vort[i] = fabs(dVdx - dUdy);
    }
    /* face loop: each face's flux, spectral radius and SA terms (summed
     * into the cells below) */
#pragma omp parallel for num_threads(nt) schedule(dynamic, 256)
    for (int f = 0; f < nf; f++) {
        int i = c->fL[f], j = c->fR[f];
        double nx = c->fnx[f], ny = c->fny[f], S = c->flen[f];
        double tx = -ny, ty = nx;
        const double *Wi = &W[5 * i];
        double rxl = c->fxm[f] - c->xc[i], ryl = c->fym[f] - c->yc[i];
        double dl = rxl * nx + ryl * ny;
        /* Eq.10 left state and its derivatives */
        double WL[4], GLx[4], GLy[4];
        for (int k = 0; k < 4; k++) {
            GLx[k] = c->gx[4 * i + k]; GLy[k] = c->gy[4 * i + k];
            WL[k] = Wi[k] + GLx[k] * rxl + GLy[k] * ryl;
        }
        if (!(WL[0] > 0) || !(WL[3] - 0.5 * (WL[1] * WL[1] + WL[2] * WL[2]) / WL[0] > 0)) {
            for (int k = 0; k < 4; k++) { WL[k] = Wi[k]; GLx[k] = GLy[k] = 0.0; }
        }
        double WR[4], GRx[4], GRy[4], WRc[5], dr, rn;
        const double *WjC;
        if (j >= 0) {
            const double *Wj = &W[5 * j];
            double rxr = c->fxm[f] - c->xc[j], ryr = c->fym[f] - c->yc[j];
            dr = -(rxr * nx + ryr * ny);
            for (int k = 0; k < 4; k++) {
                GRx[k] = c->gx[4 * j + k]; GRy[k] = c->gy[4 * j + k];
                WR[k] = Wj[k] + GRx[k] * rxr + GRy[k] * ryr;
            }
            if (!(WR[0] > 0) || !(WR[3] - 0.5 * (WR[1] * WR[1] + WR[2] * WR[2]) / WR[0] > 0)) {
                for (int k = 0; k < 4; k++) { WR[k] = Wj[k]; GRx[k] = GRy[k] = 0.0; }
            }
            for (int k = 0; k < 5; k++) WRc[k] = Wj[k];
            WjC = Wj;
            rn = fabs((c->xc[j] - c->xc[i]) * nx + (c->yc[j] - c->yc[i]) * ny);
        } else {
            /* reading (ghost-cell method): the ghost side of a boundary face
             * carries the boundary map of the reconstructed interior face
             * state (slopes: zero on free-stream and outflow faces, reflected
             * on symmetry and wall faces, below); its cell-centre value is the
             * map of the interior cell-centre value at the reflected
             * centroid. */
            double tmp[5], out[5];
            for (int k = 0; k < 4; k++) tmp[k] = WL[k];
            tmp[4] = Wi[4];
            ghost_state(c, c->fbc[f], tmp, nx, ny, out);
            for (int k = 0; k < 4; k++) { WR[k] = out[k]; GRx[k] = GRy[k] = 0.0; }
            for (int k = 0; k < 5; k++) WRc[k] = c->Wg[5 * f + k];
            WjC = &c->Wg[5 * f];
            dr = dl;
            rn = 2.0 * dl;
        }
        /* rotate into the face frame */
        double wl[4], wr[4], wlc[4], wrc[4], gln[4], glt[4], grn[4], grt[4];
#define ROT(dst, src) do { dst[0] = src[0]; dst[1] = src[1] * nx + src[2] * ny; \
                           dst[2] = src[1] * tx + src[2] * ty; dst[3] = src[3]; } while (0)
        ROT(wl, WL); ROT(wr, WR); ROT(wlc, Wi); ROT(wrc, WRc);
        double tn[4], tt[4];
        for (int k = 0; k < 4; k++) { tn[k] = GLx[k] * nx + GLy[k] * ny; tt[k] = GLx[k] * tx + GLy[k] * ty; }
        ROT(gln, tn); ROT(glt, tt);
        for (int k = 0; k < 4; k++) { tn[k] = GRx[k] * nx + GRy[k] * ny; tt[k] = GRx[k] * tx + GRy[k] * ty; }
        ROT(grn, tn); ROT(grt, tt);
#undef ROT
        if (j < 0 && (c->fbc[f] == BC_SYMMETRY || c->fbc[f] == BC_WALL)) {
            /* reading (ghost-cell method): the ghost cell of a symmetry face
             * is the mirror image of the interior cell and that of a no-slip
             * wall its point reflection through the face (momentum reversed,
             * bounce-back), slopes included.  In the face frame the normal
             * derivative flips sign and the boundary map acts on the momentum
             * components: symmetry (rho, -m_n, m_t, E), wall (rho, -m_n, -m_t,
             * E); the wall also flips the tangential derivative.  This keeps
             * the mass and energy fluxes through such faces zero. */
            double sn = -1.0, st = (c->fbc[f] == BC_WALL) ? -1.0 : 1.0;
            double bm_t = (c->fbc[f] == BC_WALL) ? -1.0 : 1.0;
            double Bk[4] = {1.0, -1.0, bm_t, 1.0};
            for (int k = 0; k < 4; k++) { grn[k] = sn * Bk[k] * gln[k]; grt[k] = st * Bk[k] * glt[k]; }
        }
        /* a moving wall (reading): the face is evaluated in the frame of
         * the wall, where it is a static no-slip wall, and the flux is
         * transformed back.  The interior face-frame state and slopes are
         * boosted by -u_w along the face, (rho, m_n, m_t, E) ->
         * (rho, m_n, m_t - u_w rho, E - u_w m_t + u_w^2 rho / 2), and the
         * ghost side is their point reflection as for a static wall. */
        /* An isothermal wall, static or moving, takes the same path with
         * u_w = 0 for a static one: the reflected states keep its mass and
         * energy fluxes zero, and the heat flux is added below. */
        double uw = 0.0;
        const int moving = j < 0 && (c->fbc[f] == BC_MOVING_WALL ||
                                     (c->fbc[f] == BC_WALL && c->opt.wall_temp > 0.0));
        if (moving) {
            if (c->fbc[f] == BC_MOVING_WALL) uw = (c->Winf[1] * tx + c->Winf[2] * ty) / c->Winf[0];
            double *bs[4] = {wl, wlc, gln, glt};
            for (int h = 0; h < 4; h++) {
                double *v = bs[h];
                v[3] = v[3] - uw * v[2] + 0.5 * uw * uw * v[0];
                v[2] = v[2] - uw * v[0];
            }
            const double Bk[4] = {1.0, -1.0, -1.0, 1.0};
            for (int k = 0; k < 4; k++) {
                wr[k] = Bk[k] * wl[k];
                wrc[k] = Bk[k] * wlc[k];
                grn[k] = -Bk[k] * gln[k];
                grt[k] = -Bk[k] * glt[k];
            }
        }
        /* tau from the interface equilibrium (Eq.34); the core needs W0
         * first, which it computes the same way */
        double sl[4], sr[4];
        {
            moms mlp, mrm;
            mk_moms(wl[1] / wl[0], wl[2] / wl[0], lam_of(wl), +1, &mlp);
            mk_moms(wr[1] / wr[0], wr[2] / wr[0], lam_of(wr), -1, &mrm);
            poly one; p_zero(&one); p_add_mono(&one, 1.0, 0, 0, 0);
            p_int_psi(&one, &mlp, sl); p_int_psi(&one, &mrm, sr);
        }
        double W0[4];
        for (int k = 0; k < 4; k++) W0[k] = wl[0] * sl[k] + wr[0] * sr[k];
        double nutf = 0.5 * (Wi[4] + WjC[4]);
        if (nutf < 0) nutf = 0;
        double tau = collision_time(c, W0[0], lam_of(W0), nutf);
        if (c->opt.tau_jump) {
            /* option (not in the paper; the usual gas-kinetic practice for
             * discontinuities): extra dissipation from the jump of the two
             * reconstructed pressures across the face */
            double pl = wl[3] - 0.5 * (wl[1] * wl[1] + wl[2] * wl[2]) / wl[0];
            double pr = wr[3] - 0.5 * (wr[1] * wr[1] + wr[2] * wr[2]) / wr[0];
            tau += c->dt_flux * fabs(pl - pr) / (pl + pr);
        }
        face_detail fd;
        gks_core(wl, gln, glt, wr, grn, grt, wlc, wrc, dl, dr, c->dt_flux, tau, &fd);
        if (j < 0 && c->opt.wall_temp > 0.0 && (c->fbc[f] == BC_WALL || c->fbc[f] == BC_MOVING_WALL)) {
            /* isothermal wall (reading): the reflected states above let no
             * mass or energy through in the wall's frame; a wall held at
             * temperature T_w adds the Navier-Stokes heat flux of the BGK
             * model (Pr = 1, kappa = mu c_p, c_p = gamma / (gamma - 1) in
             * units of R) across the distance d_l from the cell centre,
             * with mu at the cell-centre temperature */
            const double thw = c->opt.wall_temp * c->p_inf / c->Winf[0];
            const double pi = (GAMMA - 1.0) * (Wi[3] - 0.5 * (Wi[1] * Wi[1] + Wi[2] * Wi[2]) / Wi[0]);
            const double kappa = mu_lam(c, lam_of(Wi)) * GAMMA / (GAMMA - 1.0);
            fd.F[3] += c->dt_flux * kappa * (pi / Wi[0] - thw) / dl;
        }
        if (moving) {   /* back to the frame of the mesh */
            fd.F[3] += uw * fd.F[2] + 0.5 * uw * uw * fd.F[0];
            fd.F[2] += uw * fd.F[0];
        }
        double Fn = fd.F[1] / c->dt_flux, Ft = fd.F[2] / c->dt_flux;
        double Fb[4] = {fd.F[0] / c->dt_flux, Fn * nx + Ft * tx, Fn * ny + Ft * ty, fd.F[3] / c->dt_flux};
        for (int k = 0; k < 4; k++) c->ff[4 * f + k] = Fb[k] * S;
        /* LU-SGS spectral radius on the face (reading: max of the two sides'
         * |V.n| + C plus, optionally, a viscous term 2 nu_eff / |r.n|) */
        {
            double qi = (Wi[1] * nx + Wi[2] * ny) / Wi[0], qj = (WjC[1] * nx + WjC[2] * ny) / WjC[0];
            double li = fabs(qi) + sound(Wi), lj = fabs(qj) + sound(WjC);
            double lam = li > lj ? li : lj;
            if (c->opt.visc_sr) {
                double mi = mu_lam(c, lam_of(Wi)), mj = mu_lam(c, lam_of(WjC));
                if (c->sa) {
                    if (Wi[4] > 0) mi += Wi[0] * Wi[4] * sa_fv1(Wi[4] * Wi[0] / mu_lam(c, lam_of(Wi)));
                    if (WjC[4] > 0) mj += WjC[0] * WjC[4] * sa_fv1(WjC[4] * WjC[0] / mu_lam(c, lam_of(WjC)));
                }
                lam += 2.0 * 0.5 * (mi / Wi[0] + mj / WjC[0]) / rn;
            }
            c->flam[f] = lam;
            if (c->opt.lusgs_op)
                roe_abs(Wi, WjC, nx, ny, lam - (li > lj ? li : lj), c->opt.lusgs_op == 2, &c->fabsA[16 * f]);
        }
        /* SA face terms (Eq.28-30) from cell-centre values */
        if (c->sa) {
            double qi = (Wi[1] * nx + Wi[2] * ny) / Wi[0], qj = (WjC[1] * nx + WjC[2] * ny) / WjC[0];
            double nui = mu_lam(c, lam_of(Wi)) / Wi[0], nuj = mu_lam(c, lam_of(WjC)) / WjC[0];
            double ti = Wi[4], tj = WjC[4];
            double g = (tj - ti) / rn;
            double Finv = 0.5 * (qi + fabs(qi)) * ti + 0.5 * (qj - fabs(qj)) * tj;
            double Fvis = (1.0 / (2.0 * SA_SIGMA)) * ((nui + nuj) + (1.0 + SA_CB2) * (ti + tj)) * g;
            c->fsa[2 * f] = -Finv * S + Fvis * S - (SA_CB2 / SA_SIGMA) * ti * g * S;
            c->fsa[2 * f + 1] = j >= 0 ? Finv * S - Fvis * S - (SA_CB2 / SA_SIGMA) * tj * (-g) * S : 0.0;
            c->fsag[2 * f] = (fabs(Finv) + fabs(Fvis) + (SA_CB2 / SA_SIGMA) * fabs(ti * g)) * S;
            c->fsag[2 * f + 1] = j >= 0 ? (fabs(Finv) + fabs(Fvis) + (SA_CB2 / SA_SIGMA) * fabs(tj * g)) * S : 0.0;
        }
    }
    /* Eq.16: M = -sum F . S over the cell's faces (outward), summed in face
     * order; the SA right-hand side Eq.27 likewise */
    for (int k = 0; k < 5 * nc; k++) c->M[k] = 0.0;
    for (int f = 0; f < nf; f++) {
        int i = c->fL[f], j = c->fR[f];
        for (int k = 0; k < 4; k++) {
            c->M[5 * i + k] -= c->ff[4 * f + k];
            if (j >= 0) c->M[5 * j + k] += c->ff[4 * f + k];
        }
        if (c->sa) {
            c->M[5 * i + 4] += c->fsa[2 * f];
            if (j >= 0) c->M[5 * j + 4] += c->fsa[2 * f + 1];
        }
    }
    /* SA source, Omega Sr (Eq.27) */
    if (c->sa) {
#pragma omp parallel for num_threads(nt) schedule(static)
        for (int i = 0; i < nc; i++) {
            double nu = mu_lam(c, lam_of(&W[5 * i])) / W[5 * i];
            double so[4];
            sa_source(W[5 * i + 4], nu, c->dwall[i], c->vort[i], so);
            c->M[5 * i + 4] += c->area[i] * so[0];
            c->sasrc[i] = c->area[i] * so[0];
        }
    }
    return 0;
}

/* analytic Euler flux Jacobian-vector product J(W, n) dW (reading of the
 * paper's linearised first-order Roe Jacobian, Eq.18): the directional
 * derivative of F.n = (rho q, m q + p n, (E + p) q), q = V . n. */
static void jac_vec(const double *W, double nx, double ny, const double *d, double *out)
{
    double r = W[0], U = W[1] / r, V = W[2] / r, E = W[3];
    double p = (GAMMA - 1.0) * (E - 0.5 * r * (U * U + V * V));
    double q = U * nx + V * ny;
    double dmn = d[1] * nx + d[2] * ny;
    double dq = (dmn - q * d[0]) / r;
    double dp = (GAMMA - 1.0) * (d[3] - (U * d[1] + V * d[2]) + 0.5 * (U * U + V * V) * d[0]);
    out[0] = dmn;
    out[1] = d[1] * q + W[1] * dq + dp * nx;
    out[2] = d[2] * q + W[2] * dq + dp * ny;
    out[3] = (d[3] + dp) * q + (E + p) * dq;
}

/* SA implicit coefficients on a face as seen from cell i (Eq.31-32, frozen
 * coefficients, anti-diffusion left out of the implicit operator):
 * diag_i = u_i^+ S + k S / |r.n|, off_ij = -u_j^- S + k S / |r.n|. */
static void sa_face_coef(const oigks_ctx *c, const double *Wi, const double *Wj, double nx, double ny,
                         double S, double rn, double *diag, double *off)
{
    double qi = (Wi[1] * nx + Wi[2] * ny) / Wi[0], qj = (Wj[1] * nx + Wj[2] * ny) / Wj[0];
    double nui = mu_lam(c, lam_of(Wi)) / Wi[0], nuj = mu_lam(c, lam_of(Wj)) / Wj[0];
    double kf = (1.0 / SA_SIGMA) * (0.5 * (nui + nuj) + (1.0 + SA_CB2) * 0.5 * (Wi[4] + Wj[4]));
    *diag = 0.5 * (qi + fabs(qi)) * S + kf * S / rn;
    *off = -0.5 * (qj - fabs(qj)) * S + kf * S / rn;
}

/* a face between two sweep blocks (reading: the coupling the block sweeps
 * leave out; with the Roe operator such faces keep the scalar dissipation,
 * whose larger diagonal keeps the dropped coupling dominated) */
static int block_face(const oigks_ctx *c, int f)
{
    return c->sblk && c->fR[f] >= 0 && c->sblk[c->fL[f]] != c->sblk[c->fR[f]];
}

/* the dissipation of face f applied to an increment d: lambda_ij d for the
 * scalar operator (and for faces between sweep blocks), |A_ij| d for the Roe
 * matrix (the same from either side: |A(-n)| = |A(n)|) */
static void face_diss(const oigks_ctx *c, int f, const double *d, double *out)
{
    if (!c->opt.lusgs_op || block_face(c, f)) {
        for (int k = 0; k < 4; k++) out[k] = c->flam[f] * d[k];
        return;
    }
    const double *A = &c->fabsA[16 * f];
    for (int a = 0; a < 4; a++) out[a] = A[4 * a] * d[0] + A[4 * a + 1] * d[1] + A[4 * a + 2] * d[2] + A[4 * a + 3] * d[3];
}

/* D_i^-1 r: the scalar D of Eq.20, or its 4x4 block with the Roe matrix */
static void diag_solve(const oigks_ctx *c, int i, const double *r, double *x)
{
    if (!c->opt.lusgs_op) {
        for (int k = 0; k < 4; k++) x[k] = r[k] / c->D[i];
        return;
    }
    gauss4(&c->Dm[16 * i], r, x);
}

static double face_rn(const oigks_ctx *c, int f)
{
    int i = c->fL[f], j = c->fR[f];
    if (j >= 0) return fabs((c->xc[j] - c->xc[i]) * c->fnx[f] + (c->yc[j] - c->yc[i]) * c->fny[f]);
    double dl = (c->fxm[f] - c->xc[i]) * c->fnx[f] + (c->fym[f] - c->yc[i]) * c->fny[f];
    return 2.0 * dl;
}

/* Eq.19-22 matrix-free LU-SGS: forward sweep in increasing cell index,
 * backward sweep in decreasing index.  Boundary ghost increments (Sec. 2.5)
 * enter the backward sweep from the forward-sweep increment of the owner. */
/* One forward and backward sweep of Eq.22 (and Eq.31-32) over the cells in
 * index order, with the D of lusgs().  dWx (NULL: none): the increments of a
 * first block pass, whose cross-block terms then join the forward
 * right-hand side. */
static void lusgs_pass(oigks_ctx *c, const double *dWx)
{
    int nc = c->nc;
    double *W = c->W, *dW = c->dW;
    /* forward: dW*_i = D^-1 [M_i - sum_{j<i} (J(W_j, n_ij) dW*_j - lam_ij dW*_j) S_ij / 2] */
    for (int i = 0; i < nc; i++) {
        double acc[5] = {c->M[5 * i], c->M[5 * i + 1], c->M[5 * i + 2], c->M[5 * i + 3], c->M[5 * i + 4]};
        for (int q = c->cfp[i]; q < c->cfp[i + 1]; q++) {
            int f = c->cff[q];
            if (c->fR[f] < 0) continue;
            int j = c->fL[f] == i ? c->fR[f] : c->fL[f];
            /* a neighbour in another sweep block: left out, or on a second pass
             * taken with the first pass's increment, whether below or above */
            const int cross = c->sblk && c->sblk[j] != c->sblk[i];
            if (cross && !dWx) continue;
            if (!cross && j >= i) continue;
            const double *dj = cross ? &dWx[5 * j] : &dW[5 * j];
            double sg = c->fL[f] == i ? 1.0 : -1.0;
            double nx = sg * c->fnx[f], ny = sg * c->fny[f], S = c->flen[f];
            double jv[4], dv[4];
            jac_vec(&W[5 * j], nx, ny, dj, jv);
            face_diss(c, f, dj, dv);
            for (int k = 0; k < 4; k++) acc[k] -= 0.5 * (jv[k] - dv[k]) * S;
            if (c->sa) {
                double dg, of;
                sa_face_coef(c, &W[5 * i], &W[5 * j], nx, ny, S, face_rn(c, f), &dg, &of);
                acc[4] += of * dj[4];
            }
        }
        diag_solve(c, i, acc, &dW[5 * i]);
        dW[5 * i + 4] = c->sa ? acc[4] / c->Dsa[i] : 0.0;
    }
    /* backward: dW_i = dW*_i - D^-1 sum_{j>i} (...) S / 2, ghosts included */
    for (int i = nc - 1; i >= 0; i--) {
        double acc[5] = {0, 0, 0, 0, 0};
        double dWs[5];
        for (int k = 0; k < 5; k++) dWs[k] = dW[5 * i + k];
        for (int q = c->cfp[i]; q < c->cfp[i + 1]; q++) {
            int f = c->cff[q];
            double sg = c->fL[f] == i ? 1.0 : -1.0;
            double nx = sg * c->fnx[f], ny = sg * c->fny[f], S = c->flen[f];
            const double *Wj, *dj;
            double dg5[5];
            if (c->fR[f] < 0) {
                ghost_incr(c, c->fbc[f], dWs, nx, ny, dg5);
                Wj = &c->Wg[5 * f]; dj = dg5;
            } else {
                int j = c->fL[f] == i ? c->fR[f] : c->fL[f];
                if (j <= i) continue;
                if (c->sblk && c->sblk[j] != c->sblk[i]) continue;   /* another sweep block */
                Wj = &W[5 * j]; dj = &dW[5 * j];
            }
            double jv[4], dv[4];
            jac_vec(Wj, nx, ny, dj, jv);
            face_diss(c, f, dj, dv);
            for (int k = 0; k < 4; k++) acc[k] += 0.5 * (jv[k] - dv[k]) * S;
            if (c->sa) {
                double dg, of;
                sa_face_coef(c, &W[5 * i], Wj, nx, ny, S, face_rn(c, f), &dg, &of);
                acc[4] += of * dj[4];
            }
        }
        double corr[4];
        diag_solve(c, i, acc, corr);
        for (int k = 0; k < 4; k++) dW[5 * i + k] = dWs[k] - corr[k];
        dW[5 * i + 4] = c->sa ? dWs[4] + acc[4] / c->Dsa[i] : 0.0;
    }
}

static void lusgs(oigks_ctx *c)
{
    int nc = c->nc;
    double *W = c->W, *dW = c->dW;
#pragma omp parallel for num_threads(c->threads) schedule(static)
    for (int i = 0; i < nc; i++) {
        c->dtimp[i] = c->cfl * c->area[i] / c->lamc[i];             /* Eq.24 */
        double s = 0.0;
        for (int q = c->cfp[i]; q < c->cfp[i + 1]; q++) { int f = c->cff[q]; s += c->flam[f] * c->flen[f]; }
        c->D[i] = c->area[i] / c->dtimp[i] + 0.5 * s;                  /* Eq.20 */
        if (c->opt.lusgs_op) {   /* the block form: Omega / dt I + 1/2 sum |A_ij| S_ij */
            double *Dm = &c->Dm[16 * i];
            for (int k = 0; k < 16; k++) Dm[k] = k % 5 == 0 ? c->area[i] / c->dtimp[i] : 0.0;
            for (int q = c->cfp[i]; q < c->cfp[i + 1]; q++) {
                int f = c->cff[q];
                if (block_face(c, f)) {   /* lambda_ij I between sweep blocks */
                    for (int k = 0; k < 4; k++) Dm[5 * k] += 0.5 * c->flam[f] * c->flen[f];
                    continue;
                }
                for (int k = 0; k < 16; k++) Dm[k] += 0.5 * c->fabsA[16 * f + k] * c->flen[f];
            }
        }
        if (c->sa) {
            double ds = 0.0;
            for (int q = c->cfp[i]; q < c->cfp[i + 1]; q++) {
                int f = c->cff[q];
                int other = c->fR[f] < 0 ? -1 : (c->fL[f] == i ? c->fR[f] : c->fL[f]);
                double sg = c->fL[f] == i ? 1.0 : -1.0;
                const double *Wj = other >= 0 ? &W[5 * other] : &c->Wg[5 * f];
                double dg, of;
                sa_face_coef(c, &W[5 * i], Wj, sg * c->fnx[f], sg * c->fny[f], c->flen[f], face_rn(c, f), &dg, &of);
                ds += dg;
            }
            double nu = mu_lam(c, lam_of(&W[5 * i])) / W[5 * i];
            double so[4];
            sa_source(W[5 * i + 4], nu, c->dwall[i], c->vort[i], so);
            c->Dsa[i] = c->area[i] / c->dtimp[i] + ds + c->area[i] * so[3];
        }
    }
    /* block LU-SGS (sweep blocks): with two passes the second solves the
     * block-factored system again with the right-hand side
     * M - (L_o + U_o) dW1, L_o and U_o the cross-block terms and dW1 the first
     * pass's result: one block-Jacobi correction of the coupling the blocks
     * leave out */
    if (c->sblk && c->block_passes == 2) {
        if (!c->dW1) c->dW1 = malloc(sizeof(double) * 5 * nc);
        lusgs_pass(c, NULL);
        memcpy(c->dW1, c->dW, sizeof(double) * 5 * nc);
        lusgs_pass(c, c->dW1);
    } else {
        lusgs_pass(c, NULL);
    }
}

static void norms(oigks_ctx *c, double *inf, double *l2, double *sal2)
{
    double mx = 0.0, s = 0.0, comp = 0.0, sa = 0.0;
    for (int i = 0; i < c->nc; i++) {
        for (int k = 0; k < 4; k++) { double a = fabs(c->M[5 * i + k]); if (a > mx) mx = a; }
        /* Neumaier-compensated sum of squares */
        double v = c->M[5 * i] * c->M[5 * i], t = s + v;
        if (fabs(s) >= fabs(v)) comp += (s - t) + v; else comp += (v - t) + s;
        s = t;
        sa += c->M[5 * i + 4] * c->M[5 * i + 4];
    }
    *inf = mx; *l2 = sqrt(s + comp); *sal2 = sqrt(sa);
}

EXPORT int oigks_iterate(oigks_ctx *c, int n, int *n_done)
{
    if (n_done) *n_done = 0;
    if (!c->have_flow) { seterr(c, "set_freestream first"); return -1; }
    double *Wold = malloc(sizeof(double) * 5 * c->nc);
    for (int it = 0; it < n; it++) {
        residual(c);
        double inf, l2, sal2;
        norms(c, &inf, &l2, &sal2);
        /* the drop is measured from the largest ||M_rho||_2 so far (reading:
         * an impulsive start can have a mass residual of rounding size,
         * e.g. a uniform stream over a no-slip plate with the limiter on) */
        if (c->iter == 0 || l2 > c->res0) c->res0 = l2;
        if (c->iter == 0) { c->cfl = c->opt.cfl_init; }
        else if (c->opt.cfl_mode == 0 && c->opt.scheme == 0) {   /* Eq.25 */
            double cf = c->cfl * c->res_inf_prev / inf;
            if (!(cf >= c->opt.cfl_min)) cf = c->opt.cfl_min;
            if (cf > c->opt.cfl_max) cf = c->opt.cfl_max;
            c->cfl = cf;
        }
        c->res_inf_prev = inf;
        /* limiter freezing (reading: the Eq.9 factors chatter between
         * iterations near convergence and hold the residual up; from the
         * next iteration on they keep the values just computed) */
        if (c->opt.limiter && c->opt.limiter_freeze > 0.0 && !c->phi_frozen && l2 <= c->opt.limiter_freeze * c->res0)
            c->phi_frozen = 1;
        if (c->opt.scheme == 1) {
            /* Eq.15: W^{n+1} = W^n - (1/Omega) sum F S with the flux integrated
             * over a local step dt_i = CFL Omega_i / (Lambda_c)_i (the cell form
             * of Eq.21/23), i.e. dW_i = dt_i M_i / Omega_i = CFL M_i / (Lambda_c)_i;
             * nu-tilde the same way with the SA right-hand side */
            for (int i = 0; i < c->nc; i++) {
                double k = c->cfl / c->lamc[i];
                for (int q = 0; q < 4; q++) c->dW[5 * i + q] = k * c->M[5 * i + q];
                c->dW[5 * i + 4] = c->sa ? k * c->M[5 * i + 4] : 0.0;
            }
        } else {
            lusgs(c);
        }
        /* Eq.17 update; nu-tilde clipped at zero; Eq.40 criterion */
        memcpy(Wold, c->W, sizeof(double) * 5 * c->nc);
        double e40 = 0.0;
        int bad = 0;
        for (int i = 0; i < c->nc; i++) {
            double *Wi = &c->W[5 * i], num = 0.0, den = 0.0;
            for (int k = 0; k < 4; k++) {
                double d = c->dW[5 * i + k];
                num += d * d; den += Wi[k] * Wi[k];
                Wi[k] += d;
            }
            if (c->sa) { Wi[4] += c->dW[5 * i + 4]; if (Wi[4] < 0) Wi[4] = 0; }
            double r = sqrt(num / den);
            if (r > e40) e40 = r;
            double p = Wi[3] - 0.5 * (Wi[1] * Wi[1] + Wi[2] * Wi[2]) / Wi[0];
            if (!(Wi[0] > 0) || !(p > 0) || !isfinite(Wi[4])) bad = 1;
        }
        c->last.iteration = c->iter; c->last.res_l2 = l2; c->last.res_drop = c->res0 > 0 ? l2 / c->res0 : 0;
        c->last.res_inf = inf; c->last.eq40 = e40; c->last.cfl = c->cfl; c->last.dt_flux = c->dt_flux;
        c->last.sa_l2 = sal2;
        if (bad) {
            memcpy(c->W, Wold, sizeof(double) * 5 * c->nc);
            seterr(c, "non-physical state (rho <= 0, p <= 0 or non-finite)");
            free(Wold);
            return -4;
        }
        c->iter++;
        if (n_done) *n_done = it + 1;
    }
    free(Wold);
    return 0;
}

/* Sweep blocks (reading, the block form of LU-SGS used on partitioned
 * meshes): blk[i] is the block of cell i; the sweeps of Eq.22 (and Eq.31-32)
 * then couple only cells of one block, visiting them in index order, and
 * leave the neighbours in other blocks out of the lower and upper parts
 * (their increments taken as zero); the diagonal keeps every face.  NULL:
 * one block, the plain sweeps. */
/* passes of the block sweeps: 1, or 2 (see lusgs) */
EXPORT int oigks_set_block_passes(oigks_ctx *c, int n)
{
    if (n != 1 && n != 2) { seterr(c, "block passes must be 1 or 2"); return -1; }
    c->block_passes = n;
    return 0;
}

EXPORT int oigks_set_sweep_blocks(oigks_ctx *c, const int *blk)
{
    if (!c->cptr) { seterr(c, "no mesh"); return -1; }
    free(c->sblk);
    c->sblk = NULL;
    if (!blk) return 0;
    c->sblk = malloc(sizeof(int) * c->nc);
    for (int i = 0; i < c->nc; i++) {
        if (blk[i] < 0) { free(c->sblk); c->sblk = NULL; seterr(c, "negative sweep block"); return -1; }
        c->sblk[i] = blk[i];
    }
    return 0;
}

/* threads of the per-cell and per-face loops (results do not depend on it) */
EXPORT int oigks_set_threads(oigks_ctx *c, int n)
{
    if (n < 1) { seterr(c, "thread count must be at least 1"); return -1; }
    c->threads = n;
    return 0;
}

EXPORT int oigks_get_residual(oigks_ctx *c, oigks_residual *out) { *out = c->last; out->iteration = c->iter; return 0; }

/* the last computed (or held) limiter factors, 4 per cell SoA, and whether
 * they are held */
EXPORT int oigks_get_limiter(oigks_ctx *c, double *phi, int *frozen)
{
    if (phi) for (int i = 0; i < c->nc; i++) for (int k = 0; k < 4; k++) phi[k * c->nc + i] = c->phi[4 * i + k];
    if (frozen) *frozen = c->phi_frozen;
    return 0;
}

/* state in SoA layout, W[k * n_cells + i] */
EXPORT int oigks_get_state(oigks_ctx *c, double *W)
{
    for (int i = 0; i < c->nc; i++) for (int k = 0; k < 5; k++) W[k * c->nc + i] = c->W[5 * i + k];
    return 0;
}
EXPORT int oigks_set_state(oigks_ctx *c, const double *W)
{
    if (!c->have_flow) { seterr(c, "set_freestream first"); return -1; }
    for (int i = 0; i < c->nc; i++) {
        double r = W[i], mx = W[c->nc + i], my = W[2 * c->nc + i], E = W[3 * c->nc + i];
        double p = E - 0.5 * (mx * mx + my * my) / r;
        if (!(r > 0) || !(p > 0) || !isfinite(W[4 * c->nc + i])) { seterr(c, "non-physical state"); return -4; }
    }
    for (int i = 0; i < c->nc; i++) for (int k = 0; k < 5; k++) c->W[5 * i + k] = W[k * c->nc + i];
    c->phi_frozen = 0;
    return 0;
}
/* Residual of the current state: M (4 flow components, Eq.16) and the SA
 * right-hand side Omega Sr + R (Eq.27), SoA 5 x n_cells.  Also returns the
 * gross flux sum_faces |F S| per cell and component (the scale the residual
 * cancels from). */
EXPORT int oigks_compute_residual(oigks_ctx *c, double *M, double *gross)
{
    if (!c->have_flow) { seterr(c, "set_freestream first"); return -1; }
    residual(c);
    for (int i = 0; i < c->nc; i++) for (int k = 0; k < 5; k++) M[k * c->nc + i] = c->M[5 * i + k];
    if (gross) {
        for (int k = 0; k < 4 * c->nc; k++) gross[k] = 0.0;
        for (int f = 0; f < c->nf; f++)
            for (int k = 0; k < 4; k++) {
                double a = fabs(c->ff[4 * f + k]);
                gross[k * c->nc + c->fL[f]] += a;
                if (c->fR[f] >= 0) gross[k * c->nc + c->fR[f]] += a;
            }
    }
    return 0;
}
/* Gross size of the SA right-hand side of each cell at the current state:
 * the sum over its faces of the magnitudes of the convective, diffusive and
 * anti-diffusive terms of Eq.29 (times S) plus Omega |Sr| (Eq.28a), the
 * scale its residual cancels from (0 in laminar runs). */
EXPORT int oigks_sa_gross(oigks_ctx *c, double *out)
{
    if (!c->have_flow) { seterr(c, "set_freestream first"); return -1; }
    residual(c);
    for (int i = 0; i < c->nc; i++) out[i] = c->sa ? fabs(c->sasrc[i]) : 0.0;
    if (c->sa)
        for (int f = 0; f < c->nf; f++) {
            out[c->fL[f]] += c->fsag[2 * f];
            if (c->fR[f] >= 0) out[c->fR[f]] += c->fsag[2 * f + 1];
        }
    return 0;
}
/* One LU-SGS solve at the current state with the given CFL: returns dW
 * (SoA 5 x n_cells) without updating the state. */
EXPORT int oigks_lusgs_solve(oigks_ctx *c, double cfl, double *dW)
{
    if (!c->have_flow) { seterr(c, "set_freestream first"); return -1; }
    residual(c);
    c->cfl = cfl;
    lusgs(c);
    for (int i = 0; i < c->nc; i++) for (int k = 0; k < 5; k++) dW[k * c->nc + i] = c->dW[5 * i + k];
    return 0;
}

/* wall loads from the face fluxes of the current state (reading: the GKS
 * momentum flux through a no-slip face is the fluid force on that face).
 * cl, cd: per unit span, reference 0.5 rho_inf |V_inf|^2 * 1. Arrays of
 * length n_wall_faces, in the order the WALL edges appear in the input
 * boundary-edge list: Cp, Cf, x of the face midpoint. */
EXPORT int oigks_get_wall_loads(oigks_ctx *c, double *cl, double *cd, double *cf, double *cp, double *xw)
{
    if (!c->have_flow) { seterr(c, "set_freestream first"); return -1; }
    residual(c);
    double Fx = 0, Fy = 0, q = 0.5;
    double ca = cos(c->alpha), sa = sin(c->alpha);
    for (int w = 0; w < c->nwall; w++) {
        int f = c->wall_faces[w];
        double fx = c->ff[4 * f + 1], fy = c->ff[4 * f + 2], S = c->flen[f];
        Fx += fx; Fy += fy;
        double nx = c->fnx[f], ny = c->fny[f], tx = -ny, ty = nx;
        if (tx * ca + ty * sa < 0) { tx = -tx; ty = -ty; }
        if (cp) cp[w] = ((fx * nx + fy * ny) / S - c->p_inf) / q;
        if (cf) cf[w] = ((fx * tx + fy * ty) / S) / q;
        if (xw) xw[w] = c->fxm[f];
    }
    if (cd) *cd = (Fx * ca + Fy * sa) / q;
    if (cl) *cl = (-Fx * sa + Fy * ca) / q;
    return 0;
}

/* ---------------- accessors used by the tests ---------------- */
EXPORT int oigks_n_cells(const oigks_ctx *c) { return c->nc; }
EXPORT int oigks_n_faces(const oigks_ctx *c) { return c->nf; }
EXPORT int oigks_n_wall_faces(const oigks_ctx *c) { return c->nwall; }
EXPORT double oigks_dt_flux(const oigks_ctx *c) { return c->dt_flux; }
/* faces: owner, neighbour (-1), boundary type in use, normal, length, midpoint */
EXPORT int oigks_get_faces(const oigks_ctx *c, int *fl, int *fr, int *bc, double *nx, double *ny,
                           double *len, double *xm, double *ym)
{
    for (int f = 0; f < c->nf; f++) {
        if (fl) fl[f] = c->fL[f]; if (fr) fr[f] = c->fR[f]; if (bc) bc[f] = c->fbc[f];
        if (nx) nx[f] = c->fnx[f]; if (ny) ny[f] = c->fny[f]; if (len) len[f] = c->flen[f];
        if (xm) xm[f] = c->fxm[f]; if (ym) ym[f] = c->fym[f];
    }
    return 0;
}
EXPORT int oigks_get_cells(const oigks_ctx *c, double *area, double *xc, double *yc, double *dwall)
{
    for (int i = 0; i < c->nc; i++) {
        if (area) area[i] = c->area[i]; if (xc) xc[i] = c->xc[i]; if (yc) yc[i] = c->yc[i];
        if (dwall) dwall[i] = c->dwall[i];
    }
    return 0;
}
/* per-face and per-cell data of the last residual / LU-SGS call:
 * flux (4 x nf, Fbar S, global frame), lam (nf), ghost W (5 x nf, zero on
 * interior faces), D (nc), Dsa (nc), lamc (nc), dtimp (nc), grad (8 x nc:
 * limited d/dx of 4 vars then d/dy), vort (nc). */
EXPORT int oigks_get_debug(const oigks_ctx *c, double *flux, double *lam, double *wg, double *D, double *Dsa,
                           double *lamc, double *dtimp, double *grad, double *vort)
{
    int nf = c->nf, nc = c->nc;
    for (int f = 0; f < nf; f++) {
        if (flux) for (int k = 0; k < 4; k++) flux[k * nf + f] = c->ff[4 * f + k];
        if (lam) lam[f] = c->flam[f];
        if (wg) for (int k = 0; k < 5; k++) wg[k * nf + f] = c->Wg[5 * f + k];
    }
    for (int i = 0; i < nc; i++) {
        if (D) D[i] = c->D[i]; if (Dsa) Dsa[i] = c->Dsa[i]; if (lamc) lamc[i] = c->lamc[i];
        if (dtimp) dtimp[i] = c->dtimp[i];
        if (grad) for (int k = 0; k < 4; k++) { grad[k * nc + i] = c->gx[4 * i + k]; grad[(4 + k) * nc + i] = c->gy[4 * i + k]; }
        if (vort) vort[i] = c->vort[i];
    }
    return 0;
}

/* the Roe dissipation matrices of the last residual (lusgs_op 1): 16 values
 * per face, row by row; -1 when the scalar operator is in use */
EXPORT int oigks_get_roe(const oigks_ctx *c, double *absA)
{
    if (!c->opt.lusgs_op || !c->fabsA) return -1;
    memcpy(absA, c->fabsA, sizeof(double) * 16 * (size_t)c->nf);
    return 0;
}

/* ---------------- kernel-level entry points used by the pins ---------------- */
EXPORT void oigks_roe_abs(const double *Wl, const double *Wr, double nx, double ny, double vis, int kin, double *A)
{
    roe_abs(Wl, Wr, nx, ny, vis, kin, A);
}
EXPORT void oigks_moments(double U, double lam, int kind, int n, double *out)
{
    double m[MOMN];
    mom_line(U, lam, kind, m);
    for (int k = 0; k < n && k < MOMN; k++) out[k] = m[k];
}
EXPORT void oigks_moment_matrix(double U, double V, double lam, double *M)
{
    moms m; mk_moms(U, V, lam, 0, &m); moment_matrix(&m, M);
}
EXPORT void oigks_slope(const double *W, const double *dW, double *a)
{
    moms m; mk_moms(W[1] / W[0], W[2] / W[0], lam_of(W), 0, &m); solve_slope(&m, W[0], dW, a);
}
/* face-frame GKS flux with explicit tau and dt; out packs face_detail:
 * W0[4] lam0 aln alt arn art abnl abnr abt Al Ar Ab T[6] F[4] (59 values) */
EXPORT void oigks_face_detail(const double *Wl, const double *Gln, const double *Glt, const double *Wr,
                              const double *Grn, const double *Grt, const double *Wlc, const double *Wrc,
                              double dl, double dr, double dt, double tau, double *out)
{
    face_detail o;
    gks_core(Wl, Gln, Glt, Wr, Grn, Grt, Wlc, Wrc, dl, dr, dt, tau, &o);
    double *p = out;
    for (int i = 0; i < 4; i++) *p++ = o.W0[i];
    *p++ = o.lam0;
    const double *blocks[] = {o.aln, o.alt, o.arn, o.art, o.abnl, o.abnr, o.abt, o.Al, o.Ar, o.Ab};
    for (int b = 0; b < 10; b++) for (int i = 0; i < 4; i++) *p++ = blocks[b][i];
    for (int i = 0; i < 6; i++) *p++ = o.T[i];
    for (int i = 0; i < 4; i++) *p++ = o.F[i];
}
EXPORT void oigks_sa_source(double nut, double nu, double d, double omega, double *out) { sa_source(nut, nu, d, omega, out); }
EXPORT void oigks_jac_vec(const double *W, double nx, double ny, const double *d, double *out) { jac_vec(W, nx, ny, d, out); }
EXPORT double oigks_collision_time(oigks_ctx *c, double rho0, double lam0, double nut_f) { return collision_time(c, rho0, lam0, nut_f); }
EXPORT void oigks_ghost_state(oigks_ctx *c, int bc, const double *Wi, double nx, double ny, double *Wg) { ghost_state(c, bc, Wi, nx, ny, Wg); }
EXPORT double oigks_mu(oigks_ctx *c, double lam) { return mu_lam(c, lam); }
