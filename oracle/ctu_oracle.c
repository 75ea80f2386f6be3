/*
 * ctu_oracle.c -- plain, slow FP64 CPU reference of the unsplit CTU/PPM
 * Godunov advance of an ideal gamma-law gas.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the tests, the package smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  It shares no code,
 * header, table or helper with the HIP path.
 *
 * What the method computes: the paper states that Castro's main hydrodynamics
 * scheme is an unsplit piecewise parabolic method, advanced box by box on a
 * block-structured grid with coarse levels advanced first, fine levels
 * subcycled and the levels then synchronised (section 3 and section 3.2).  The
 * paper gives no further detail, so every step below follows the published
 * method it names, in this reading:
 *   - PPM reconstruction, limiter and flattening: Colella & Woodward 1984
 *     (CW84), JCP 54:174, section 1 and appendix; optionally the
 *     extremum-preserving limiter of Colella & Sekora 2008 (CS08), JCP
 *     227:7069;
 *   - corner-transport-upwind (unsplit) coupling and characteristic tracing:
 *     Colella 1990, JCP 87:171; Saltzman 1994, JCP 115:153; Miller & Colella
 *     2002, JCP 183:26;
 *   - HLLC Riemann flux with Davis wave-speed bounds: Toro, Spruce & Speares
 *     1994, Shock Waves 4:25; Davis 1988, SIAM J. Sci. Stat. Comput. 9:445;
 *   - or the two-shock approximate Riemann solver of the PPM lineage (both
 *     waves on their shock curves, Newton iteration for the star pressure):
 *     Colella 1982, SIAM J. Sci. Stat. Comput. 3:76; Colella & Glaz 1985,
 *     JCP 59:264;
 *   - two-level refluxing: Berger & Colella 1989, JCP 82:64.
 * Steps are coded in the order the method takes them, on whole arrays, one
 * stage after another.  Floating-point expressions are written exactly as the
 * stated formulas parenthesise them and are compiled without contraction
 * (-ffp-contract=off) and without fast-math.
 *
 * Method-of-lines variant (the formulation of the paper's GPU proxy, section
 * 4, which names it and nothing more): the spatial operator reconstructs the
 * same PPM parabolas (with flattening) and takes their edge values as the face
 * states, with no characteristic tracing and no transverse corrections, then
 * the interface flux and the flux divergence; gravity enters as a source term.
 * Time integration is the strong-stability-preserving Runge-Kutta method of
 * Shu & Osher 1988 (JCP 77:439) of order 2 or 3, ghost cells refilled before
 * every stage, dt from the CFL condition on the sum over directions of the
 * signal speeds (an unsplit multi-stage scheme sees all three at once).
 *
 * Passive species (mass fractions X_s, conserved rho X_s after rho E) follow
 * the flow: reconstructed like any primitive, traced with the contact family
 * (like the transverse velocities), corrected and fluxed like the transverse
 * momenta (HLLC star state scaled by the same factor), updated conservatively.
 *
 * Layouts.  A box of n = (nx, ny, nz) valid cells is stored "grown" by 4 ghost
 * cells: U[c][k][j][i], c in 0..4 = (rho, rho u, rho v, rho w, rho E), then
 * c = 5.. the species rho X_s, i fastest,
 * cell (i,j,k) of the box at offset ((c*(nz+8)+k+4)*(ny+8)+j+4)*(nx+8)+i+4.
 * Stage arrays use the "halo-1" geometry, indices -1..n in every direction,
 * offset ((c*(nz+2)+k+1)*(ny+2)+j+1)*(nx+2)+i+1.  A face array for direction d
 * stores face f (between cells f-1 and f along d) at index f along d.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#define NG 4
#define MAXSPEC 16
#define MAXV (5 + MAXSPEC)

enum { BC_PERIODIC = 0, BC_OUTFLOW = 1, BC_REFLECT = 2, BC_INFLOW = 3 };

/* counters: 0 density floor in cons->prim, 1 pressure floor in cons->prim,
 * 2 floors on traced states, 3 transverse fall-backs, 4 update failures */
#define NCNT 5

typedef struct {
    double gamma, cfl, small_dens, small_pres, grav_z;
    double dx[3];
    int bc_lo[3], bc_hi[3];
    double inflow[5]; /* rho, u, v, w, p */
    int nspec;        /* passive species (0..16) */
    int pad;
    double inflow_X[MAXSPEC];
    int scheme;       /* 0 unsplit CTU/PPM, 1 MOL with SSP-RK2, 2 MOL with SSP-RK3 */
    int riemann;      /* 0 HLLC, 1 two-shock approximate solver */
    int limiter;      /* 0 CW84, 1 Colella & Sekora 2008 extremum-preserving */
    int steepen;      /* 1: CW84 contact steepening of the density (with limiter 0) */
    /* where the domain's faces lie in the box being advanced (box-local face
     * index); faces_set = 0 means the box is the whole domain (faces 0 and n) */
    int faces_set;
    int face_lo[3], face_hi[3];
} orc_params;

static int nvar_of(const orc_params *P) { return 5 + P->nspec; }

/* optional stage outputs (NULL entries are allocated internally) */
typedef struct {
    double *q;        /* (6 + nspec) x grown: rho,u,v,w,p,c,X_s */
    double *phi;      /* 1 x halo-1 */
    double *ql[3];    /* nvar x halo-1, permuted primitives (+ X_s), left state of face */
    double *qr[3];    /* nvar x halo-1, right state of face */
    double *fn[3];    /* nvar x halo-1, normal fluxes (conserved order) */
    double *f1[6];    /* nvar x halo-1, stage-1 fluxes, pair index 2a+(b==(a+1)%3?0:1) */
    double *ff[3];    /* nvar x halo-1, final fluxes */
} orc_stages;

static double omin(double a, double b) { return a < b ? a : b; }
static double omax(double a, double b) { return a > b ? a : b; }

/* ---------------------------------------------------------------- indexing */

typedef struct { int n[3]; long gx, gy, gz, hx, hy, hz; } geom;

static geom mkgeom(const int n[3]) {
    geom g;
    for (int d = 0; d < 3; ++d) g.n[d] = n[d];
    g.gx = n[0] + 2 * NG; g.gy = n[1] + 2 * NG; g.gz = n[2] + 2 * NG;
    g.hx = n[0] + 2; g.hy = n[1] + 2; g.hz = n[2] + 2;
    return g;
}
static long gidx(const geom *g, int c, int i, int j, int k) {
    return ((c * g->gz + (k + NG)) * g->gy + (j + NG)) * g->gx + (i + NG);
}
static long hidx(const geom *g, int c, int i, int j, int k) {
    return ((c * g->hz + (k + 1)) * g->hy + (j + 1)) * g->hx + (i + 1);
}
static long gsize(const geom *g) { return g->gx * g->gy * g->gz; }
static long hsize(const geom *g) { return g->hx * g->hy * g->hz; }

/* tangential directions of a sweep along d: x:(y,z) y:(z,x) z:(x,y) */
static int t1of(int d) { return (d + 1) % 3; }
static int t2of(int d) { return (d + 2) % 3; }

/* ---------------------------------------------------- state conversions (O1, O3) */

/* Conserved -> primitive for a cell (rho,u,v,w,p,c), with the density and
 * pressure floors; the kinetic energy sums u^2+v^2 first, then w^2. */
static void cons_to_prim_cell(const double *U, const orc_params *P, double *q, long long *cnt) {
    const double gm1 = P->gamma - 1.0;
    double rho = U[0];
    if (rho < P->small_dens) { rho = P->small_dens; cnt[0]++; }
    double u = U[1] / rho, v = U[2] / rho, w = U[3] / rho;
    double ke = 0.5 * rho * ((u * u + v * v) + w * w);
    double p = gm1 * (U[4] - ke);
    if (p < P->small_pres) { p = P->small_pres; cnt[1]++; }
    q[0] = rho; q[1] = u; q[2] = v; q[3] = w; q[4] = p;
    q[5] = sqrt(P->gamma * p / rho);
    for (int sp = 0; sp < P->nspec; ++sp) q[6 + sp] = U[5 + sp] / rho;
}

/* Permuted primitive state of a sweep along d (rho, u_n, u_t1, u_t2, p) to the
 * conserved state in global component order. */
static void perm_prim_to_cons(const double *s, int d, const orc_params *P, double *U) {
    const double rgm1 = 1.0 / (P->gamma - 1.0);
    double rho = s[0];
    U[0] = rho;
    U[1 + d] = rho * s[1];
    U[1 + t1of(d)] = rho * s[2];
    U[1 + t2of(d)] = rho * s[3];
    U[4] = s[4] * rgm1 + 0.5 * rho * ((s[1] * s[1] + s[2] * s[2]) + s[3] * s[3]);
    for (int sp = 0; sp < P->nspec; ++sp) U[5 + sp] = rho * s[5 + sp];
}

/* Conserved (global order) to the permuted primitive state of a sweep along d,
 * without floors (the caller decides what a non-physical result means). */
static void cons_to_perm_prim(const double *U, int d, const orc_params *P, double *s) {
    const double gm1 = P->gamma - 1.0;
    double rho = U[0];
    double un = U[1 + d] / rho, ut1 = U[1 + t1of(d)] / rho, ut2 = U[1 + t2of(d)] / rho;
    double ke = 0.5 * rho * ((un * un + ut1 * ut1) + ut2 * ut2);
    s[0] = rho; s[1] = un; s[2] = ut1; s[3] = ut2;
    s[4] = gm1 * (U[4] - ke);
    for (int sp = 0; sp < P->nspec; ++sp) s[5 + sp] = U[5 + sp] / rho;
}

/* ------------------------------------------------------------ HLLC flux (O7) */

/* HLLC flux (Toro, Spruce & Speares 1994) with Davis (1988) speed bounds
 * S_L = min(u_L-c_L, u_R-c_R), S_R = max(u_L+c_L, u_R+c_R).  L and R are
 * permuted primitives of a sweep along d (species after p); the flux is
 * returned in global conserved order.  Species X ride the contact: their star
 * state is the same factor times X_K as the transverse momenta. */
static void hllc_n(const double *L, const double *R, int d, const orc_params *P, double *Fg) {
    const int ns = P->nspec;
    const double g = P->gamma, rgm1 = 1.0 / (g - 1.0);
    const double rL = L[0], uL = L[1], vL = L[2], wL = L[3], pL = L[4];
    const double rR = R[0], uR = R[1], vR = R[2], wR = R[3], pR = R[4];
    const double cL = sqrt(g * pL / rL), cR = sqrt(g * pR / rR);
    const double SL = omin(uL - cL, uR - cR);
    const double SR = omax(uL + cL, uR + cR);
    const double EL = pL * rgm1 + 0.5 * rL * ((uL * uL + vL * vL) + wL * wL);
    const double ER = pR * rgm1 + 0.5 * rR * ((uR * uR + vR * vR) + wR * wR);
    double F[MAXV];
    if (SL >= 0.0) {
        double m = rL * uL;
        F[0] = m; F[1] = m * uL + pL; F[2] = m * vL; F[3] = m * wL; F[4] = uL * (EL + pL);
        for (int sp = 0; sp < ns; ++sp) F[5 + sp] = m * L[5 + sp];
    } else {
        const double Ss = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) /
                          (rL * (SL - uL) - rR * (SR - uR));
        if (Ss >= 0.0 || SR > 0.0) {
            /* one star region: K = L if S* >= 0, else K = R */
            const int left = (Ss >= 0.0);
            const double *K = left ? L : R;
            const double rK = left ? rL : rR, uK = left ? uL : uR, vK = left ? vL : vR;
            const double wK = left ? wL : wR, pK = left ? pL : pR, EK = left ? EL : ER;
            const double SK = left ? SL : SR;
            const double m = rK * uK;
            double FK[MAXV], UK[MAXV], Us[MAXV];
            FK[0] = m; FK[1] = m * uK + pK; FK[2] = m * vK; FK[3] = m * wK; FK[4] = uK * (EK + pK);
            UK[0] = rK; UK[1] = m; UK[2] = rK * vK; UK[3] = rK * wK; UK[4] = EK;
            const double fac = rK * (SK - uK) / (SK - Ss);
            Us[0] = fac;
            Us[1] = fac * Ss;
            Us[2] = fac * vK;
            Us[3] = fac * wK;
            Us[4] = fac * (EK / rK + (Ss - uK) * (Ss + pK / (rK * (SK - uK))));
            for (int sp = 0; sp < ns; ++sp) {
                FK[5 + sp] = m * K[5 + sp];
                UK[5 + sp] = rK * K[5 + sp];
                Us[5 + sp] = fac * K[5 + sp];
            }
            for (int c = 0; c < 5 + ns; ++c) F[c] = FK[c] + SK * (Us[c] - UK[c]);
        } else {
            double m = rR * uR;
            F[0] = m; F[1] = m * uR + pR; F[2] = m * vR; F[3] = m * wR; F[4] = uR * (ER + pR);
            for (int sp = 0; sp < ns; ++sp) F[5 + sp] = m * R[5 + sp];
        }
    }
    Fg[0] = F[0];
    Fg[1 + d] = F[1];
    Fg[1 + t1of(d)] = F[2];
    Fg[1 + t2of(d)] = F[3];
    Fg[4] = F[4];
    for (int sp = 0; sp < ns; ++sp) Fg[5 + sp] = F[5 + sp];
}

/* Five-component entry point (pins). */
void orc_hllc(const double L[5], const double R[5], int d, const orc_params *P, double Fg[5]) {
    orc_params Q = *P;
    Q.nspec = 0;
    hllc_n(L, R, d, &Q, Fg);
}

/* ------------------------------------------- two-shock Riemann solver (f3) */

#define TWOSHOCK_ITERS 6

/* Godunov flux of the two-shock approximate Riemann solution between the
 * permuted primitive states L and R (species after p).  Both nonlinear waves
 * are put on their shock curves: with Lagrangian sound speeds C_K =
 * sqrt(gamma p_K rho_K) and shock speeds W_K(p) = C_K sqrt(1 + (gamma+1)/(2
 * gamma) (p/p_K - 1)), the star pressure solves u*_L(p) = u*_R(p), u*_L =
 * u_L - (p - p_L)/W_L, u*_R = u_R + (p - p_R)/W_R, by Newton steps with the
 * curve slopes Z_K = 2 W_K^3 / (W_K^2 + C_K^2), from the acoustic estimate,
 * a fixed number of times, floored at small_pres.  The contact velocity is
 * u* = (W_L u_L + W_R u_R + p_L - p_R) / (W_L + W_R).  The state at x/t = 0
 * is taken on the upwind side of the contact (K = L if u* >= 0): the
 * unperturbed state K beyond the K wave, the star state (rho* from the shock
 * relation 1/rho* = 1/rho_K - (p* - p_K)/W_K^2) behind it, and for a
 * rarefaction whose fan straddles x/t = 0 the linear blend of the two between
 * the head u_K -+ c_K and the tail u* -+ c*.  Transverse velocities and
 * species come from K.  The flux is the Euler flux of that state. */
static void twoshock_n(const double *L, const double *R, int d, const orc_params *P, double *Fg) {
    const int ns = P->nspec;
    const double g = P->gamma, rgm1 = 1.0 / (g - 1.0), gp = (g + 1.0) / (2.0 * g);
    const double rL = L[0], uL = L[1], pL = L[4];
    const double rR = R[0], uR = R[1], pR = R[4];
    const double CL = sqrt(g * pL * rL), CR = sqrt(g * pR * rR);
    double ps = ((CR * pL + CL * pR) + CL * CR * (uL - uR)) / (CL + CR);
    ps = omax(ps, P->small_pres);
    double WL = CL, WR = CR;
    for (int it = 0; it < TWOSHOCK_ITERS; ++it) {
        WL = CL * sqrt(1.0 + gp * (ps / pL - 1.0));
        WR = CR * sqrt(1.0 + gp * (ps / pR - 1.0));
        const double ZL = 2.0 * (WL * WL * WL) / (WL * WL + CL * CL);
        const double ZR = 2.0 * (WR * WR * WR) / (WR * WR + CR * CR);
        const double usL = uL - (ps - pL) / WL;
        const double usR = uR + (ps - pR) / WR;
        ps = ps - (ZL * ZR) * (usR - usL) / (ZL + ZR);
        ps = omax(ps, P->small_pres);
    }
    WL = CL * sqrt(1.0 + gp * (ps / pL - 1.0));
    WR = CR * sqrt(1.0 + gp * (ps / pR - 1.0));
    const double us = ((WL * uL + WR * uR) + (pL - pR)) / (WL + WR);
    const int left = us >= 0.0;
    const double *K = left ? L : R;
    const double WK = left ? WL : WR;
    const double rK = K[0], uK = K[1], pK = K[4];
    const double sgn = left ? -1.0 : 1.0;
    double rs = 1.0 / (1.0 / rK - (ps - pK) / (WK * WK));
    rs = omax(rs, P->small_dens);
    const double cK = sqrt(g * pK / rK), cs = sqrt(g * ps / rs);
    double head, tail;
    if (ps > pK) {
        head = uK + sgn * (WK / rK);
        tail = head;
    } else {
        head = uK + sgn * cK;
        tail = us + sgn * cs;
    }
    double ri, ui, pi;
    if (left ? head >= 0.0 : head <= 0.0) {
        ri = rK; ui = uK; pi = pK;
    } else if (left ? tail <= 0.0 : tail >= 0.0) {
        ri = rs; ui = us; pi = ps;
    } else {
        const double f = (0.0 - tail) / (head - tail);
        ri = rs + f * (rK - rs);
        ui = us + f * (uK - us);
        pi = ps + f * (pK - ps);
    }
    const double vK = K[2], wK = K[3];
    const double m = ri * ui;
    const double Ei = pi * rgm1 + 0.5 * ri * ((ui * ui + vK * vK) + wK * wK);
    Fg[0] = m;
    Fg[1 + d] = m * ui + pi;
    Fg[1 + t1of(d)] = m * vK;
    Fg[1 + t2of(d)] = m * wK;
    Fg[4] = ui * (Ei + pi);
    for (int sp = 0; sp < ns; ++sp) Fg[5 + sp] = m * K[5 + sp];
}

/* The interface flux of the chosen Riemann solver. */
static void riemann_n(const double *L, const double *R, int d, const orc_params *P, double *Fg) {
    if (P->riemann == 1) twoshock_n(L, R, d, P, Fg);
    else hllc_n(L, R, d, P, Fg);
}

/* Five-component entry point of the two-shock flux (pins). */
/* Reflecting walls: a solid wall lets nothing through, so the Riemann
 * problem on a face that lies on a reflecting domain boundary takes the
 * mirror image of the inside state (normal velocity negated, everything else
 * kept) as the outside state, as the PPM codes of the paper's lineage impose
 * on their interface states.  States are permuted primitives (slot 1 normal).
 * f is the box-local face index along d, n the box's cells. */
static void wall_mirror(double *L, double *R, int d, int f, const int n[3], const orc_params *P) {
    const int lo = P->faces_set ? P->face_lo[d] : 0;
    const int hi = P->faces_set ? P->face_hi[d] : n[d];
    const int nv = nvar_of(P);
    if (f == lo && P->bc_lo[d] == BC_REFLECT) {
        for (int m = 0; m < nv; ++m) L[m] = R[m];
        L[1] = -R[1];
    } else if (f == hi && P->bc_hi[d] == BC_REFLECT) {
        for (int m = 0; m < nv; ++m) R[m] = L[m];
        R[1] = -L[1];
    }
}

void orc_twoshock(const double L[5], const double R[5], int d, const orc_params *P, double Fg[5]) {
    orc_params Q = *P;
    Q.nspec = 0;
    twoshock_n(L, R, d, &Q, Fg);
}

/* ------------------------------------------------------ PPM pieces (O5, O6) */

/* Monotonised-central slope (CW84 eq. 1.7-1.8). */
static double mc_slope(double am, double a0, double ap) {
    double dm = a0 - am, dp = ap - a0, dc = 0.5 * (ap - am);
    if (dm * dp > 0.0) {
        double lim = omin(fabs(dc), omin(2.0 * fabs(dm), 2.0 * fabs(dp)));
        return copysign(lim, dc);
    }
    return 0.0;
}

/* Interface value between cells with averages a0, a1 and slopes s0, s1
 * (CW84 eq. 1.6 with the MC slopes). */
static double ppm_edge(double a0, double a1, double s0, double s1) {
    return 0.5 * (a0 + a1) - (1.0 / 6.0) * (s1 - s0);
}

/* Full reconstruction of one cell from the five-cell stencil a[0..4] (cell at
 * a[2]), flattening coefficient phi and contact-steepening weight eta (0: none;
 * CW84 section 1.3): interface values, steepening towards the edge values of
 * the neighbours' linear profiles a[1] + dm a[1] / 2 and a[3] - dm a[3] / 2,
 * flattening, CW84 monotonicity (eq. 1.10), then the parabola's
 * (aL, aR, da, a6). */
static void ppm_cw84(const double a[5], double phi, double eta, double out[4]) {
    const double C6 = 1.0 / 6.0;
    double sm = mc_slope(a[0], a[1], a[2]);
    double s0 = mc_slope(a[1], a[2], a[3]);
    double sp = mc_slope(a[2], a[3], a[4]);
    double ai = a[2];
    double aL = ppm_edge(a[1], a[2], sm, s0);
    double aR = ppm_edge(a[2], a[3], s0, sp);
    if (eta > 0.0) {
        const double aLd = a[1] + 0.5 * sm;
        const double aRd = a[3] - 0.5 * sp;
        aL = aL * (1.0 - eta) + eta * aLd;
        aR = aR * (1.0 - eta) + eta * aRd;
    }
    aL = phi * aL + (1.0 - phi) * ai;
    aR = phi * aR + (1.0 - phi) * ai;
    if ((aR - ai) * (ai - aL) <= 0.0) {
        aL = ai; aR = ai;
    } else {
        double dd = aR - aL;
        double m = ai - 0.5 * (aL + aR);
        if (dd * m > C6 * (dd * dd)) aL = 3.0 * ai - 2.0 * aR;
        else if (-C6 * (dd * dd) > dd * m) aR = 3.0 * ai - 2.0 * aL;
    }
    out[0] = aL;
    out[1] = aR;
    out[2] = aR - aL;
    out[3] = 6.0 * (ai - 0.5 * (aL + aR));
}

void orc_ppm_cell(const double a[5], double phi, double out[4]) { ppm_cw84(a, phi, 0.0, out); }

/* CW84 contact detection for the density stencil r[0..4] (cell at r[2]) with
 * the neighbours' pressures pm, pp: with second differences d2 = (r_{+1} -
 * 2 r + r_{-1}) / 6 of the two neighbours, eta~ = -(d2_{+} - d2_{-}) /
 * (r[3] - r[1]) where the d2 change sign and the jump exceeds 0.01 of the
 * smaller neighbour (else 0), eta = clamp(20 (eta~ - 0.05), 0, 1), and 0 unless
 * the pressure jump is small against the density jump: gamma K0 |r[3] -
 * r[1]| / min(r[3], r[1]) >= |pp - pm| / min(pp, pm), K0 = 0.1. */
double orc_steep_eta(const double r[5], double pm, double pp, double gamma) {
    const double d2m = ((r[2] - 2.0 * r[1]) + r[0]) / 6.0;
    const double d2p = ((r[4] - 2.0 * r[3]) + r[2]) / 6.0;
    const double dr = r[3] - r[1];
    double eta = 0.0;
    if (d2p * d2m < 0.0 && fabs(dr) - 0.01 * omin(fabs(r[3]), fabs(r[1])) > 0.0) {
        const double et = -(d2p - d2m) / dr;
        eta = omax(0.0, omin(20.0 * (et - 0.05), 1.0));
    }
    if (gamma * 0.1 * fabs(dr) / omin(r[3], r[1]) < fabs(pp - pm) / omin(pp, pm)) eta = 0.0;
    return eta;
}

void orc_ppm_cell_steep(const double a[5], double phi, double eta, double out[4]) { ppm_cw84(a, phi, eta, out); }

/* ------------------------------------- extremum-preserving limiter (f3) */

#define CS_C 1.25

/* Sign test of CS08: v if a, b, c (and d) share v's sign, else 0, with the
 * magnitude min(C|b|, C|c|, (C|d|,) |a|). */
static double cs_lim3(double a, double b, double c) {
    if ((a > 0.0 && b > 0.0 && c > 0.0) || (a < 0.0 && b < 0.0 && c < 0.0))
        return copysign(omin(omin(CS_C * fabs(b), CS_C * fabs(c)), fabs(a)), a);
    return 0.0;
}
static double cs_lim4(double a, double b, double c, double d) {
    if ((a > 0.0 && b > 0.0 && c > 0.0 && d > 0.0) || (a < 0.0 && b < 0.0 && c < 0.0 && d < 0.0))
        return copysign(omin(omin(CS_C * fabs(b), CS_C * fabs(c)), omin(CS_C * fabs(d), fabs(a))), a);
    return 0.0;
}

/* CS08 interface value between cells with averages a0, a1 (neighbours am1,
 * a2): the fourth-order value 7/12 (a0 + a1) - 1/12 (am1 + a2); where it is
 * not between a0 and a1, the second difference 3 (a0 - 2 f + a1) is limited
 * against those of the two cells and f = (a0 + a1)/2 - lim/6. */
static double cs_face(double am1, double a0, double a1, double a2) {
    double f = (7.0 / 12.0) * (a0 + a1) - (1.0 / 12.0) * (am1 + a2);
    if ((f - a0) * (a1 - f) < 0.0) {
        const double d2 = 3.0 * ((a0 - 2.0 * f) + a1);
        const double d2L = (am1 - 2.0 * a0) + a1;
        const double d2R = (a0 - 2.0 * a1) + a2;
        f = 0.5 * (a0 + a1) - cs_lim3(d2, d2L, d2R) / 6.0;
    }
    return f;
}

/* PPM parabola of one cell with the CS08 limiter: limited interface values,
 * flattening towards the average, then at a local extremum (of the parabola
 * or of the cell averages) the parabola's second difference -2 (6 a - 3 (aL +
 * aR)) limited against the three neighbouring second differences of the
 * averages (scaling both edges' offsets from the average by lim / d2, flat if
 * d2 = 0); elsewhere the overshoot correction (an edge farther than twice the
 * other from the average is moved to twice, the right edge first). */
static void ppm_cell_cs(const double a[5], double phi, double out[4]) {
    const double ai = a[2];
    double aL = cs_face(a[0], a[1], a[2], a[3]);
    double aR = cs_face(a[1], a[2], a[3], a[4]);
    aL = phi * aL + (1.0 - phi) * ai;
    aR = phi * aR + (1.0 - phi) * ai;
    if ((aR - ai) * (ai - aL) <= 0.0 || (a[1] - ai) * (ai - a[3]) <= 0.0) {
        const double d2 = -2.0 * (6.0 * ai - 3.0 * (aL + aR));
        const double d2C = (a[1] - 2.0 * ai) + a[3];
        const double d2L = (a[0] - 2.0 * a[1]) + ai;
        const double d2R = (ai - 2.0 * a[3]) + a[4];
        if (d2 != 0.0) {
            const double r = cs_lim4(d2, d2L, d2R, d2C) / d2;
            aL = ai + (aL - ai) * r;
            aR = ai + (aR - ai) * r;
        } else {
            aL = ai;
            aR = ai;
        }
    } else {
        if (fabs(aR - ai) >= 2.0 * fabs(aL - ai)) aR = ai - 2.0 * (aL - ai);
        if (fabs(aL - ai) >= 2.0 * fabs(aR - ai)) aL = ai - 2.0 * (aR - ai);
    }
    out[0] = aL;
    out[1] = aR;
    out[2] = aR - aL;
    out[3] = 6.0 * (ai - 0.5 * (aL + aR));
}

/* The parabola of the chosen limiter (eta: contact steepening, CW84 only). */
static void ppm_cell(const double a[5], double phi, int limiter, double eta, double out[4]) {
    if (limiter == 1) ppm_cell_cs(a, phi, out);
    else ppm_cw84(a, phi, eta, out);
}

/* Steepening weight of cell (i, j, k) along the unit vector e from the
 * primitive array q (density comp 0, pressure comp 4). */
static double steep_eta_at(const double *q, const geom *g, const int e[3], int i, int j, int k, double gamma) {
    double r[5];
    for (int s = -2; s <= 2; ++s) r[s + 2] = q[gidx(g, 0, i + s * e[0], j + s * e[1], k + s * e[2])];
    const double pm = q[gidx(g, 4, i - e[0], j - e[1], k - e[2])];
    const double pp = q[gidx(g, 4, i + e[0], j + e[1], k + e[2])];
    return orc_steep_eta(r, pm, pp, gamma);
}

/* Entry point of the CS08 parabola (pins). */
void orc_ppm_cell_cs(const double a[5], double phi, double out[4]) { ppm_cell_cs(a, phi, out); }

/* Average of the parabola over the domain of dependence of the right edge
 * (I+) and of the left edge (I-) for a wave travelling sigma cells per dt. */
double orc_iplus(double aR, double da, double a6, double sig) {
    const double C23 = 2.0 / 3.0;
    return aR - 0.5 * sig * (da - (1.0 - C23 * sig) * a6);
}
double orc_iminus(double aL, double da, double a6, double sig) {
    const double C23 = 2.0 / 3.0;
    return aL + 0.5 * sig * (da + (1.0 - C23 * sig) * a6);
}

/* Characteristic tracing of one cell to t + dt/2 (CW84 section 3, reference
 * state form; Colella 1990).  par[m] = (aL, aR, da, a6) of permuted component
 * m (ncomp >= 5: species after p ride the contact family like the transverse
 * velocities), rho, un, c are the cell's centre values.  Returns the left
 * state of the upper face (qL) and the right state of the lower face (qR),
 * before floors. */
static void trace_cell_n(const double (*par)[4], int ncomp, double rho, double un, double c, double dtdx,
                         double *qL, double *qR) {
    const double lam[3] = {un - c, un, un + c};
    double I[3][MAXV];
    const double csq = c * c;
    /* upper face: waves with lam > 0 reach it */
    for (int nu = 0; nu < 3; ++nu) {
        double sig = fabs(lam[nu]) * dtdx;
        for (int m = 0; m < ncomp; ++m)
            I[nu][m] = lam[nu] > 0.0 ? orc_iplus(par[m][1], par[m][2], par[m][3], sig) : par[m][1];
    }
    {
        const double *ref = I[2];
        double bm = -(rho / (2.0 * c)) * (ref[1] - I[0][1]) + (ref[4] - I[0][4]) / (2.0 * csq);
        double b0 = (ref[0] - I[1][0]) - (ref[4] - I[1][4]) / csq;
        for (int m = 0; m < ncomp; ++m) qL[m] = ref[m];
        if (lam[0] > 0.0) {
            qL[0] = qL[0] - bm;
            qL[1] = qL[1] - bm * (-(c / rho));
            qL[4] = qL[4] - bm * csq;
        }
        if (lam[1] > 0.0) {
            qL[0] = qL[0] - b0;
            for (int m = 2; m < ncomp; ++m) {
                if (m == 4) continue;
                double bt = ref[m] - I[1][m];
                qL[m] = qL[m] - bt;
            }
        }
    }
    /* lower face: waves with lam < 0 reach it */
    for (int nu = 0; nu < 3; ++nu) {
        double sig = fabs(lam[nu]) * dtdx;
        for (int m = 0; m < ncomp; ++m)
            I[nu][m] = lam[nu] < 0.0 ? orc_iminus(par[m][0], par[m][2], par[m][3], sig) : par[m][0];
    }
    {
        const double *ref = I[0];
        double bp = (rho / (2.0 * c)) * (ref[1] - I[2][1]) + (ref[4] - I[2][4]) / (2.0 * csq);
        double b0 = (ref[0] - I[1][0]) - (ref[4] - I[1][4]) / csq;
        for (int m = 0; m < ncomp; ++m) qR[m] = ref[m];
        if (lam[2] < 0.0) {
            qR[0] = qR[0] - bp;
            qR[1] = qR[1] - bp * (c / rho);
            qR[4] = qR[4] - bp * csq;
        }
        if (lam[1] < 0.0) {
            qR[0] = qR[0] - b0;
            for (int m = 2; m < ncomp; ++m) {
                if (m == 4) continue;
                double bt = ref[m] - I[1][m];
                qR[m] = qR[m] - bt;
            }
        }
    }
}

/* Five-component entry point (pins). */
void orc_trace_cell(const double par[5][4], double rho, double un, double c, double dtdx,
                    double qL[5], double qR[5]) {
    trace_cell_n(par, 5, rho, un, c, dtdx, qL, qR);
}

/* ------------------------------------------------------------ flattening (O4) */

/* CW84 appendix: shock indicator f~ of cell i along d with eps = 0.33,
 * omega1 = 0.75, omega2 = 10. */
static double ftilde(const double *q, const geom *g, int d, const int c[3]) {
    int e[3] = {0, 0, 0};
    e[d] = 1;
#define QAT(comp, s) q[gidx(g, comp, c[0] + (s) * e[0], c[1] + (s) * e[1], c[2] + (s) * e[2])]
    double dp1 = QAT(4, 1) - QAT(4, -1);
    double dp2 = QAT(4, 2) - QAT(4, -2);
    double f = 0.0;
    if (fabs(dp1) > 0.33 * omin(QAT(4, 1), QAT(4, -1)) && QAT(1 + d, -1) - QAT(1 + d, 1) > 0.0) {
        f = omin(1.0, omax(0.0, 10.0 * (fabs(dp1) / omax(fabs(dp2), 1e-300) - 0.75)));
    }
    return f;
#undef QAT
}

static double flatten_cell(const double *q, const geom *g, const int c[3]) {
    double phi = 1.0;
    for (int d = 0; d < 3; ++d) {
        int e[3] = {0, 0, 0};
        e[d] = 1;
        double dp1 = q[gidx(g, 4, c[0] + e[0], c[1] + e[1], c[2] + e[2])] -
                     q[gidx(g, 4, c[0] - e[0], c[1] - e[1], c[2] - e[2])];
        int s = dp1 > 0.0 ? 1 : -1;
        int cs[3] = {c[0] - s * e[0], c[1] - s * e[1], c[2] - s * e[2]};
        double fd = omax(ftilde(q, g, d, c), ftilde(q, g, d, cs));
        double v = 1.0 - fd;
        phi = d == 0 ? v : omin(phi, v);
    }
    return phi;
}

/* ---------------------------------------------------------- the box advance */

static double *xalloc(long n) {
    double *p = (double *)malloc(sizeof(double) * (size_t)(n > 0 ? n : 1));
    return p;
}

/* Advance one grown box (ghost cells already filled) by dt.  Unew receives the
 * new valid cells (grown layout; ghosts untouched).  Stage arrays may be
 * supplied through st (for inspection); the rest are allocated here. */
int orc_advance_box(const double *U, const int n[3], const orc_params *P, double dt,
                    double *Unew, long long *cnt, orc_stages *st) {
    const geom G = mkgeom(n);
    const geom *g = &G;
    const long gs = gsize(g), hs = hsize(g);
    orc_stages S;
    memset(&S, 0, sizeof(S));
    if (st) S = *st;
    double *own[32];
    int nown = 0;
#define NEED(ptr, count)                         \
    do {                                         \
        if (!(ptr)) { ptr = xalloc(count); own[nown++] = ptr; } \
    } while (0)
    const int nv = nvar_of(P), nq = 6 + P->nspec;
    NEED(S.q, nq * gs);
    NEED(S.phi, hs);
    for (int d = 0; d < 3; ++d) { NEED(S.ql[d], nv * hs); NEED(S.qr[d], nv * hs); NEED(S.fn[d], nv * hs); NEED(S.ff[d], nv * hs); }
    for (int p = 0; p < 6; ++p) NEED(S.f1[p], nv * hs);
#undef NEED
    for (int i = 0; i < nown; ++i) if (!own[i]) return -2;

    const double dtdx[3] = {dt / P->dx[0], dt / P->dx[1], dt / P->dx[2]};
    double c3[3], c2[3];
    for (int d = 0; d < 3; ++d) { c3[d] = dtdx[d] / 3.0; c2[d] = 0.5 * dtdx[d]; }
    const double hdtg = 0.5 * dt * P->grav_z;
    long long c0 = 0, c1 = 0, c2cnt = 0, c3cnt = 0, c4 = 0;

    /* (a3) primitive state on every grown cell */
#pragma omp parallel for reduction(+ : c0, c1) schedule(static)
    for (int k = -NG; k < n[2] + NG; ++k)
        for (int j = -NG; j < n[1] + NG; ++j)
            for (int i = -NG; i < n[0] + NG; ++i) {
                double Uc[MAXV], q[MAXV + 1];
                long long lc[NCNT] = {0, 0, 0, 0, 0};
                for (int c = 0; c < nv; ++c) Uc[c] = U[gidx(g, c, i, j, k)];
                cons_to_prim_cell(Uc, P, q, lc);
                c0 += lc[0]; c1 += lc[1];
                for (int c = 0; c < nq; ++c) S.q[gidx(g, c, i, j, k)] = q[c];
            }

    /* (a4) flattening coefficient on cells -1..n */
#pragma omp parallel for schedule(static)
    for (int k = -1; k <= n[2]; ++k)
        for (int j = -1; j <= n[1]; ++j)
            for (int i = -1; i <= n[0]; ++i) {
                int c[3] = {i, j, k};
                S.phi[hidx(g, 0, i, j, k)] = flatten_cell(S.q, g, c);
            }

    /* (a5, a6) reconstruction and tracing along each direction, cells -1..n */
    for (int d = 0; d < 3; ++d) {
        const int t1 = t1of(d), t2 = t2of(d);
        int comp[MAXV] = {0, 1 + d, 1 + t1, 1 + t2, 4};
        for (int sp = 0; sp < P->nspec; ++sp) comp[5 + sp] = 6 + sp;
        const int zpos = 1 + (2 - d + 3) % 3; /* permuted position of the z velocity */
#pragma omp parallel for reduction(+ : c2cnt) schedule(static)
        for (int k = -1; k <= n[2]; ++k)
            for (int j = -1; j <= n[1]; ++j)
                for (int i = -1; i <= n[0]; ++i) {
                    int c[3] = {i, j, k};
                    int e[3] = {0, 0, 0};
                    e[d] = 1;
                    double par[MAXV][4], a[5];
                    double phi = S.phi[hidx(g, 0, i, j, k)];
                    const double eta = P->steepen ? steep_eta_at(S.q, g, e, i, j, k, P->gamma) : 0.0;
                    for (int m = 0; m < nv; ++m) {
                        for (int s = -2; s <= 2; ++s)
                            a[s + 2] = S.q[gidx(g, comp[m], i + s * e[0], j + s * e[1], k + s * e[2])];
                        ppm_cell(a, phi, P->limiter, m == 0 ? eta : 0.0, par[m]);
                    }
                    double rho = S.q[gidx(g, 0, i, j, k)];
                    double un = S.q[gidx(g, 1 + d, i, j, k)];
                    double cs = S.q[gidx(g, 5, i, j, k)];
                    double qL[MAXV], qR[MAXV];
                    trace_cell_n((const double (*)[4])par, nv, rho, un, cs, dtdx[d], qL, qR);
                    /* floors, gravity predictor; keep the left state of the
                     * upper face (faces 0..n) and the right state of the lower face */
                    double *both[2] = {qL, qR};
                    const int keep[2] = {c[d] <= n[d] - 1, c[d] >= 0};
                    for (int b = 0; b < 2; ++b) {
                        if (!keep[b]) continue;
                        double *s = both[b];
                        if (s[0] < P->small_dens) { s[0] = P->small_dens; c2cnt++; }
                        if (s[4] < P->small_pres) { s[4] = P->small_pres; c2cnt++; }
                        if (P->grav_z != 0.0) s[zpos] = s[zpos] + hdtg;
                    }
                    if (keep[0])
                        for (int m = 0; m < nv; ++m)
                            S.ql[d][hidx(g, m, i + e[0], j + e[1], k + e[2])] = qL[m];
                    if (keep[1])
                        for (int m = 0; m < nv; ++m) S.qr[d][hidx(g, m, i, j, k)] = qR[m];
                }
    }

    /* (a7) normal fluxes: faces 0..n along d, cells -1..n across */
    for (int d = 0; d < 3; ++d) {
#pragma omp parallel for schedule(static)
        for (int k = -1; k <= n[2]; ++k)
            for (int j = -1; j <= n[1]; ++j)
                for (int i = -1; i <= n[0]; ++i) {
                    int c[3] = {i, j, k};
                    if (c[d] < 0) continue;
                    double L[MAXV], R[MAXV], F[MAXV];
                    for (int m = 0; m < nv; ++m) {
                        L[m] = S.ql[d][hidx(g, m, i, j, k)];
                        R[m] = S.qr[d][hidx(g, m, i, j, k)];
                    }
                    wall_mirror(L, R, d, c[d], n, P);
                    riemann_n(L, R, d, P, F);
                    for (int m = 0; m < nv; ++m) S.fn[d][hidx(g, m, i, j, k)] = F[m];
                }
    }

    /* (a8) stage 1: states along a corrected by dt/(3 dx_b) times the
     * difference of the normal b-fluxes of their owner cell, then HLLC. */
    for (int a = 0; a < 3; ++a)
        for (int which = 0; which < 2; ++which) {
            const int b = which == 0 ? t1of(a) : t2of(a);
            const int cdir = which == 0 ? t2of(a) : t1of(a);
            const int pidx = 2 * a + which;
            long long lfb = 0;
#pragma omp parallel for reduction(+ : lfb) schedule(static)
            for (int k = -1; k <= n[2]; ++k)
                for (int j = -1; j <= n[1]; ++j)
                    for (int i = -1; i <= n[0]; ++i) {
                        int c[3] = {i, j, k};
                        if (c[a] < 0) continue;              /* a faces 0..n */
                        if (c[b] < 0 || c[b] >= n[b]) continue; /* b cells 0..n-1 */
                        (void)cdir;                          /* c cells -1..n */
                        int ea[3] = {0, 0, 0}, eb[3] = {0, 0, 0};
                        ea[a] = 1; eb[b] = 1;
                        double st2[2][MAXV];
                        for (int side = 0; side < 2; ++side) {
                            const double *src = side == 0 ? S.ql[a] : S.qr[a];
                            int o[3] = {i - (side == 0 ? ea[0] : 0), j - (side == 0 ? ea[1] : 0),
                                        k - (side == 0 ? ea[2] : 0)};
                            double s0[MAXV], Uc[MAXV], s1[MAXV];
                            for (int m = 0; m < nv; ++m) s0[m] = src[hidx(g, m, i, j, k)];
                            perm_prim_to_cons(s0, a, P, Uc);
                            for (int m = 0; m < nv; ++m)
                                Uc[m] = Uc[m] - c3[b] * (S.fn[b][hidx(g, m, o[0] + eb[0], o[1] + eb[1], o[2] + eb[2])] -
                                                         S.fn[b][hidx(g, m, o[0], o[1], o[2])]);
                            cons_to_perm_prim(Uc, a, P, s1);
                            if (s1[0] < P->small_dens || s1[4] < P->small_pres) {
                                for (int m = 0; m < nv; ++m) s1[m] = s0[m];
                                lfb++;
                            }
                            for (int m = 0; m < nv; ++m) st2[side][m] = s1[m];
                        }
                        double F[MAXV];
                        wall_mirror(st2[0], st2[1], a, c[a], n, P);
                        riemann_n(st2[0], st2[1], a, P, F);
                        for (int m = 0; m < nv; ++m) S.f1[pidx][hidx(g, m, i, j, k)] = F[m];
                    }
            c3cnt += lfb;
        }

    /* (a9) stage 2: states along a corrected by dt/(2 dx_b) dF^{b|c} and
     * dt/(2 dx_c) dF^{c|b}, with (b, c) the cyclic successors of a; final HLLC. */
    for (int a = 0; a < 3; ++a) {
        const int b = t1of(a), cdir = t2of(a);
        const int pbc = 2 * b + (cdir == t1of(b) ? 0 : 1); /* F^{b|c} */
        const int pcb = 2 * cdir + (b == t1of(cdir) ? 0 : 1); /* F^{c|b} */
        long long lfb = 0;
#pragma omp parallel for reduction(+ : lfb) schedule(static)
        for (int k = 0; k <= n[2]; ++k)
            for (int j = 0; j <= n[1]; ++j)
                for (int i = 0; i <= n[0]; ++i) {
                    int c[3] = {i, j, k};
                    if (c[b] >= n[b] || c[cdir] >= n[cdir]) continue; /* a faces 0..n, others 0..n-1 */
                    int ea[3] = {0, 0, 0}, eb[3] = {0, 0, 0}, ec[3] = {0, 0, 0};
                    ea[a] = 1; eb[b] = 1; ec[cdir] = 1;
                    double st2[2][MAXV];
                    for (int side = 0; side < 2; ++side) {
                        const double *src = side == 0 ? S.ql[a] : S.qr[a];
                        int o[3] = {i - (side == 0 ? ea[0] : 0), j - (side == 0 ? ea[1] : 0),
                                    k - (side == 0 ? ea[2] : 0)};
                        double s0[MAXV], Uc[MAXV], s1[MAXV];
                        for (int m = 0; m < nv; ++m) s0[m] = src[hidx(g, m, i, j, k)];
                        perm_prim_to_cons(s0, a, P, Uc);
                        for (int m = 0; m < nv; ++m)
                            Uc[m] = Uc[m] - c2[b] * (S.f1[pbc][hidx(g, m, o[0] + eb[0], o[1] + eb[1], o[2] + eb[2])] -
                                                     S.f1[pbc][hidx(g, m, o[0], o[1], o[2])]);
                        for (int m = 0; m < nv; ++m)
                            Uc[m] = Uc[m] - c2[cdir] * (S.f1[pcb][hidx(g, m, o[0] + ec[0], o[1] + ec[1], o[2] + ec[2])] -
                                                        S.f1[pcb][hidx(g, m, o[0], o[1], o[2])]);
                        cons_to_perm_prim(Uc, a, P, s1);
                        if (s1[0] < P->small_dens || s1[4] < P->small_pres) {
                            for (int m = 0; m < nv; ++m) s1[m] = s0[m];
                            lfb++;
                        }
                        for (int m = 0; m < nv; ++m) st2[side][m] = s1[m];
                    }
                    double F[MAXV];
                    wall_mirror(st2[0], st2[1], a, c[a], n, P);
                    riemann_n(st2[0], st2[1], a, P, F);
                    for (int m = 0; m < nv; ++m) S.ff[a][hidx(g, m, i, j, k)] = F[m];
                }
        c3cnt += lfb;
    }

    /* (a10) conservative update, gravity corrector and failure check */
    const double gm1 = P->gamma - 1.0;
#pragma omp parallel for reduction(+ : c4) schedule(static)
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                double Un[MAXV];
                for (int m = 0; m < nv; ++m) {
                    double du = dtdx[0] * (S.ff[0][hidx(g, m, i, j, k)] - S.ff[0][hidx(g, m, i + 1, j, k)]);
                    du = du + dtdx[1] * (S.ff[1][hidx(g, m, i, j, k)] - S.ff[1][hidx(g, m, i, j + 1, k)]);
                    du = du + dtdx[2] * (S.ff[2][hidx(g, m, i, j, k)] - S.ff[2][hidx(g, m, i, j, k + 1)]);
                    Un[m] = U[gidx(g, m, i, j, k)] + du;
                }
                if (P->grav_z != 0.0) {
                    Un[3] = Un[3] + hdtg * (U[gidx(g, 0, i, j, k)] + Un[0]);
                    Un[4] = Un[4] + hdtg * (U[gidx(g, 3, i, j, k)] + Un[3]);
                }
                int bad = 0;
                for (int m = 0; m < nv; ++m) if (!isfinite(Un[m])) bad = 1;
                if (Un[0] < P->small_dens) bad = 1;
                if (!bad) {
                    double u = Un[1] / Un[0], v = Un[2] / Un[0], w = Un[3] / Un[0];
                    double ke = 0.5 * Un[0] * ((u * u + v * v) + w * w);
                    if (gm1 * (Un[4] - ke) < P->small_pres) bad = 1;
                }
                c4 += bad;
                for (int m = 0; m < nv; ++m) Unew[gidx(g, m, i, j, k)] = Un[m];
            }

    if (cnt) { cnt[0] += c0; cnt[1] += c1; cnt[2] += c2cnt; cnt[3] += c3cnt; cnt[4] += c4; }
    for (int i = 0; i < nown; ++i) free(own[i]);
    return 0;
}

/* ------------------------------------------------ method of lines (f2) */

/* One Runge-Kutta stage of the MOL variant on a grown box whose ghost cells
 * are filled: with T = Us + dt L(Us), where
 *   dt L(Us) = sum over x, y, z of dt/dx_d (F_lo - F_hi), then the gravity
 *   source dt g (0, 0, 0, rho, rho w) of Us added to rho w and rho E,
 * the valid cells of Uout receive T when U0 is NULL, else the convex
 * combination (1 - c) U0 + c T, evaluated as U0 + c (T - U0) so that a
 * constant state stays exactly constant.
 * The fluxes are HLLC fluxes between the PPM edge values of the two cells of
 * each face (left: the upper edge of the lower cell, right: the lower edge of
 * the upper cell), floored like the CTU face states.  Failures (density or
 * pressure below the floors, non-finite values) of the result are counted. */
int orc_mol_stage(const double *Us, const double *U0, const int n[3], const orc_params *P, double dt,
                  double c, double *Uout, long long *cnt) {
    const geom G = mkgeom(n);
    const geom *g = &G;
    const long gs = gsize(g), hs = hsize(g);
    const int nv = nvar_of(P), nq = 6 + P->nspec;
    double *q = xalloc(nq * gs), *phi = xalloc(hs);
    double *ql[3], *qr[3], *fn[3];
    for (int d = 0; d < 3; ++d) { ql[d] = xalloc(nv * hs); qr[d] = xalloc(nv * hs); fn[d] = xalloc(nv * hs); }
    int bad_alloc = !q || !phi;
    for (int d = 0; d < 3; ++d) bad_alloc |= !ql[d] || !qr[d] || !fn[d];
    if (bad_alloc) return -2;
    long long c0n = 0, c1n = 0, c2n = 0, c4n = 0;

    /* primitive state on every grown cell, flattening on cells -1..n */
#pragma omp parallel for reduction(+ : c0n, c1n) schedule(static)
    for (int k = -NG; k < n[2] + NG; ++k)
        for (int j = -NG; j < n[1] + NG; ++j)
            for (int i = -NG; i < n[0] + NG; ++i) {
                double Uc[MAXV], qc[MAXV + 1];
                long long lc[NCNT] = {0, 0, 0, 0, 0};
                for (int c = 0; c < nv; ++c) Uc[c] = Us[gidx(g, c, i, j, k)];
                cons_to_prim_cell(Uc, P, qc, lc);
                c0n += lc[0]; c1n += lc[1];
                for (int c = 0; c < nq; ++c) q[gidx(g, c, i, j, k)] = qc[c];
            }
#pragma omp parallel for schedule(static)
    for (int k = -1; k <= n[2]; ++k)
        for (int j = -1; j <= n[1]; ++j)
            for (int i = -1; i <= n[0]; ++i) {
                int c[3] = {i, j, k};
                phi[hidx(g, 0, i, j, k)] = flatten_cell(q, g, c);
            }

    /* edge values of the parabolas as face states, cells -1..n */
    for (int d = 0; d < 3; ++d) {
        int comp[MAXV] = {0, 1 + d, 1 + t1of(d), 1 + t2of(d), 4};
        for (int sp = 0; sp < P->nspec; ++sp) comp[5 + sp] = 6 + sp;
#pragma omp parallel for reduction(+ : c2n) schedule(static)
        for (int k = -1; k <= n[2]; ++k)
            for (int j = -1; j <= n[1]; ++j)
                for (int i = -1; i <= n[0]; ++i) {
                    int c[3] = {i, j, k}, e[3] = {0, 0, 0};
                    e[d] = 1;
                    double up[MAXV], dn[MAXV], par[4], a[5];
                    const double ph = phi[hidx(g, 0, i, j, k)];
                    const double eta = P->steepen ? steep_eta_at(q, g, e, i, j, k, P->gamma) : 0.0;
                    for (int m = 0; m < nv; ++m) {
                        for (int s = -2; s <= 2; ++s)
                            a[s + 2] = q[gidx(g, comp[m], i + s * e[0], j + s * e[1], k + s * e[2])];
                        ppm_cell(a, ph, P->limiter, m == 0 ? eta : 0.0, par);
                        up[m] = par[1]; /* upper edge: left state of face c+1 */
                        dn[m] = par[0]; /* lower edge: right state of face c */
                    }
                    if (c[d] <= n[d] - 1) {
                        if (up[0] < P->small_dens) { up[0] = P->small_dens; c2n++; }
                        if (up[4] < P->small_pres) { up[4] = P->small_pres; c2n++; }
                        for (int m = 0; m < nv; ++m) ql[d][hidx(g, m, i + e[0], j + e[1], k + e[2])] = up[m];
                    }
                    if (c[d] >= 0) {
                        if (dn[0] < P->small_dens) { dn[0] = P->small_dens; c2n++; }
                        if (dn[4] < P->small_pres) { dn[4] = P->small_pres; c2n++; }
                        for (int m = 0; m < nv; ++m) qr[d][hidx(g, m, i, j, k)] = dn[m];
                    }
                }
    }

    /* HLLC fluxes on faces 0..n along d, valid cells across */
    for (int d = 0; d < 3; ++d) {
#pragma omp parallel for schedule(static)
        for (int k = 0; k <= n[2]; ++k)
            for (int j = 0; j <= n[1]; ++j)
                for (int i = 0; i <= n[0]; ++i) {
                    int c[3] = {i, j, k};
                    int skip = 0;
                    for (int e = 0; e < 3; ++e) if (e != d && c[e] >= n[e]) skip = 1;
                    if (skip) continue;
                    double L[MAXV], R[MAXV], F[MAXV];
                    for (int m = 0; m < nv; ++m) {
                        L[m] = ql[d][hidx(g, m, i, j, k)];
                        R[m] = qr[d][hidx(g, m, i, j, k)];
                    }
                    wall_mirror(L, R, d, c[d], n, P);
                    riemann_n(L, R, d, P, F);
                    for (int m = 0; m < nv; ++m) fn[d][hidx(g, m, i, j, k)] = F[m];
                }
    }

    /* T = Us + dt L(Us), then the stage combination, failure check */
    const double dtdx[3] = {dt / P->dx[0], dt / P->dx[1], dt / P->dx[2]};
    const double dtg = dt * P->grav_z;
    const double gm1 = P->gamma - 1.0;
#pragma omp parallel for reduction(+ : c4n) schedule(static)
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                double T[MAXV];
                for (int m = 0; m < nv; ++m) {
                    double du = dtdx[0] * (fn[0][hidx(g, m, i, j, k)] - fn[0][hidx(g, m, i + 1, j, k)]);
                    du = du + dtdx[1] * (fn[1][hidx(g, m, i, j, k)] - fn[1][hidx(g, m, i, j + 1, k)]);
                    du = du + dtdx[2] * (fn[2][hidx(g, m, i, j, k)] - fn[2][hidx(g, m, i, j, k + 1)]);
                    T[m] = Us[gidx(g, m, i, j, k)] + du;
                }
                if (P->grav_z != 0.0) {
                    T[3] = T[3] + dtg * Us[gidx(g, 0, i, j, k)];
                    T[4] = T[4] + dtg * Us[gidx(g, 3, i, j, k)];
                }
                if (U0)
                    for (int m = 0; m < nv; ++m) {
                        const double a = U0[gidx(g, m, i, j, k)];
                        T[m] = a + c * (T[m] - a);
                    }
                int bad = 0;
                for (int m = 0; m < nv; ++m) if (!isfinite(T[m])) bad = 1;
                if (T[0] < P->small_dens) bad = 1;
                if (!bad) {
                    double u = T[1] / T[0], v = T[2] / T[0], w = T[3] / T[0];
                    double ke = 0.5 * T[0] * ((u * u + v * v) + w * w);
                    if (gm1 * (T[4] - ke) < P->small_pres) bad = 1;
                }
                c4n += bad;
                for (int m = 0; m < nv; ++m) Uout[gidx(g, m, i, j, k)] = T[m];
            }
    if (cnt) { cnt[0] += c0n; cnt[1] += c1n; cnt[2] += c2n; cnt[4] += c4n; }
    free(q); free(phi);
    for (int d = 0; d < 3; ++d) { free(ql[d]); free(qr[d]); free(fn[d]); }
    return 0;
}

/* ------------------------------------------------------- ghost fill (O11) */

/* Conserved state of the inflow primitive (rho, u, v, w, p). */
static void inflow_cons(const orc_params *P, double *U) {
    const double rgm1 = 1.0 / (P->gamma - 1.0);
    const double *s = P->inflow;
    U[0] = s[0];
    U[1] = s[0] * s[1];
    U[2] = s[0] * s[2];
    U[3] = s[0] * s[3];
    U[4] = s[4] * rgm1 + 0.5 * s[0] * ((s[1] * s[1] + s[2] * s[2]) + s[3] * s[3]);
    for (int sp = 0; sp < P->nspec; ++sp) U[5 + sp] = s[0] * P->inflow_X[sp];
}

/* Fill the ghost cells of a whole-domain grown array: first every ghost cell
 * whose periodic image is a valid cell, then the physical boundaries of the
 * non-periodic directions in the order x, y, z, each over the full grown extent
 * of the other two directions. */
void orc_fill_domain(double *U, const int n[3], const orc_params *P) {
    const geom G = mkgeom(n);
    const geom *g = &G;
    const int nv = nvar_of(P);
#pragma omp parallel for schedule(static)
    for (int k = -NG; k < n[2] + NG; ++k)
        for (int j = -NG; j < n[1] + NG; ++j)
            for (int i = -NG; i < n[0] + NG; ++i) {
                int c[3] = {i, j, k}, s[3];
                int valid = 1, ok = 1;
                for (int d = 0; d < 3; ++d) {
                    if (c[d] >= 0 && c[d] < n[d]) { s[d] = c[d]; continue; }
                    valid = 0;
                    if (P->bc_lo[d] == BC_PERIODIC) s[d] = ((c[d] % n[d]) + n[d]) % n[d];
                    else ok = 0;
                }
                if (valid || !ok) continue;
                for (int m = 0; m < nv; ++m) U[gidx(g, m, i, j, k)] = U[gidx(g, m, s[0], s[1], s[2])];
            }
    for (int d = 0; d < 3; ++d) {
        if (P->bc_lo[d] == BC_PERIODIC) continue;
        for (int side = 0; side < 2; ++side) {
            const int bc = side == 0 ? P->bc_lo[d] : P->bc_hi[d];
            double Uin[MAXV];
            inflow_cons(P, Uin);
            for (int k = -NG; k < n[2] + NG; ++k)
                for (int j = -NG; j < n[1] + NG; ++j)
                    for (int i = -NG; i < n[0] + NG; ++i) {
                        int c[3] = {i, j, k};
                        if (side == 0 ? c[d] >= 0 : c[d] < n[d]) continue;
                        int s[3] = {i, j, k};
                        if (bc == BC_OUTFLOW) s[d] = side == 0 ? 0 : n[d] - 1;
                        else if (bc == BC_REFLECT) s[d] = side == 0 ? -c[d] - 1 : 2 * n[d] - 1 - c[d];
                        for (int m = 0; m < nv; ++m) {
                            double v;
                            if (bc == BC_INFLOW) v = Uin[m];
                            else {
                                v = U[gidx(g, m, s[0], s[1], s[2])];
                                if (bc == BC_REFLECT && m == 1 + d) v = -v;
                            }
                            U[gidx(g, m, i, j, k)] = v;
                        }
                    }
        }
    }
}

/* --------------------------------------------------------------- dt (O2) */

/* Largest signal speed over valid cells: max over cells and directions of
 * (|u_d| + c) / dx_d, using the floored primitive state; for the MOL schemes
 * the max over cells of the sum over directions (x + y) + z. */
double orc_signal_speed(const double *U, const int n[3], const orc_params *P) {
    const geom G = mkgeom(n);
    const geom *g = &G;
    const double rdx[3] = {1.0 / P->dx[0], 1.0 / P->dx[1], 1.0 / P->dx[2]};
    double smax = 0.0;
#pragma omp parallel for reduction(max : smax) schedule(static)
    for (int k = 0; k < n[2]; ++k)
        for (int j = 0; j < n[1]; ++j)
            for (int i = 0; i < n[0]; ++i) {
                double Uc[MAXV], q[MAXV + 1];
                long long lc[NCNT] = {0, 0, 0, 0, 0};
                for (int m = 0; m < nvar_of(P); ++m) Uc[m] = U[gidx(g, m, i, j, k)];
                cons_to_prim_cell(Uc, P, q, lc);
                double sd[3];
                for (int d = 0; d < 3; ++d) sd[d] = (fabs(q[1 + d]) + q[5]) * rdx[d];
                if (P->scheme == 0) {
                    for (int d = 0; d < 3; ++d)
                        if (sd[d] > smax) smax = sd[d];
                } else {
                    double s = (sd[0] + sd[1]) + sd[2];
                    if (s > smax) smax = s;
                }
            }
    return smax;
}

/* One single-level step on a whole-domain grown array: fill ghosts, dt from
 * the CFL condition (unless dt_fixed > 0), advance.  Returns dt via dt_used. */
int orc_step(double *U, const int n[3], const orc_params *P, double dt_fixed, double *dt_used,
             long long *cnt) {
    const geom G = mkgeom(n);
    const long gs = gsize(&G);
    orc_fill_domain(U, n, P);
    double dt = dt_fixed;
    if (!(dt_fixed > 0.0)) {
        double s = orc_signal_speed(U, n, P);
        dt = P->cfl / s;
    }
    const int nv = nvar_of(P);
    double *Un = xalloc(nv * gs);
    if (!Un) return -2;
    memcpy(Un, U, sizeof(double) * nv * gs);
    int rc;
    if (P->scheme == 0) {
        rc = orc_advance_box(U, n, P, dt, Un, cnt, NULL);
    } else {
        /* SSP-RK2: W = U + dt L(U); U' = 1/2 U + 1/2 (W + dt L(W)).
         * SSP-RK3: W1 = U + dt L(U); W2 = 3/4 U + 1/4 (W1 + dt L(W1));
         *          U' = 1/3 U + 2/3 (W2 + dt L(W2)). */
        double *W1 = xalloc(nv * gs), *W2 = xalloc(nv * gs);
        if (!W1 || !W2) return -2;
        memcpy(W1, U, sizeof(double) * nv * gs);
        rc = orc_mol_stage(U, NULL, n, P, dt, 0.0, W1, cnt);
        if (rc == 0) orc_fill_domain(W1, n, P);
        if (P->scheme == 1) {
            if (rc == 0) rc = orc_mol_stage(W1, U, n, P, dt, 0.5, Un, cnt);
        } else {
            memcpy(W2, U, sizeof(double) * nv * gs);
            if (rc == 0) rc = orc_mol_stage(W1, U, n, P, dt, 0.25, W2, cnt);
            if (rc == 0) orc_fill_domain(W2, n, P);
            if (rc == 0) rc = orc_mol_stage(W2, U, n, P, dt, 2.0 / 3.0, Un, cnt);
        }
        free(W1);
        free(W2);
    }
    if (rc == 0) memcpy(U, Un, sizeof(double) * nv * gs);
    free(Un);
    if (dt_used) *dt_used = dt;
    return rc;
}

int orc_run(double *U, const int n[3], const orc_params *P, int nsteps, double dt_fixed,
            double *dts, long long *cnt) {
    for (int s = 0; s < nsteps; ++s) {
        double dt;
        int rc = orc_step(U, n, P, dt_fixed, &dt, cnt);
        if (rc) return rc;
        if (dts) dts[s] = dt;
    }
    return 0;
}
