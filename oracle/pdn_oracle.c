/*
 * pdn_oracle.c -- plain FP64 CPU reference of the explicit PDN impact step.
 *
 * TEST INFRASTRUCTURE ONLY (see pdn_oracle.h).  Deliberately plain: the mesh
 * is held as unstructured connectivity, element geometry is integrated with
 * 2x2x2 Gauss quadrature, every element is evaluated in ascending order and
 * nodal sums follow that order.  Compiled with -ffp-contract=off.
 *
 * Readings of points the paper leaves open are marked "reading:".
 */
#include "pdn_oracle.h"

#include <math.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define MAXPLY 64

/* natural coordinates of the 8 hex nodes: bottom face counter-clockwise seen
 * from +Z starting at (-,-), then the top face */
static const double XI_[8]   = {-1, 1, 1, -1, -1, 1, 1, -1};
static const double ETA_[8]  = {-1, -1, 1, 1, -1, -1, 1, 1};
static const double ZETA_[8] = {-1, -1, -1, -1, 1, 1, 1, 1};

struct orc_sim {
    char err[256];
    /* mesh */
    int nx, ny, P, epp, K, NL, cohesive, bc;
    int ngp;                       /* Gauss points of a bulk element: 1 or 8 */
    int64_t nn, ne, nc, ntop;
    int layer_is_coh[4 * MAXPLY + 8];
    int layer_ply[4 * MAXPLY + 8];
    int *bulk_layer_of;            /* bulk element layer index -> layer */
    double *X;                     /* 3 nn */
    int64_t *conn;                 /* 8 ne */
    int *eply;                     /* ne */
    int64_t *cconn;                /* 8 nc: bottom 4, top 4 */
    int *cply;                     /* nc: ply below the interface */
    unsigned char *fix;            /* 3 nn */
    int64_t *top;                  /* ntop */
    double *mass;                  /* nn */
    /* cached element geometry */
    double *eb, *evol, *egam, *elc_band;   /* 24, 1, 32, 1 per bulk element */
    double *carea;                          /* 4 per cohesive element */
    /* materials */
    orc_material mat[MAXPLY];
    int mat_set[MAXPLY];
    double ang[MAXPLY];
    double phi, safety, grav, kappa, dt;
    int have_imp;
    orc_impactor imp;
    int nthreads;
    int reverse_assembly;          /* sensitivity runs: nodal sums in descending element order */
    /* state at level n */
    int64_t step;                  /* completed steps */
    int needs_init;
    double *d, *v, *a, *fint;
    double *fint_prev;             /* f_int at level n-1 */
    double *fc, *fc_prev;          /* contact force found in the last step / the one before */
    double *v_prev;                /* v at level n-1 */
    double *r;                     /* 4 per Gauss point: 4 ne ngp */
    double *ep;                    /* 3 per Gauss point: plastic gamma12, gamma13, accumulated */
    double *rd;                    /* 4 nc */
    unsigned char *active;         /* nn */
    double *ework;                 /* per-element scratch: 24 forces */
    double *cwork;                 /* per-cohesive scratch: 24 forces */
    double u_el_cur, u_el_prev;
    /* striker */
    double c[3], V[3], c0[3], Fprev[3];
    double ke0;
    /* energy accumulators, last complete level */
    double e_level, e_kep, e_kes, e_wint, e_wgrav_p, e_wgrav_s, e_wc, e_ws;
    double kes_prev_level;         /* striker KE at the level being closed */
    double ws_prev_level, wgs_prev_level;
    /* history */
    double *hist;                  /* 3 per step */
    int64_t hist_cap;
    /* stats */
    int64_t reset_passes, released, max_passes;
};

static int fail(orc_sim *s, const char *msg)
{
    if (s) snprintf(s->err, sizeof s->err, "%s", msg);
    return -1;
}

const char *orc_error(const orc_sim *s) { return s ? s->err : "null"; }

/* ------------------------------------------------------------------------ */
/* small dense helpers                                                       */
/* ------------------------------------------------------------------------ */

static double det3(const double A[3][3])
{
    return A[0][0] * (A[1][1] * A[2][2] - A[1][2] * A[2][1])
         - A[0][1] * (A[1][0] * A[2][2] - A[1][2] * A[2][0])
         + A[0][2] * (A[1][0] * A[2][1] - A[1][1] * A[2][0]);
}

/* signed cofactor matrix, cof = det(A) * A^{-T} */
static void cofactor3(const double A[3][3], double C[3][3])
{
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            int i1 = (i + 1) % 3, i2 = (i + 2) % 3, j1 = (j + 1) % 3, j2 = (j + 2) % 3;
            C[i][j] = A[i1][j1] * A[i2][j2] - A[i1][j2] * A[i2][j1];
        }
}

static void inv3(const double A[3][3], double B[3][3])
{
    double C[3][3];
    cofactor3(A, C);
    double dt = det3(A);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) B[i][j] = C[j][i] / dt;
}

/* ------------------------------------------------------------------------ */
/* hex8: mean (uniform) gradient by 2x2x2 Gauss of the cofactor form,        */
/* Flanagan-Belytschko hourglass base vectors                                */
/* ------------------------------------------------------------------------ */

static void dN_nat(double xi, double eta, double zeta, double dN[8][3])
{
    for (int a = 0; a < 8; ++a) {
        dN[a][0] = 0.125 * XI_[a] * (1 + ETA_[a] * eta) * (1 + ZETA_[a] * zeta);
        dN[a][1] = 0.125 * ETA_[a] * (1 + XI_[a] * xi) * (1 + ZETA_[a] * zeta);
        dN[a][2] = 0.125 * ZETA_[a] * (1 + XI_[a] * xi) * (1 + ETA_[a] * eta);
    }
}

void orc_hex8_geometry(const double X[24], double b[24], double *vol, double gam[32])
{
    const double gp = 1.0 / sqrt(3.0);
    double V = 0;
    for (int i = 0; i < 24; ++i) b[i] = 0;
    for (int g = 0; g < 8; ++g) {
        double xi = (g & 1) ? gp : -gp, eta = (g & 2) ? gp : -gp, zeta = (g & 4) ? gp : -gp;
        double dN[8][3], J[3][3] = {{0}}, C[3][3];
        dN_nat(xi, eta, zeta, dN);
        for (int a = 0; a < 8; ++a)
            for (int I = 0; I < 3; ++I)
                for (int k = 0; k < 3; ++k) J[I][k] += X[3 * a + I] * dN[a][k];
        cofactor3(J, C);
        V += det3(J);
        /* dN_a/dX_I * det J = sum_k cof(J)_{Ik} dN_a/dxi_k */
        for (int a = 0; a < 8; ++a)
            for (int I = 0; I < 3; ++I)
                for (int k = 0; k < 3; ++k) b[3 * a + I] += C[I][k] * dN[a][k];
    }
    for (int i = 0; i < 24; ++i) b[i] /= V;
    *vol = V;
    if (gam) {
        double h[4][8];
        for (int a = 0; a < 8; ++a) {
            h[0][a] = ETA_[a] * ZETA_[a];
            h[1][a] = XI_[a] * ZETA_[a];
            h[2][a] = XI_[a] * ETA_[a];
            h[3][a] = XI_[a] * ETA_[a] * ZETA_[a];
        }
        for (int al = 0; al < 4; ++al) {
            double hx[3] = {0, 0, 0};
            for (int bn = 0; bn < 8; ++bn)
                for (int I = 0; I < 3; ++I) hx[I] += h[al][bn] * X[3 * bn + I];
            for (int a = 0; a < 8; ++a) {
                double s = h[al][a];
                for (int I = 0; I < 3; ++I) s -= hx[I] * b[3 * a + I];
                gam[8 * al + a] = 0.125 * s;
            }
        }
    }
}

void orc_hex8_mass(const double X[24], double rho, double m[8])
{
    const double gp = 1.0 / sqrt(3.0);
    for (int a = 0; a < 8; ++a) m[a] = 0;
    for (int g = 0; g < 8; ++g) {
        double xi = (g & 1) ? gp : -gp, eta = (g & 2) ? gp : -gp, zeta = (g & 4) ? gp : -gp;
        double dN[8][3], J[3][3] = {{0}};
        dN_nat(xi, eta, zeta, dN);
        for (int a = 0; a < 8; ++a)
            for (int I = 0; I < 3; ++I)
                for (int k = 0; k < 3; ++k) J[I][k] += X[3 * a + I] * dN[a][k];
        double dj = det3(J);
        for (int a = 0; a < 8; ++a) {
            double N = 0.125 * (1 + XI_[a] * xi) * (1 + ETA_[a] * eta) * (1 + ZETA_[a] * zeta);
            m[a] += rho * N * dj;
        }
    }
}

/* area of the quad face (4 points, bilinear) and its nodal (Newton-Cotes) weights */
static double quad_area(const double P[4][3], double w[4])
{
    static const double s_[4] = {-1, 1, 1, -1}, t_[4] = {-1, -1, 1, 1};
    const double gp = 1.0 / sqrt(3.0);
    double A = 0;
    if (w) w[0] = w[1] = w[2] = w[3] = 0;
    for (int g = 0; g < 4; ++g) {
        double s = (g & 1) ? gp : -gp, t = (g & 2) ? gp : -gp;
        double xs[3] = {0, 0, 0}, xt[3] = {0, 0, 0};
        for (int a = 0; a < 4; ++a)
            for (int I = 0; I < 3; ++I) {
                xs[I] += 0.25 * s_[a] * (1 + t_[a] * t) * P[a][I];
                xt[I] += 0.25 * t_[a] * (1 + s_[a] * s) * P[a][I];
            }
        double n0 = xs[1] * xt[2] - xs[2] * xt[1];
        double n1 = xs[2] * xt[0] - xs[0] * xt[2];
        double n2 = xs[0] * xt[1] - xs[1] * xt[0];
        double jac = sqrt(n0 * n0 + n1 * n1 + n2 * n2);
        A += jac;
        if (w)
            for (int a = 0; a < 4; ++a) w[a] += 0.25 * (1 + s_[a] * s) * (1 + t_[a] * t) * jac;
    }
    return A;
}

/* ------------------------------------------------------------------------ */
/* constitutive: transversely isotropic compliance (Voigt, engineering shear) */
/* ------------------------------------------------------------------------ */

/* normal 3x3 block of the compliance with damage d1 (fibre) and d2 (matrix) */
static void compliance_normal(const orc_material *m, double d1, double d2, double H[3][3])
{
    H[0][0] = 1.0 / ((1.0 - d1) * m->E1);
    H[1][1] = 1.0 / ((1.0 - d2) * m->E2);
    H[2][2] = 1.0 / m->E3;
    H[0][1] = H[1][0] = -m->nu12 / m->E1;
    H[0][2] = H[2][0] = -m->nu13 / m->E1;
    H[1][2] = H[2][1] = -m->nu23 / m->E2;
}

/* sigma = H(d)^{-1} eps with shear damage d4 on 23 and d6 on 13, 12 */
static void stress_from_compliance(const orc_material *m, double d1, double d2, double d4, double d6,
                                   const double eps[6], double sig[6])
{
    double H[3][3], C[3][3];
    compliance_normal(m, d1, d2, H);
    inv3(H, C);
    for (int i = 0; i < 3; ++i) sig[i] = C[i][0] * eps[0] + C[i][1] * eps[1] + C[i][2] * eps[2];
    sig[3] = (1.0 - d4) * m->G23 * eps[3];
    sig[4] = (1.0 - d6) * m->G13 * eps[4];
    sig[5] = (1.0 - d6) * m->G12 * eps[5];
}

/* largest entry of the undamaged material-frame stiffness */
static double cmax_of(const orc_material *m)
{
    double H[3][3], C[3][3], mx = 0;
    compliance_normal(m, 0, 0, H);
    inv3(H, C);
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j)
            if (fabs(C[i][j]) > mx) mx = fabs(C[i][j]);
    if (m->G23 > mx) mx = m->G23;
    if (m->G13 > mx) mx = m->G13;
    if (m->G12 > mx) mx = m->G12;
    return mx;
}

/* reading (crack band, snap-back): a strength X whose softening would snap
 * back at this element size (l_c X^2 >= 2 E G) is lowered so that
 * l_c X^2 = 0.9 (2 E G); the dissipated energy G / l_c is unchanged. */
static double capped_strength(double X, double E, double G, double lc)
{
    double lim = 0.9 * 2.0 * E * G / lc;
    return (X * X > lim) ? sqrt(lim) : X;
}

/* exponential softening damage of a matrix/shear mode */
static double dmg_expo(double r, double X, double E, double G, double lc)
{
    if (r <= 1.0) return 0.0;
    double A = 2.0 * lc * X * X / (2.0 * E * G - lc * X * X);
    double d = 1.0 - exp(A * (1.0 - r)) / r;
    if (d > 1.0 - 1e-6) d = 1.0 - 1e-6;
    if (d < 0.0) d = 0.0;
    return d;
}

/* bilinear softening damage of a fibre mode at threshold r (strain r*eps0) */
static double dmg_bilinear(double r, double X, double E, double G, double fX, double fG, double lc)
{
    if (r <= 1.0) return 0.0;
    double e0 = X / E, g = G / lc;
    double eB = 2.0 * fG * g / X + fX * e0;
    double eC = 2.0 * (1.0 - fG) * g / (fX * X);
    double e = r * e0, sg;
    if (e <= e0) sg = E * e;
    else if (e <= eB) sg = X + (fX * X - X) * (e - e0) / (eB - e0);
    else if (e <= eC) sg = fX * X * (eC - e) / (eC - eB);
    else sg = 0.0;
    double d = 1.0 - sg / (E * e);
    if (d > 1.0 - 1e-6) d = 1.0 - 1e-6;
    if (d < 0.0) d = 0.0;
    return d;
}

void orc_cdm(const orc_material *m, double lc, const double eps[6], double r[4],
             double sig[6], double dmg[5])
{
    /* Algorithm 4, elastic-damage reading: effective stress, loading
     * functions, thresholds, damage variables, nominal stress. */
    double se[6];
    stress_from_compliance(m, 0, 0, 0, 0, eps, se);       /* effective stress */
    if (m->law == 0) {
        for (int i = 0; i < 6; ++i) sig[i] = se[i];
        if (dmg) for (int i = 0; i < 5; ++i) dmg[i] = 0;
        return;
    }
    double YT = capped_strength(m->YT, m->E2, m->GYT, lc);
    double YC = capped_strength(m->YC, m->E2, m->GYC, lc);
    double SL = capped_strength(m->SL, m->G12, m->GSL, lc);
    double a0 = m->alpha0_deg * M_PI / 180.0;
    double phi1p = (eps[0] > 0 ? eps[0] : 0) * m->E1 / m->XT;   /* max-strain criterion */
    double phi1m = (eps[0] < 0 ? -eps[0] : 0) * m->E1 / m->XC;
    double s22 = se[1];
    double tauL = sqrt(se[5] * se[5] + se[4] * se[4]);
    double phi2p, phi2m = 0.0;
    double etaL = -SL * cos(2 * a0) / (YC * cos(a0) * cos(a0));
    if (s22 >= 0) {
        phi2p = sqrt((s22 / YT) * (s22 / YT) + (tauL / SL) * (tauL / SL));
    } else {
        double t = tauL + etaL * s22;
        phi2p = (t > 0 ? t : 0) / SL;
        double ST = YC * cos(a0) * (sin(a0) + cos(a0) / tan(2 * a0));
        double etaT = -1.0 / tan(2 * a0);
        double th = atan(tauL / (-s22 * sin(a0)));
        double tte = -s22 * cos(a0) * (sin(a0) - etaT * cos(a0) * cos(th));
        double tle = cos(a0) * (tauL + etaL * s22 * cos(a0) * sin(th));
        if (tte < 0) tte = 0;
        if (tle < 0) tle = 0;
        phi2m = sqrt((tte / ST) * (tte / ST) + (tle / SL) * (tle / SL));
    }
    if (phi1p > r[0]) r[0] = phi1p;
    if (phi1m > r[1]) r[1] = phi1m;
    if (phi2p > r[2]) r[2] = phi2p;
    if (phi2m > r[3]) r[3] = phi2m;
    if (r[1] > r[0]) r[0] = r[1];
    if (r[3] > r[2]) r[2] = r[3];
    double d1p = dmg_bilinear(r[0], m->XT, m->E1, m->GXT, m->fXT, m->fGT, lc);
    double d1m = dmg_bilinear(r[1], m->XC, m->E1, m->GXC, m->fXC, m->fGC, lc);
    double d2p = dmg_expo(r[2], YT, m->E2, m->GYT, lc);
    double d2m = dmg_expo(r[3], YC, m->E2, m->GYC, lc);
    double d6 = dmg_expo(r[2], SL, m->G12, m->GSL, lc);
    /* crack closure (tension or compression variable by the sign of the
     * effective stress) acts on the normal terms only; the transverse shear
     * keeps the tensile matrix damage, so that no closed strain cycle
     * returns energy (the model is thermodynamically consistent, Sec. 2.3.1) */
    double d1 = se[0] >= 0 ? d1p : d1m;
    double d2 = se[1] >= 0 ? d2p : d2m;
    stress_from_compliance(m, d1, d2, d2p, d6, eps, sig);
    if (dmg) { dmg[0] = d1p; dmg[1] = d1m; dmg[2] = d2p; dmg[3] = d2m; dmg[4] = d6; }
}

/* Algorithm 4, first line (reading): plasticity of the longitudinal shear in
 * effective stress.  The shear plane through the fibre is isotropic
 * (G13 = G12), so the yield function is on tau_L = |(tau12, tau13)|:
 *   F = tau_L - (S_p + H abar),  H = K_p G12 (linear isotropic hardening on
 * the accumulated plastic shear abar).  Where F > 0, the radial return along
 * the trial stress direction n: dl = F / (G12 + H), gamma_p += dl n,
 * abar += dl.  ep = {gamma12_p, gamma13_p, abar}. */
static void plastic_return(const orc_material *m, const double eps[6], double ep[3])
{
    double G = m->G12, H = m->Kp * m->G12;
    double t12 = G * (eps[5] - ep[0]), t13 = G * (eps[4] - ep[1]);
    double tL = sqrt(t12 * t12 + t13 * t13);
    double F = tL - (m->Sp + H * ep[2]);
    if (!(F > 0)) return;
    double dl = F / (G + H);
    ep[0] += dl * t12 / tL;
    ep[1] += dl * t13 / tL;
    ep[2] += dl;
}

void orc_cdm_plastic(const orc_material *m, double lc, const double eps[6], double r[4], double ep[3],
                     double sig[6], double dmg[5])
{
    /* Algorithm 4: plastic strains, effective elastic strains, then the
     * damage law on the elastic strains */
    double ee[6] = {eps[0], eps[1], eps[2], eps[3], eps[4], eps[5]};
    if (m->law != 0 && m->Sp > 0) {
        plastic_return(m, eps, ep);
        ee[5] = eps[5] - ep[0];
        ee[4] = eps[4] - ep[1];
    }
    orc_cdm(m, lc, ee, r, sig, dmg);
}

double orc_czm(const orc_material *m, const double dl[3], double *rd, double tau[3])
{
    /* Algorithm 5 with Turon-2018 variables; reading: shear penalty
     * K_sh = K_I (G_Ic/G_IIc) (tau_II/tau_I)^2, normal = reference +Z. */
    double KI = m->KI;
    double Ksh = KI * (m->GIc / m->GIIc) * (m->tauII / m->tauI) * (m->tauII / m->tauI);
    double sh2 = dl[0] * dl[0] + dl[1] * dl[1];
    double d3p = dl[2] > 0 ? dl[2] : 0;
    double den = Ksh * sh2 + KI * d3p * d3p;
    double B = den > 0 ? Ksh * sh2 / den : 0.0;
    double KB = (1 - B) * KI + B * Ksh;
    double lam = sqrt((KI * d3p * d3p + Ksh * sh2) / KB);
    double Gc = m->GIc + (m->GIIc - m->GIc) * pow(B, m->eta_bk);
    double GIo = m->tauI * m->tauI / (2 * KI);
    double lo = sqrt(2 * GIo * Gc / (m->GIc * KB));
    double lc = 2 * Gc / (KB * lo);
    double H = (lam - lo) / (lc - lo);
    if (H > 1) H = 1;
    if (H > *rd) *rd = H;
    double r = *rd;
    double D = r * lc / (r * lc + (1 - r) * lo);
    tau[0] = (1 - D) * Ksh * dl[0];
    tau[1] = (1 - D) * Ksh * dl[1];
    tau[2] = dl[2] >= 0 ? (1 - D) * KI * dl[2] : KI * dl[2];
    return D;
}

/* ------------------------------------------------------------------------ */
/* element internal force                                                     */
/* ------------------------------------------------------------------------ */

/* f = V sum_J (F S)_{iJ} b_{aJ} + hourglass; updates r (if law) ;
 * returns the element's secant energy 0.5 V sigma.eps + 0.5 k q.q */
/* Response at one point of displacement gradient H (= F - I): Green strain,
 * material frame, law (thresholds r, updated), back to the global frame and
 * the nominal stress Pn = F S.  Returns the secant energy density S:E/2. */
static double point_response(const double H[3][3], const orc_material *m, double angle_deg, double lc,
                             double *r, double *ep, double Pn[3][3])
{
    /* the Green strain E = (F^T F - I)/2 is evaluated as (H + H^T + H^T H)/2,
     * the same tensor without the cancellation of 1 + small - 1 */
    double F[3][3];
    for (int i = 0; i < 3; ++i)
        for (int J = 0; J < 3; ++J) F[i][J] = H[i][J] + ((i == J) ? 1.0 : 0.0);
    double E[3][3];
    for (int I = 0; I < 3; ++I)
        for (int J = 0; J < 3; ++J) {
            double s = 0;
            for (int k = 0; k < 3; ++k) s += H[k][I] * H[k][J];
            E[I][J] = 0.5 * (H[I][J] + H[J][I] + s);
        }
    /* material axes: fibre at angle theta about Z; Q rows = material axes */
    double th = angle_deg * M_PI / 180.0, c = cos(th), s = sin(th);
    double Q[3][3] = {{c, s, 0}, {-s, c, 0}, {0, 0, 1}};
    double Em[3][3], T[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double t = 0;
            for (int k = 0; k < 3; ++k) t += Q[i][k] * E[k][j];
            T[i][j] = t;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double t = 0;
            for (int k = 0; k < 3; ++k) t += T[i][k] * Q[j][k];
            Em[i][j] = t;
        }
    double eps[6] = {Em[0][0], Em[1][1], Em[2][2], 2 * Em[1][2], 2 * Em[0][2], 2 * Em[0][1]};
    double sg[6];
    double rloc[4] = {1, 1, 1, 1}, eploc[3] = {0, 0, 0};
    double *epp = ep ? ep : eploc;
    orc_cdm_plastic(m, lc, eps, r ? r : rloc, epp, sg, NULL);
    if (m->law != 0 && m->Sp > 0) {           /* recoverable energy: the elastic strains */
        eps[5] -= epp[0];
        eps[4] -= epp[1];
    }
    double Sm[3][3] = {{sg[0], sg[5], sg[4]}, {sg[5], sg[1], sg[3]}, {sg[4], sg[3], sg[2]}};
    double S[3][3];
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double t = 0;
            for (int k = 0; k < 3; ++k) t += Q[k][i] * Sm[k][j];
            T[i][j] = t;
        }
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
            double t = 0;
            for (int k = 0; k < 3; ++k) t += T[i][k] * Q[k][j];
            S[i][j] = t;
        }
    for (int i = 0; i < 3; ++i)
        for (int J = 0; J < 3; ++J) {
            double t = 0;
            for (int K = 0; K < 3; ++K) t += F[i][K] * S[K][J];
            Pn[i][J] = t;
        }
    double w = 0;
    for (int k = 0; k < 6; ++k) w += sg[k] * eps[k];
    return 0.5 * w;
}

static double hex8_force(const double *b, double V, const double *gam, const double *u,
                         const orc_material *m, double angle_deg, double kappa, double lc,
                         double *r, double *ep, double f[24])
{
    /* one point: H = sum_a u_a (x) b_a with the mean gradients b */
    double H[3][3], Pn[3][3];
    for (int i = 0; i < 3; ++i)
        for (int J = 0; J < 3; ++J) {
            double s = 0.0;
            for (int a = 0; a < 8; ++a) s += u[3 * a + i] * b[3 * a + J];
            H[i][J] = s;
        }
    double wd = point_response(H, m, angle_deg, lc, r, ep, Pn);
    for (int a = 0; a < 8; ++a)
        for (int i = 0; i < 3; ++i) {
            double t = 0;
            for (int J = 0; J < 3; ++J) t += Pn[i][J] * b[3 * a + J];
            f[3 * a + i] = V * t;
        }
    /* Flanagan-Belytschko stiffness hourglass on total displacement */
    double bb = 0;
    for (int i = 0; i < 24; ++i) bb += b[i] * b[i];
    double khg = kappa * cmax_of(m) * V * bb / 3.0;
    double q[4][3];
    double ehg = 0;
    for (int al = 0; al < 4; ++al)
        for (int i = 0; i < 3; ++i) {
            double t = 0;
            for (int a = 0; a < 8; ++a) t += gam[8 * al + a] * u[3 * a + i];
            q[al][i] = t;
            ehg += 0.5 * khg * t * t;
        }
    for (int a = 0; a < 8; ++a)
        for (int i = 0; i < 3; ++i) {
            double t = 0;
            for (int al = 0; al < 4; ++al) t += gam[8 * al + a] * q[al][i];
            f[3 * a + i] += khg * t;
        }
    return V * wd + ehg;
}

/* Full integration (the paper's element, Section 2): 2x2x2 Gauss points of
 * weight 1; at each, the Jacobian of the reference map, dN_a/dX by cofactors,
 * H = sum_a u_a (x) dN_a/dX, the law with the point's own thresholds
 * r[4 g .. 4 g + 3], and f_a += det J Pn dN_a/dX.  No hourglass control. */
static double hex8_force_full(const double X[24], const double *u, const orc_material *m, double angle_deg,
                              double lc, double *r, double *ep, double f[24])
{
    const double gp = 1.0 / sqrt(3.0);
    double energy = 0;
    for (int i = 0; i < 24; ++i) f[i] = 0;
    for (int g = 0; g < 8; ++g) {
        double xi = (g & 1) ? gp : -gp, eta = (g & 2) ? gp : -gp, zeta = (g & 4) ? gp : -gp;
        double dN[8][3], J[3][3] = {{0}}, C[3][3];
        dN_nat(xi, eta, zeta, dN);
        for (int a = 0; a < 8; ++a)
            for (int I = 0; I < 3; ++I)
                for (int k = 0; k < 3; ++k) J[I][k] += X[3 * a + I] * dN[a][k];
        cofactor3(J, C);
        double dJ = det3(J);
        double B[8][3];
        for (int a = 0; a < 8; ++a)
            for (int I = 0; I < 3; ++I) {
                double t = 0;
                for (int k = 0; k < 3; ++k) t += C[I][k] * dN[a][k];
                B[a][I] = t / dJ;
            }
        double H[3][3], Pn[3][3];
        for (int i = 0; i < 3; ++i)
            for (int I = 0; I < 3; ++I) {
                double t = 0;
                for (int a = 0; a < 8; ++a) t += u[3 * a + i] * B[a][I];
                H[i][I] = t;
            }
        energy += dJ * point_response(H, m, angle_deg, lc, r ? r + 4 * g : NULL, ep ? ep + 3 * g : NULL, Pn);
        for (int a = 0; a < 8; ++a)
            for (int i = 0; i < 3; ++i) {
                double t = 0;
                for (int I = 0; I < 3; ++I) t += Pn[i][I] * B[a][I];
                f[3 * a + i] += dJ * t;
            }
    }
    return energy;
}

double orc_hex8_force_elastic(const double X[24], const double u[24], const orc_material *m,
                              double angle_deg, double kappa, double f[24])
{
    double b[24], V, gam[32];
    orc_hex8_geometry(X, b, &V, gam);
    orc_material me = *m;
    me.law = 0;
    return hex8_force(b, V, gam, u, &me, angle_deg, kappa, cbrt(V), NULL, NULL, f);
}

double orc_hex8_force_elastic_full(const double X[24], const double u[24], const orc_material *m,
                                   double angle_deg, double f[24])
{
    double b[24], V;
    orc_hex8_geometry(X, b, &V, NULL);
    orc_material me = *m;
    me.law = 0;
    return hex8_force_full(X, u, &me, angle_deg, cbrt(V), NULL, NULL, f);
}

/* ------------------------------------------------------------------------ */
/* RK4 (Section 2.2.2; weights k1/6 + k2/3 + k3/3 + k4/6)                     */
/* ------------------------------------------------------------------------ */

void orc_rk4(orc_rhs_fn f, void *ctx, double t, double *y, int n, double dt)
{
    double k1[16], k2[16], k3[16], k4[16], yt[16];
    f(t, y, k1, ctx);
    for (int i = 0; i < n; ++i) { k1[i] *= dt; yt[i] = y[i] + 0.5 * k1[i]; }
    f(t + 0.5 * dt, yt, k2, ctx);
    for (int i = 0; i < n; ++i) { k2[i] *= dt; yt[i] = y[i] + 0.5 * k2[i]; }
    f(t + 0.5 * dt, yt, k3, ctx);
    for (int i = 0; i < n; ++i) { k3[i] *= dt; yt[i] = y[i] + k3[i]; }
    f(t + dt, yt, k4, ctx);
    for (int i = 0; i < n; ++i) {
        k4[i] *= dt;
        y[i] = y[i] + k1[i] / 6.0 + k2[i] / 3.0 + k3[i] / 3.0 + k4[i] / 6.0;
    }
}

/* ------------------------------------------------------------------------ */
/* mesh generation                                                            */
/* ------------------------------------------------------------------------ */

static int build_layers(const orc_mesh_desc *d, int *is_coh, int *ply, int *NL_out)
{
    int NL = 0;
    for (int p = 0; p < d->n_plies; ++p) {
        for (int e = 0; e < d->elems_per_ply; ++e) { is_coh[NL] = 0; ply[NL] = p; ++NL; }
        if (p + 1 < d->n_plies && d->cohesive && d->ply_angle_deg[p] != d->ply_angle_deg[p + 1]) {
            is_coh[NL] = 1; ply[NL] = p; ++NL;
        }
    }
    *NL_out = NL;
    return 0;
}

int orc_mesh_counts(const orc_mesh_desc *d, int64_t out[7])
{
    if (d->n_plies < 1 || d->n_plies > MAXPLY || d->elems_per_ply < 1 || d->nx < 1 || d->ny < 1)
        return -1;
    int is_coh[4 * MAXPLY + 8], ply[4 * MAXPLY + 8], NL;
    build_layers(d, is_coh, ply, &NL);
    int64_t ncol = (int64_t)d->nx * d->ny, nplane = (int64_t)(d->nx + 1) * (d->ny + 1);
    int nb = 0, ncl = 0;
    for (int l = 0; l < NL; ++l) { if (is_coh[l]) ++ncl; else ++nb; }
    out[0] = nplane * (NL + 1);
    out[1] = ncol * nb;
    out[2] = ncol * ncl;
    out[3] = NL + 1;
    out[4] = NL;
    out[5] = nplane;
    out[6] = 0;
    return 0;
}

static int64_t nid(const orc_sim *s, int i, int j, int k)
{
    return (int64_t)i + (int64_t)(s->nx + 1) * ((int64_t)j + (int64_t)(s->ny + 1) * k);
}

static int window_index(int n, double len, double win)
{
    double q = n * (len - win) / (2.0 * len);
    return (int)floor(q + 0.5 + 1e-9);
}

orc_sim *orc_create(const orc_mesh_desc *d)
{
    orc_sim *s = (orc_sim *)calloc(1, sizeof(orc_sim));
    int64_t cnt[7];
    if (orc_mesh_counts(d, cnt) != 0) { free(s); return NULL; }
    if (d->integration != 0 && d->integration != 1 && d->integration != 8) { free(s); return NULL; }
    s->ngp = d->integration == 8 ? 8 : 1;
    s->nx = d->nx; s->ny = d->ny; s->P = d->n_plies; s->epp = d->elems_per_ply;
    build_layers(d, s->layer_is_coh, s->layer_ply, &s->NL);
    s->K = s->NL + 1;
    s->nn = cnt[0]; s->ne = cnt[1]; s->nc = cnt[2]; s->ntop = cnt[5];
    s->cohesive = d->cohesive; s->bc = d->bc;
    s->phi = d->phi; s->safety = d->cfl_safety; s->grav = d->gravity; s->kappa = d->hourglass_kappa;
    s->nthreads = 1;
    for (int p = 0; p < s->P; ++p) s->ang[p] = d->ply_angle_deg[p];
    int64_t nn = s->nn, ne = s->ne, nc = s->nc;
    s->X = (double *)calloc(3 * nn, sizeof(double));
    s->conn = (int64_t *)calloc(8 * (ne ? ne : 1), sizeof(int64_t));
    s->eply = (int *)calloc(ne ? ne : 1, sizeof(int));
    s->cconn = (int64_t *)calloc(8 * (nc ? nc : 1), sizeof(int64_t));
    s->cply = (int *)calloc(nc ? nc : 1, sizeof(int));
    s->fix = (unsigned char *)calloc(3 * nn, 1);
    s->top = (int64_t *)calloc(s->ntop, sizeof(int64_t));
    s->mass = (double *)calloc(nn, sizeof(double));
    /* plane heights */
    double *zk = (double *)calloc(s->K, sizeof(double));
    double hz = d->ply_thickness / d->elems_per_ply;
    for (int l = 0; l < s->NL; ++l) zk[l + 1] = zk[l] + (s->layer_is_coh[l] ? 0.0 : hz);
    for (int k = 0; k < s->K; ++k)
        for (int j = 0; j <= s->ny; ++j)
            for (int i = 0; i <= s->nx; ++i) {
                int64_t n = nid(s, i, j, k);
                if (d->node_coords) {
                    s->X[3 * n] = d->node_coords[3 * n];
                    s->X[3 * n + 1] = d->node_coords[3 * n + 1];
                    s->X[3 * n + 2] = d->node_coords[3 * n + 2];
                } else {
                    s->X[3 * n] = d->lx * i / d->nx;
                    s->X[3 * n + 1] = d->ly * j / d->ny;
                    s->X[3 * n + 2] = zk[k];
                }
            }
    free(zk);
    /* elements: i fastest, then j, then layer (bulk and cohesive numbered separately) */
    int64_t eb = 0, ec = 0;
    for (int l = 0; l < s->NL; ++l)
        for (int j = 0; j < s->ny; ++j)
            for (int i = 0; i < s->nx; ++i) {
                int64_t nodes[8] = {nid(s, i, j, l), nid(s, i + 1, j, l), nid(s, i + 1, j + 1, l),
                                    nid(s, i, j + 1, l), nid(s, i, j, l + 1), nid(s, i + 1, j, l + 1),
                                    nid(s, i + 1, j + 1, l + 1), nid(s, i, j + 1, l + 1)};
                if (s->layer_is_coh[l]) {
                    memcpy(&s->cconn[8 * ec], nodes, sizeof nodes);
                    s->cply[ec] = s->layer_ply[l];
                    ++ec;
                } else {
                    memcpy(&s->conn[8 * eb], nodes, sizeof nodes);
                    s->eply[eb] = s->layer_ply[l];
                    ++eb;
                }
            }
    for (int j = 0, t = 0; j <= s->ny; ++j)
        for (int i = 0; i <= s->nx; ++i) s->top[t++] = nid(s, i, j, s->K - 1);
    /* boundary conditions (reading of Section 3.2 / workload statements) */
    if (d->bc == 2) {
        /* free: no support */
    } else if (d->bc == 0) {
        for (int k = 0; k < s->K; ++k)
            for (int j = 0; j <= s->ny; ++j)
                for (int i = 0; i <= s->nx; ++i)
                    if (i == 0 || i == s->nx || j == 0 || j == s->ny) {
                        int64_t n = nid(s, i, j, k);
                        s->fix[3 * n] = s->fix[3 * n + 1] = s->fix[3 * n + 2] = 1;
                    }
    } else {
        int ilo = window_index(s->nx, d->lx, d->window_lx), ihi = s->nx - ilo;
        int jlo = window_index(s->ny, d->ly, d->window_ly), jhi = s->ny - jlo;
        double r2 = d->clamp_radius * d->clamp_radius * (1.0 + 1e-9);
        for (int j = 0; j <= s->ny; ++j)
            for (int i = 0; i <= s->nx; ++i) {
                int64_t n = nid(s, i, j, 0);
                int on_x = (i == ilo || i == ihi) && j >= jlo && j <= jhi;
                int on_y = (j == jlo || j == jhi) && i >= ilo && i <= ihi;
                if (on_x || on_y) s->fix[3 * n + 2] = 1;
                int ci[2] = {ilo, ihi}, cj[2] = {jlo, jhi};
                for (int a = 0; a < 2; ++a)
                    for (int bq = 0; bq < 2; ++bq) {
                        int64_t cn = nid(s, ci[a], cj[bq], 0);
                        double dx = s->X[3 * n] - s->X[3 * cn], dy = s->X[3 * n + 1] - s->X[3 * cn + 1];
                        if (dx * dx + dy * dy <= r2) s->fix[3 * n] = s->fix[3 * n + 1] = s->fix[3 * n + 2] = 1;
                    }
            }
    }
    /* cached geometry */
    s->eb = (double *)calloc(24 * (ne ? ne : 1), sizeof(double));
    s->evol = (double *)calloc(ne ? ne : 1, sizeof(double));
    s->egam = (double *)calloc(32 * (ne ? ne : 1), sizeof(double));
    s->elc_band = (double *)calloc(ne ? ne : 1, sizeof(double));
    s->carea = (double *)calloc(4 * (nc ? nc : 1), sizeof(double));
    for (int64_t e = 0; e < ne; ++e) {
        double Xe[24];
        for (int a = 0; a < 8; ++a)
            for (int I = 0; I < 3; ++I) Xe[3 * a + I] = s->X[3 * s->conn[8 * e + a] + I];
        orc_hex8_geometry(Xe, &s->eb[24 * e], &s->evol[e], &s->egam[32 * e]);
        s->elc_band[e] = cbrt(s->evol[e]);
    }
    for (int64_t e = 0; e < nc; ++e) {
        double Pq[4][3];
        for (int a = 0; a < 4; ++a)
            for (int I = 0; I < 3; ++I) Pq[a][I] = s->X[3 * s->cconn[8 * e + a] + I];
        quad_area(Pq, &s->carea[4 * e]);
    }
    /* state */
    s->d = (double *)calloc(3 * nn, sizeof(double));
    s->v = (double *)calloc(3 * nn, sizeof(double));
    s->a = (double *)calloc(3 * nn, sizeof(double));
    s->fint = (double *)calloc(3 * nn, sizeof(double));
    s->fint_prev = (double *)calloc(3 * nn, sizeof(double));
    s->fc = (double *)calloc(3 * nn, sizeof(double));
    s->fc_prev = (double *)calloc(3 * nn, sizeof(double));
    s->v_prev = (double *)calloc(3 * nn, sizeof(double));
    s->r = (double *)calloc(4 * s->ngp * (ne ? ne : 1), sizeof(double));
    s->ep = (double *)calloc(3 * s->ngp * (ne ? ne : 1), sizeof(double));
    s->rd = (double *)calloc(4 * (nc ? nc : 1), sizeof(double));
    s->active = (unsigned char *)calloc(nn, 1);
    s->ework = (double *)calloc(24 * (ne ? ne : 1), sizeof(double));
    s->cwork = (double *)calloc(24 * (nc ? nc : 1), sizeof(double));
    for (int64_t i = 0; i < 4 * s->ngp * ne; ++i) s->r[i] = 1.0;
    s->needs_init = 1;
    return s;
}

void orc_destroy(orc_sim *s)
{
    if (!s) return;
    void *p[] = {s->bulk_layer_of, s->X, s->conn, s->eply, s->cconn, s->cply, s->fix, s->top,
                 s->mass, s->eb, s->evol, s->egam, s->elc_band, s->carea, s->d, s->v, s->a,
                 s->fint, s->fint_prev, s->fc, s->fc_prev, s->v_prev, s->r, s->ep, s->rd, s->active,
                 s->ework, s->cwork, s->hist};
    for (size_t i = 0; i < sizeof p / sizeof p[0]; ++i) free(p[i]);
    free(s);
}

int orc_set_assembly_order(orc_sim *s, int32_t reverse)
{
    s->reverse_assembly = reverse != 0;
    return 0;
}

int orc_set_threads(orc_sim *s, int32_t n)
{
    s->nthreads = n < 1 ? 1 : n;
    return 0;
}

static int all_materials_set(const orc_sim *s)
{
    for (int p = 0; p < s->P; ++p)
        if (!s->mat_set[p]) return 0;
    return 1;
}

static void compute_mass(orc_sim *s)
{
    for (int64_t n = 0; n < s->nn; ++n) s->mass[n] = 0;
    for (int64_t e = 0; e < s->ne; ++e) {
        double Xe[24], me[8];
        for (int a = 0; a < 8; ++a)
            for (int I = 0; I < 3; ++I) Xe[3 * a + I] = s->X[3 * s->conn[8 * e + a] + I];
        orc_hex8_mass(Xe, s->mat[s->eply[e]].rho, me);
        for (int a = 0; a < 8; ++a) s->mass[s->conn[8 * e + a]] += me[a];
    }
}

int orc_set_material(orc_sim *s, int32_t ply, const orc_material *m)
{
    if (ply < -1 || ply >= s->P) return fail(s, "ply index out of range");
    if (m->E1 <= 0 || m->E2 <= 0 || m->E3 <= 0 || m->rho <= 0 || m->G12 <= 0 || m->G13 <= 0 || m->G23 <= 0)
        return fail(s, "elastic constants must be positive");
    double lcmax = 0;
    for (int64_t e = 0; e < s->ne; ++e)
        if ((ply < 0 || s->eply[e] == ply) && s->elc_band[e] > lcmax) lcmax = s->elc_band[e];
    if (m->Sp < 0 || m->Kp < 0) return fail(s, "plasticity needs S_p >= 0 and K_p >= 0");
    if (m->Sp > 0 && m->law != 0 && m->G13 != m->G12)
        return fail(s, "longitudinal shear plasticity needs an isotropic shear plane (G13 = G12)");
    if (m->law != 0) {
        double ls[2] = {m->XT, m->XC}, gs[2] = {m->GXT, m->GXC}, fx[2] = {m->fXT, m->fXC}, fg[2] = {m->fGT, m->fGC};
        for (int k = 0; k < 2; ++k) {
            double e0 = ls[k] / m->E1, g = gs[k] / lcmax;
            double eB = 2 * fg[k] * g / ls[k] + fx[k] * e0, eC = 2 * (1 - fg[k]) * g / (fx[k] * ls[k]);
            if (!(eB > e0 && eC > eB)) return fail(s, "fibre bilinear softening not ordered at this element size");
        }
    }
    for (int p = 0; p < s->P; ++p)
        if (ply < 0 || p == ply) { s->mat[p] = *m; s->mat_set[p] = 1; }
    if (all_materials_set(s)) compute_mass(s);
    s->dt = 0;
    return 0;
}

int orc_set_impactor(orc_sim *s, const orc_impactor *imp)
{
    if (imp->radius <= 0 || imp->mass <= 0) return fail(s, "impactor radius and mass must be positive");
    s->imp = *imp;
    double h = 0;
    for (int64_t t = 0; t < s->ntop; ++t) if (s->X[3 * s->top[t] + 2] > h) h = s->X[3 * s->top[t] + 2];
    double lx = s->X[3 * nid(s, s->nx, 0, 0)], ly = s->X[3 * nid(s, 0, s->ny, 0) + 1];
    double x0 = isnan(imp->x0) ? 0.5 * lx : imp->x0, y0 = isnan(imp->y0) ? 0.5 * ly : imp->y0;
    double v0 = imp->energy > 0 ? sqrt(2.0 * imp->energy / imp->mass) : imp->v0;
    if (!s->have_imp || s->step == 0) {
        s->c0[0] = x0; s->c0[1] = y0; s->c0[2] = h + imp->radius + imp->gap;
        memcpy(s->c, s->c0, sizeof s->c);
        s->Fprev[0] = s->Fprev[1] = s->Fprev[2] = 0;
        s->ke0 = 0.5 * imp->mass * v0 * v0;
        s->e_kes = s->ke0;
    }
    /* impact direction e = -Z; lateral striker motion is constrained */
    s->V[0] = 0; s->V[1] = 0; s->V[2] = -v0;
    s->have_imp = 1;
    return 0;
}

/* ------------------------------------------------------------------------ */
/* stable time step (Section 2.3.1 / 2.3.2 readings)                          */
/* ------------------------------------------------------------------------ */

double orc_stable_dt(orc_sim *s)
{
    double dtb = INFINITY, dtc = INFINITY;
    for (int64_t e = 0; e < s->ne; ++e) {
        const orc_material *m = &s->mat[s->eply[e]];
        /* characteristic length V / largest face area */
        static const int faces[6][4] = {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4},
                                        {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}};
        double Amax = 0;
        for (int f = 0; f < 6; ++f) {
            double Pq[4][3];
            for (int a = 0; a < 4; ++a)
                for (int I = 0; I < 3; ++I) Pq[a][I] = s->X[3 * s->conn[8 * e + faces[f][a]] + I];
            double A = quad_area(Pq, NULL);
            if (A > Amax) Amax = A;
        }
        double lc = s->evol[e] / Amax;
        double t = lc * sqrt(m->rho / cmax_of(m));
        if (t < dtb) dtb = t;
    }
    if (s->nc > 0) {
        /* node-pair spring: tributary area summed over the interface elements */
        double *Ap = (double *)calloc(s->nn, sizeof(double));
        int64_t *partner = (int64_t *)malloc(s->nn * sizeof(int64_t));
        double *kip = (double *)calloc(s->nn, sizeof(double));
        for (int64_t n = 0; n < s->nn; ++n) partner[n] = -1;
        for (int64_t e = 0; e < s->nc; ++e)
            for (int a = 0; a < 4; ++a) {
                int64_t nb = s->cconn[8 * e + a], nt = s->cconn[8 * e + 4 + a];
                Ap[nb] += s->carea[4 * e + a];
                partner[nb] = nt;
                kip[nb] = s->mat[s->cply[e]].KI;
            }
        for (int64_t n = 0; n < s->nn; ++n)
            if (partner[n] >= 0 && Ap[n] > 0) {
                double mb = s->mass[n], mt = s->mass[partner[n]];
                double meff = mb * mt / (mb + mt);
                double t = 2.0 * sqrt(meff / (kip[n] * Ap[n]));
                if (t < dtc) dtc = t;
            }
        free(Ap); free(partner); free(kip);
    }
    if (s->nc > 0) return s->safety / sqrt(1.0 / (dtb * dtb) + 1.0 / (dtc * dtc));
    return s->safety * dtb;
}

double orc_dt(orc_sim *s)
{
    if (s->dt == 0 && all_materials_set(s)) s->dt = orc_stable_dt(s);
    return s->dt;
}

/* ------------------------------------------------------------------------ */
/* internal force of the whole mesh at s->d; updates damage state             */
/* ------------------------------------------------------------------------ */

static void internal_force(orc_sim *s)
{
    int64_t ne = s->ne, nc = s->nc;
    double uel = 0;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(s->nthreads) reduction(+ : uel)
#endif
    for (int64_t e = 0; e < ne; ++e) {
        double ue[24];
        for (int a = 0; a < 8; ++a)
            for (int i = 0; i < 3; ++i) ue[3 * a + i] = s->d[3 * s->conn[8 * e + a] + i];
        int p = s->eply[e];
        if (s->ngp == 8) {
            double Xe[24];
            for (int a = 0; a < 8; ++a)
                for (int i = 0; i < 3; ++i) Xe[3 * a + i] = s->X[3 * s->conn[8 * e + a] + i];
            uel += hex8_force_full(Xe, ue, &s->mat[p], s->ang[p], s->elc_band[e], &s->r[32 * e],
                                   &s->ep[24 * e], &s->ework[24 * e]);
        } else {
            uel += hex8_force(&s->eb[24 * e], s->evol[e], &s->egam[32 * e], ue, &s->mat[p], s->ang[p],
                              s->kappa, s->elc_band[e], &s->r[4 * e], &s->ep[3 * e], &s->ework[24 * e]);
        }
    }
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(s->nthreads) reduction(+ : uel)
#endif
    for (int64_t e = 0; e < nc; ++e) {
        const orc_material *m = &s->mat[s->cply[e]];
        for (int a = 0; a < 4; ++a) {
            int64_t nb = s->cconn[8 * e + a], nt = s->cconn[8 * e + 4 + a];
            double dl[3] = {s->d[3 * nt] - s->d[3 * nb], s->d[3 * nt + 1] - s->d[3 * nb + 1],
                            s->d[3 * nt + 2] - s->d[3 * nb + 2]};
            double tau[3];
            orc_czm(m, dl, &s->rd[4 * e + a], tau);
            double A = s->carea[4 * e + a];
            for (int i = 0; i < 3; ++i) {
                s->cwork[24 * e + 3 * a + i] = -A * tau[i];          /* bottom node */
                s->cwork[24 * e + 12 + 3 * a + i] = A * tau[i];      /* top node */
            }
            uel += 0.5 * A * (tau[0] * dl[0] + tau[1] * dl[1] + tau[2] * dl[2]);
        }
    }
    /* assembly in ascending element order (descending for a sensitivity run:
     * the same sums in another order, to measure how the problem amplifies
     * rounding) */
    for (int64_t n = 0; n < 3 * s->nn; ++n) s->fint[n] = 0;
    for (int64_t k = 0; k < ne; ++k) {
        int64_t e = s->reverse_assembly ? ne - 1 - k : k;
        for (int a = 0; a < 8; ++a)
            for (int i = 0; i < 3; ++i) s->fint[3 * s->conn[8 * e + a] + i] += s->ework[24 * e + 3 * a + i];
    }
    for (int64_t k = 0; k < nc; ++k) {
        int64_t e = s->reverse_assembly ? nc - 1 - k : k;
        for (int a = 0; a < 4; ++a)
            for (int i = 0; i < 3; ++i) {
                s->fint[3 * s->cconn[8 * e + a] + i] += s->cwork[24 * e + 3 * a + i];
                s->fint[3 * s->cconn[8 * e + 4 + a] + i] += s->cwork[24 * e + 12 + 3 * a + i];
            }
    }
    s->u_el_cur = uel;
}

static void accel_from_force(orc_sim *s)
{
    for (int64_t n = 0; n < s->nn; ++n)
        for (int i = 0; i < 3; ++i) {
            double fe = (i == 2) ? -s->mass[n] * s->grav : 0.0;    /* gravity along e = -Z */
            s->a[3 * n + i] = s->fix[3 * n + i] ? 0.0 : (fe - s->fint[3 * n + i]) / s->mass[n];
        }
}

/* ------------------------------------------------------------------------ */
/* striker: point mass, force frozen over the step, RK4                       */
/* ------------------------------------------------------------------------ */

typedef struct { double g, m, F; } striker_ctx;

static void striker_rhs(double t, const double *y, double *dy, void *ctx)
{
    (void)t;
    const striker_ctx *c = (const striker_ctx *)ctx;
    dy[0] = y[3]; dy[1] = y[4]; dy[2] = y[5];
    /* lateral DOFs constrained; along e = -Z: m a = m g - F_c . e */
    dy[3] = 0; dy[4] = 0;
    dy[5] = -(c->g - c->F / c->m);
}

/* ------------------------------------------------------------------------ */
/* one explicit PDN step (Algorithms 1 and 2)                                 */
/* ------------------------------------------------------------------------ */

static void init_level(orc_sim *s)
{
    internal_force(s);
    accel_from_force(s);
    s->needs_init = 0;
}

static void hist_push(orc_sim *s, double t, double F, double disp)
{
    if (s->step >= s->hist_cap) {
        int64_t cap = s->hist_cap ? 2 * s->hist_cap : 1024;
        while (cap <= s->step) cap *= 2;
        s->hist = (double *)realloc(s->hist, 3 * cap * sizeof(double));
        s->hist_cap = cap;
    }
    s->hist[3 * s->step] = t;
    s->hist[3 * s->step + 1] = F;
    s->hist[3 * s->step + 2] = disp;
}

static void one_step(orc_sim *s)
{
    int64_t nn = s->nn;
    double dt = s->dt, phi = s->phi;
    const double R = s->imp.radius, ms = s->imp.mass, g = s->grav;
    /* rigid body first (Gauss-Seidel): force from the plate's previous step */
    double kes_before = 0.5 * ms * (s->V[0] * s->V[0] + s->V[1] * s->V[1] + s->V[2] * s->V[2]);
    double cz_before = s->c[2];
    {
        striker_ctx ctx = {g, ms, -s->Fprev[2]};       /* F_c . e with e = -Z */
        double y[6] = {s->c[0], s->c[1], s->c[2], s->V[0], s->V[1], s->V[2]};
        orc_rk4(striker_rhs, &ctx, s->step * dt, y, 6, dt);
        s->c[0] = y[0]; s->c[1] = y[1]; s->c[2] = y[2];
        s->V[0] = y[3]; s->V[1] = y[4]; s->V[2] = y[5];
    }
    double dXe = -(s->c[2] - cz_before);                /* displacement along e */
    double ws_inc = (-s->Fprev[2]) * dXe;
    double wgs_inc = ms * g * dXe;
    /* plate predictor (TW with contact correction zero) */
    double *vold = s->v_prev;
    memcpy(vold, s->v, 3 * nn * sizeof(double));
    for (int64_t k = 0; k < 3 * nn; ++k) {
        if (s->fix[k]) { s->v[k] = 0.0; continue; }
        double dn = s->d[k] + dt * s->v[k] + phi * dt * dt * s->a[k];
        s->v[k] = s->v[k] + dt * s->a[k];
        s->d[k] = dn;
    }
    /* contact: candidates are top-surface nodes; active set persists */
    {   /* fc_prev <- force found in the previous step; fc <- this step's */
        double *t = s->fc_prev; s->fc_prev = s->fc; s->fc = t;
    }
    double *fcn = s->fc;
    for (int64_t k = 0; k < 3 * nn; ++k) fcn[k] = 0;
    for (int64_t t = 0; t < s->ntop; ++t) {
        int64_t n = s->top[t];
        double x[3], rv[3];
        for (int i = 0; i < 3; ++i) { x[i] = s->X[3 * n + i] + s->d[3 * n + i]; rv[i] = x[i] - s->c[i]; }
        double dist = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
        double gap = dist - R;
        int hemi = (-rv[2]) >= 0.0;                     /* (x - c) . e >= 0 */
        if (gap < 0.0 && hemi) s->active[n] = 1;
    }
    int passes = 0;
    int64_t released = 0;
    for (;;) {
        int kfl_reset = 0;
        ++passes;
        for (int64_t t = 0; t < s->ntop; ++t) {
            int64_t n = s->top[t];
            for (int i = 0; i < 3; ++i) fcn[3 * n + i] = 0;
            if (!s->active[n]) continue;
            double rv[3];
            for (int i = 0; i < 3; ++i) rv[i] = s->X[3 * n + i] + s->d[3 * n + i] - s->c[i];
            double dist = sqrt(rv[0] * rv[0] + rv[1] * rv[1] + rv[2] * rv[2]);
            double nv[3];
            if (dist > 0) for (int i = 0; i < 3; ++i) nv[i] = rv[i] / dist;
            else { nv[0] = 0; nv[1] = 0; nv[2] = -1; }
            double gap = dist - R;
            double fn = 0;
            for (int i = 0; i < 3; ++i) {
                double ddi = s->fix[3 * n + i] ? 0.0 : -gap * nv[i];
                fcn[3 * n + i] = s->mass[n] * ddi / (phi * dt * dt);
                fn += fcn[3 * n + i] * nv[i];
            }
            if (fn < 0.0) {                              /* adhesion node (Eq. 2 violated) */
                s->active[n] = 0;
                for (int i = 0; i < 3; ++i) fcn[3 * n + i] = 0;
                kfl_reset = 1;
                ++released;
            }
        }
        if (!kfl_reset || passes >= 8) break;
    }
    s->reset_passes += passes;
    s->released += released;
    if (passes > s->max_passes) s->max_passes = passes;
    /* apply the Dirichlet correction: da = f_c / m */
    double Fc[3] = {0, 0, 0};
    for (int64_t n = 0; n < nn; ++n) {
        if (!s->active[n]) continue;
        for (int i = 0; i < 3; ++i) {
            double da = fcn[3 * n + i] / s->mass[n];
            s->v[3 * n + i] += dt * da;
            s->d[3 * n + i] += phi * dt * dt * da;
            Fc[i] += fcn[3 * n + i];
        }
    }
    /* energies of level L = step (previous level), now complete */
    {
        double kep = 0, wint = 0, wg = 0, wc = 0;
        for (int64_t n = 0; n < nn; ++n)
            for (int i = 0; i < 3; ++i) {
                int64_t k = 3 * n + i;
                kep += 0.5 * s->mass[n] * vold[k] * s->v[k];
                if (s->step >= 1) {
                    double fe = (i == 2) ? -s->mass[n] * g : 0.0;
                    wint += 0.5 * dt * vold[k] * (s->fint_prev[k] + s->fint[k]);
                    wg += dt * vold[k] * fe;
                    wc += 0.5 * dt * vold[k] * (s->fc_prev[k] + fcn[k]);
                }
            }
        s->e_level = (double)s->step;
        s->e_kep = kep;
        s->e_wint += wint;
        s->e_wgrav_p += wg;
        s->e_wc += wc;
        s->e_kes = kes_before;
        s->e_ws = s->ws_prev_level;
        s->e_wgrav_s = s->wgs_prev_level;
        s->u_el_prev = s->u_el_cur;
        s->ws_prev_level += ws_inc;
        s->wgs_prev_level += wgs_inc;
    }
    /* element pass at the new configuration */
    memcpy(s->fint_prev, s->fint, 3 * nn * sizeof(double));
    internal_force(s);
    accel_from_force(s);
    s->Fprev[0] = Fc[0]; s->Fprev[1] = Fc[1]; s->Fprev[2] = Fc[2];
    /* history of step s = step+1: time, contact force along e, striker displacement along e */
    hist_push(s, (s->step + 1) * dt, -Fc[2], -(s->c[2] - s->c0[2]));
    s->step += 1;
}

int orc_step(orc_sim *s, int64_t n)
{
    if (!all_materials_set(s)) return fail(s, "material not set for every ply");
    if (!s->have_imp) return fail(s, "impactor not set");
    if (s->dt == 0) s->dt = orc_stable_dt(s);
    if (s->needs_init) init_level(s);
    for (int64_t k = 0; k < n; ++k) {
        one_step(s);
        for (int64_t i = 0; i < 3 * s->nn; ++i)
            if (!isfinite(s->d[i])) return fail(s, "non-finite displacement");
    }
    return 0;
}

/* ------------------------------------------------------------------------ */
/* accessors                                                                  */
/* ------------------------------------------------------------------------ */

int orc_get(const orc_sim *s, int32_t kind, double *out, int64_t cap)
{
    int64_t n;
    switch (kind) {
    case ORC_DISP: n = 3 * s->nn; if (cap < n) return -1; memcpy(out, s->d, n * 8); return 0;
    case ORC_VEL: n = 3 * s->nn; if (cap < n) return -1; memcpy(out, s->v, n * 8); return 0;
    case ORC_FINT: n = 3 * s->nn; if (cap < n) return -1; memcpy(out, s->fint, n * 8); return 0;
    case ORC_FCONTACT: n = 3 * s->nn; if (cap < n) return -1; memcpy(out, s->fc, n * 8); return 0;
    case ORC_GP_R: n = 4 * s->ngp * s->ne; if (cap < n) return -1; memcpy(out, s->r, n * 8); return 0;
    case ORC_GP_EP: n = 3 * s->ngp * s->ne; if (cap < n) return -1; memcpy(out, s->ep, n * 8); return 0;
    case ORC_COH_R_IP: n = 4 * s->nc; if (cap < n) return -1; memcpy(out, s->rd, n * 8); return 0;
    case ORC_MASS: n = s->nn; if (cap < n) return -1; memcpy(out, s->mass, n * 8); return 0;
    case ORC_COORDS: n = 3 * s->nn; if (cap < n) return -1; memcpy(out, s->X, n * 8); return 0;
    case ORC_ACTIVE:
        if (cap < s->nn) return -1;
        for (int64_t i = 0; i < s->nn; ++i) out[i] = s->active[i];
        return 0;
    case ORC_COH_R_BY_BOTTOM_NODE:
        if (cap < s->nn) return -1;
        for (int64_t i = 0; i < s->nn; ++i) out[i] = 0;
        for (int64_t e = 0; e < s->nc; ++e)
            for (int a = 0; a < 4; ++a) out[s->cconn[8 * e + a]] = s->rd[4 * e + a];
        return 0;
    }
    return -1;
}

int orc_set(orc_sim *s, int32_t kind, const double *in, int64_t n)
{
    switch (kind) {
    case ORC_DISP: if (n != 3 * s->nn) return -1; memcpy(s->d, in, n * 8); break;
    case ORC_VEL: if (n != 3 * s->nn) return -1; memcpy(s->v, in, n * 8); break;
    case ORC_GP_R: if (n != 4 * s->ngp * s->ne) return -1; memcpy(s->r, in, n * 8); break;
    case ORC_GP_EP: if (n != 3 * s->ngp * s->ne) return -1; memcpy(s->ep, in, n * 8); break;
    case ORC_COH_R_IP: if (n != 4 * s->nc) return -1; memcpy(s->rd, in, n * 8); break;
    case ORC_COH_R_BY_BOTTOM_NODE:
        if (n != s->nn) return -1;
        for (int64_t e = 0; e < s->nc; ++e)
            for (int a = 0; a < 4; ++a) s->rd[4 * e + a] = in[s->cconn[8 * e + a]];
        break;
    case ORC_FIX:
        if (n != 3 * s->nn) return -1;
        for (int64_t k = 0; k < n; ++k) s->fix[k] = in[k] != 0.0;
        s->dt = 0;
        break;
    default: return -1;
    }
    /* fixed DOFs stay at rest */
    for (int64_t k = 0; k < 3 * s->nn; ++k)
        if (s->fix[k]) { s->d[k] = 0; s->v[k] = 0; }
    s->needs_init = 1;
    return 0;
}

int64_t orc_history(const orc_sim *s, double *t, double *f, double *disp, int64_t cap)
{
    int64_t n = s->step < cap ? s->step : cap;
    for (int64_t i = 0; i < n; ++i) {
        if (t) t[i] = s->hist[3 * i];
        if (f) f[i] = s->hist[3 * i + 1];
        if (disp) disp[i] = s->hist[3 * i + 2];
    }
    return s->step;
}

int orc_energies(orc_sim *s, orc_energy *o)
{
    o->level = s->e_level;
    o->ke_plate = s->e_kep;
    o->ke_striker = s->e_kes;
    o->w_int = s->e_wint;
    o->w_grav = s->e_wgrav_p + s->e_wgrav_s;
    o->w_contact_plate = s->e_wc;
    o->w_striker = s->e_ws;
    o->d_pdn = s->e_ws - s->e_wc;
    o->ke0 = s->ke0;
    o->u_el = s->u_el_prev;
    o->residual = o->ke_plate + o->ke_striker + o->w_int + o->d_pdn - (o->ke0 + o->w_grav);
    return 0;
}

int orc_stats(const orc_sim *s, int64_t out[5])
{
    int64_t act = 0;
    for (int64_t n = 0; n < s->nn; ++n) act += s->active[n];
    out[0] = s->step; out[1] = s->reset_passes; out[2] = s->released; out[3] = act; out[4] = s->max_passes;
    return 0;
}

int orc_impactor_state(const orc_sim *s, double out[9])
{
    for (int i = 0; i < 3; ++i) { out[i] = s->c[i]; out[3 + i] = s->V[i]; out[6 + i] = s->Fprev[i]; }
    return 0;
}

/* damage fields: per bulk element (i fastest, j, layer), per cohesive element
 * (max over its 4 points), or projected nx*ny (max over thickness) */
int64_t orc_damage_field(const orc_sim *s, int32_t kind, double *out, int64_t cap)
{
    int64_t ncol = (int64_t)s->nx * s->ny;
    int proj = kind >= ORC_DMG_PROJ_FIBRE;
    int base = proj ? (kind == ORC_DMG_PROJ_COHESIVE ? ORC_DMG_COHESIVE : kind - 4) : kind;
    int64_t n = proj ? ncol : (base == ORC_DMG_COHESIVE ? s->nc : s->ne);
    if (cap < n) return -n;
    if (proj) for (int64_t i = 0; i < n; ++i) out[i] = 0;
    if (base == ORC_DMG_COHESIVE) {
        for (int64_t e = 0; e < s->nc; ++e) {
            const orc_material *m = &s->mat[s->cply[e]];
            double mx = 0;
            for (int a = 0; a < 4; ++a) {
                /* D of the stored threshold at the current mode mix */
                double r = s->rd[4 * e + a];
                int64_t nb = s->cconn[8 * e + a], nt = s->cconn[8 * e + 4 + a];
                double dl[3] = {s->d[3 * nt] - s->d[3 * nb], s->d[3 * nt + 1] - s->d[3 * nb + 1],
                                s->d[3 * nt + 2] - s->d[3 * nb + 2]};
                double rr = r, tau[3];
                double D = orc_czm(m, dl, &rr, tau);
                (void)tau;
                if (D > mx) mx = D;
            }
            if (proj) { int64_t c = e % ncol; if (mx > out[c]) out[c] = mx; }
            else out[e] = mx;
        }
        return n;
    }
    for (int64_t e = 0; e < s->ne; ++e) {
        const orc_material *m = &s->mat[s->eply[e]];
        double val = 0;
        /* largest over the element's Gauss points */
        for (int g = 0; g < s->ngp && m->law != 0; ++g) {
            double lc = s->elc_band[e], vg;
            const double *r = &s->r[4 * (s->ngp * e + g)];
            if (base == ORC_DMG_FIBRE) {
                double a = dmg_bilinear(r[0], m->XT, m->E1, m->GXT, m->fXT, m->fGT, lc);
                double b = dmg_bilinear(r[1], m->XC, m->E1, m->GXC, m->fXC, m->fGC, lc);
                vg = a > b ? a : b;
            } else if (base == ORC_DMG_MATRIX) {
                double a = dmg_expo(r[2], capped_strength(m->YT, m->E2, m->GYT, lc), m->E2, m->GYT, lc);
                double b = dmg_expo(r[3], capped_strength(m->YC, m->E2, m->GYC, lc), m->E2, m->GYC, lc);
                vg = a > b ? a : b;
            } else {
                vg = dmg_expo(r[2], capped_strength(m->SL, m->G12, m->GSL, lc), m->G12, m->GSL, lc);
            }
            if (vg > val) val = vg;
        }
        if (proj) { int64_t c = e % ncol; if (val > out[c]) out[c] = val; }
        else out[e] = val;
    }
    return n;
}
