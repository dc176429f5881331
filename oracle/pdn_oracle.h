/*
 * pdn_oracle.h -- plain FP64 CPU reference of one explicit PDN impact step.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg may build, load or call this code.  It shares
 * no code, header or table with the HIP library and never reads its output.
 *
 * It follows the paper "Application of the partial Dirichlet-Neumann contact
 * algorithm to simulate low-velocity impact events on composite structures"
 * (Guillamet et al.):
 *   - Section 2.1, Eqs. (1)-(3) and Algorithms 1-2: PDN contact with node
 *     release and repeat-step flag;
 *   - Section 2.2: Tchamwa-Wielgosz explicit scheme (phi = 1 is central
 *     difference) with lumped mass; rigid striker integrated by RK4 (the
 *     printed k3/4 weight is read as k3/3);
 *   - Section 2.3.1, Algorithm 4: intralaminar continuum damage with
 *     plasticity of the longitudinal shear (Table 1's S_p, K_p);
 *   - Section 2.3.2, Algorithm 5: Turon cohesive law on zero-thickness
 *     interface elements with nodal (Newton-Cotes) integration;
 *   - critical time step of Section 2.3.1 / 2.3.2.
 * Units are SI throughout.
 */
#ifndef PDN_ORACLE_H
#define PDN_ORACLE_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct orc_sim orc_sim;

typedef struct {
    int32_t nx, ny, n_plies, elems_per_ply;
    double lx, ly, ply_thickness;
    const double *ply_angle_deg;      /* n_plies, bottom to top */
    int32_t cohesive;                 /* interface layer where adjacent angles differ */
    int32_t bc;                       /* 0 clamped lateral faces, 1 ASTM window + corner clamps, 2 free */
    double window_lx, window_ly, clamp_radius;
    double phi, cfl_safety, gravity, hourglass_kappa;
    const double *node_coords;        /* optional 3*n_nodes reference coordinates */
    int32_t integration;              /* bulk element: 1 (or 0) one point + hourglass control,
                                         8 full 2x2x2 Gauss with its own state per point */
} orc_mesh_desc;

typedef struct {
    double E1, E2, E3, nu12, nu13, nu23, G12, G13, G23, rho;
    int32_t law;                      /* 0 elastic, 1 damage (2 = surrogate, run as 1) */
    double XT, XC, YT, YC, SL, alpha0_deg;
    double GXT, GXC, GYT, GYC, GSL;
    double fXT, fGT, fXC, fGC;
    double KI, tauI, tauII, GIc, GIIc, eta_bk;   /* interface above this ply */
    double Sp, Kp;                    /* longitudinal shear plasticity: yield stress, hardening
                                         modulus / G12 (Sp = 0: none) */
} orc_material;

typedef struct {
    double radius, mass, v0, energy, gap, x0, y0;   /* x0/y0 NaN = plate centre */
} orc_impactor;

/* energy terms at the last complete level (one step behind the state) */
typedef struct {
    double level;          /* time level index L */
    double ke_plate, ke_striker, w_int, w_grav, w_contact_plate, w_striker;
    double d_pdn, ke0, u_el, residual;
} orc_energy;

enum { ORC_DISP = 0, ORC_VEL = 1, ORC_GP_R = 2, ORC_COH_R_IP = 3,
       ORC_COH_R_BY_BOTTOM_NODE = 4, ORC_MASS = 5, ORC_COORDS = 6,
       ORC_FINT = 7, ORC_ACTIVE = 8, ORC_FIX = 9 /* set only: 3*n_nodes 0/1 */,
       ORC_FCONTACT = 10 /* contact force found in the last step */,
       ORC_GP_EP = 11 /* 3 per Gauss point: plastic gamma12, gamma13, accumulated plastic shear */ };

enum { ORC_DMG_FIBRE = 0, ORC_DMG_MATRIX = 1, ORC_DMG_SHEAR = 2, ORC_DMG_COHESIVE = 3,
       ORC_DMG_PROJ_FIBRE = 4, ORC_DMG_PROJ_MATRIX = 5, ORC_DMG_PROJ_COHESIVE = 6 };

/* counts: [n_nodes, n_bulk, n_cohesive, n_planes, n_layers, n_top, n_fixed_dofs] */
int  orc_mesh_counts(const orc_mesh_desc *desc, int64_t out[7]);
orc_sim *orc_create(const orc_mesh_desc *desc);
void orc_destroy(orc_sim *s);
const char *orc_error(const orc_sim *s);
int  orc_set_material(orc_sim *s, int32_t ply, const orc_material *m);
int  orc_set_impactor(orc_sim *s, const orc_impactor *imp);
int  orc_set_threads(orc_sim *s, int32_t n);
/* sensitivity runs: 1 = sum nodal forces in descending element order */
int  orc_set_assembly_order(orc_sim *s, int32_t reverse);
int  orc_step(orc_sim *s, int64_t n);
double orc_dt(orc_sim *s);
int  orc_get(const orc_sim *s, int32_t kind, double *out, int64_t cap);
int  orc_set(orc_sim *s, int32_t kind, const double *in, int64_t n);
int64_t orc_history(const orc_sim *s, double *t, double *f, double *disp, int64_t cap);
int  orc_energies(orc_sim *s, orc_energy *out);
int64_t orc_damage_field(const orc_sim *s, int32_t kind, double *out, int64_t cap);
/* stats: [steps, reset_passes_total, released_total, active_now, max_passes] */
int  orc_stats(const orc_sim *s, int64_t out[5]);
/* impactor: centre[3], velocity[3], contact force on plate[3] */
int  orc_impactor_state(const orc_sim *s, double out[9]);

/* ---- single routines, for pins ---- */
/* hex8 mean-gradient geometry: b[8*3], volume, hourglass gamma[4*8] */
void orc_hex8_geometry(const double X[24], double b[24], double *vol, double gam[32]);
/* element internal force (elastic law) at displacement u; returns strain energy */
double orc_hex8_force_elastic(const double X[24], const double u[24], const orc_material *m,
                              double angle_deg, double kappa, double f[24]);
/* the same with full 2x2x2 Gauss integration (no hourglass control) */
double orc_hex8_force_elastic_full(const double X[24], const double u[24], const orc_material *m,
                                   double angle_deg, double f[24]);
/* lumped mass of one hex8: m[8] */
void orc_hex8_mass(const double X[24], double rho, double m[8]);
/* intralaminar law: eps Voigt (eng. shear), r[4] in/out, lc crack band; sigma out, dmg[5] */
void orc_cdm(const orc_material *m, double lc, const double eps[6], double r[4],
             double sig[6], double dmg[5]);
/* the same with the plastic state ep[3] (in/out: plastic gamma12, gamma13,
 * accumulated plastic shear) of Algorithm 4's first two lines */
void orc_cdm_plastic(const orc_material *m, double lc, const double eps[6], double r[4], double ep[3],
                     double sig[6], double dmg[5]);
/* cohesive law: delta[3] (shear1, shear2, normal), rd in/out; tau[3]; returns D */
double orc_czm(const orc_material *m, const double delta[3], double *rd, double tau[3]);
/* classical RK4 on y' = f(t, y) */
typedef void (*orc_rhs_fn)(double t, const double *y, double *dy, void *ctx);
void orc_rk4(orc_rhs_fn f, void *ctx, double t, double *y, int n, double dt);
/* stable step of the whole mesh */
double orc_stable_dt(orc_sim *s);

#ifdef __cplusplus
}
#endif
#endif
