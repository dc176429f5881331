// pdn_internal.h -- device-side data layout of libpdn (not part of the ABI).
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#define PDN_MAX_PLIES 64
#define PDN_MAX_LAYERS (3 * PDN_MAX_PLIES)
#define PDN_K1_THREADS 256
#define PDN_NTERMS 16         // per-block partials of the element/node kernel
#define PDN_STAGE 64          // rows of the first reduction stage of the books
// element slots: 0.5 m v^n.v~^{n+1}, 0.5 dt v^n.f^n, 0.5 dt v~^{n+1}.f^n,
// sum m d_z^n, secant energy, surrogate points updated by the exact law,
// surrogate points updated in total;
// contact slots (the contact step done in the same pass): reaction sum (3),
// kinetic-energy correction, internal-work correction, contact work on the
// plate, active nodes, nodes at the edge of the search window, released nodes
enum { T_KE = 0, T_WA = 1, T_WB = 2, T_MZ = 3, T_UEL = 4, T_AUX = 5, T_SURN = 6, T_FC = 7, T_KEC = 10, T_WIC = 11,
       T_WCP = 12, T_ACT = 13, T_OVF = 14, T_REL = 15 };

// Per-ply constants in the arithmetic type R of the element kernel.
template <typename R>
struct PlyC {
    R C11, C12, C13, C22, C23, C33, G23, G13, G12;   // undamaged material-frame stiffness
    R iE1, iE2, iE3, mn12, mn13, mn23;               // compliance: 1/E_i and -nu_ij/E_i
    R c, s;                                          // fibre angle about Z
    R cmax;                                          // largest stiffness entry (hourglass, dt)
    R E1, E2, G12v;
    R XT, XC, YT, YC, SL;
    R GXT, GXC, GYT, GYC, GSL;
    R fXT, fGT, fXC, fGC;
    R sa0, ca0, kST, etaT, kEtaL;                    // fracture-plane (alpha0) constants
    R rho;
    int law;                                         // 0 elastic, 1 damage, 2 damage by the surrogate
    int sur;                                         // network of a surrogate ply
    // elastic screen, valid for every element of the ply: E1/XT, E1/XC, 1/YT,
    // 1/SL, 1/ST with the strengths capped at the ply's largest crack band,
    // eta_L of the largest magnitude over its crack-band range (with a margin)
    R scr_kXT, scr_kXC, scr_iYT, scr_iSL, scr_iST, scr_etaL;
    R scr_vmax;                                      // largest element volume the constants hold for
    R kT;                                            // ca0 (sa0 + |etaT| ca0): bound of tau_T^eff / -s22
    // interface on top of this ply
    R KI, Ksh, tauI, GIc, GIIc, eta_bk, GIo;
    R den_onset;                                     // screen of the cohesive law: below onset at any mixity
    R kE1XT, iYT, iSL;                               // surrogate input scales: E1/XT, 1/YT, 1/SL (uncapped)
    // longitudinal shear plasticity: yield stress, plastic modulus Kp G12;
    // plas = 1 on a ply with the exact damage law and Sp > 0
    R Sp, Hp;
    int plas;
};

// Layer table: layer l joins node planes l and l+1.
struct LayerInfo {
    int type;      // 0 bulk, 1 cohesive
    int ply;       // ply (bulk) or ply below (cohesive)
    int index;     // bulk layer index or interface index
    int pad;
    double hz;     // bulk layer thickness (0 for cohesive)
    double ihz;    // 1 / hz (0 for cohesive)
};

// Scalars owned by the contact kernel (striker, books, counters).
struct DevGlobals {
    double c[3], V[3], c0[3];
    double Fprev[3];                 // contact force on the plate found in the last step
    double ms, R, g, dt, phi;
    int64_t step;                    // completed steps
    int64_t hist_cap;
    int32_t first;                   // first contact pass after (re)initialisation
    int32_t flag_unstable, flag_overflow;
    int32_t plain_prev;              // the pass whose element terms the books sum next ran the plain build
    // energy books at the last complete level
    double e_level, e_kep, e_kes, e_wint, e_wgp, e_wgs, e_wc, e_ws, e_uel, ke0;
    double half_int, mz0;            // opening half of the current interval; initial sum m d_z
    double ws_acc, wgs_acc;          // striker works up to the current striker level
    int64_t reset_passes, released, max_passes, active;
    double fallback_gp;              // surrogate: consulted GP updates that the exact law produced
    double sur_gp;                   // surrogate: GP updates on which the network was consulted
    double sur_unscreened;           // surrogate plies stepped by the plain build: GP updates the
                                     // screen did not pass (the exact law produced them)
    unsigned int pad1;
};


// Everything the element/node kernel needs, passed by value.
template <typename R>
struct ElemArgs {
    int nx, ny, K, NL;
    int tiles_x, tiles_y;
    int clamp_lateral;
    int ci0, ci1, cj0, cj1;          // contact candidate window (node columns, half-open)
    double dt, phi, grav;
    R kappa;
    const double *d_in, *v_in;       // state at level n (AoS xyz)
    double *d_out, *v_out;           // predictor for level n+1
    R *r;                            // 4 per bulk GP
    R *rd;                           // 1 per cohesive node pair
    const R *hx, *hy;                // element sizes (nx, ny)
    const R *ihx, *ihy;              // their reciprocals
    const double *mx, *my, *mz;      // separable lumped-mass factors (nx+1, ny+1, K)
    const double *imx, *imy, *imz;   // their reciprocals
    const LayerInfo *layers;         // NL
    const PlyC<R> *ply;              // n_plies
    const uint8_t *bc_bottom;        // (nx+1)(ny+1) fixed-DOF bits of plane 0
    double *fside;                   // 3 per candidate: internal force at level n
    double *partials;                // term-major [PDN_NTERMS][prow], a column per block (written by this pass)
    int prow;                        // term stride of the partials
    // books reduction: a contact pass's first PDN_STAGE tiles sum the element
    // terms of the previous pass into stage rows (PDN_NTERMS apart); contact
    // terms are summed over tiles [wt0, wt1) x [wu0, wu1), which hold every
    // owner of a candidate node
    double *stage;
    int wt0, wt1, wu0, wu1;
    // contact step (Algorithms 1-2) done by this pass on the top plane; 0 for
    // passes that only restart the scheme from a state
    int contact;
    DevGlobals *gl;                  // striker, books, counters
    const double *xs, *ys;           // grid lines (top-plane node positions)
    double ztop;
    const uint8_t *active_in;        // per candidate: active set found in the previous step
    uint8_t *active_out;
    double *vprev, *fcprev;          // per candidate, 3 each: velocity and reaction of the last step
    double *cand;                    // per candidate: corrected displacement and velocity (3 + 3)
    const double *partials_prev;     // block partials of the previous pass
    double *hist;                    // 3 per step
    // constitutive surrogate: packed networks (PlyC::sur selects one), fallback thresholds
    const uint4 *mlp;
    float sur_dmg, sur_res;
    // the build without the network steps surrogate plies (exact law): count
    // their points that the screen does not pass
    int count_sur;
    // 4 per bulk GP (plastic gamma12, gamma13, accumulated, unused); null unless
    // a ply is plastic (then the plastic kernel runs).  Last: a field inserted
    // among the ones above moved their offsets and cost the batched kernel
    // (which copies its arguments from a table) 6 % of its time.
    R *ep;
};

// candidate bookkeeping of the contact step (initialisation, state arrays)
struct ContactArgs {
    double *d, *v;                   // state buffers of the last completed level
    int nx, ny, K;
    int ci0, ci1, cj0, cj1;          // candidate window (node columns, half-open)
    uint8_t *active;                 // 2 per candidate (the two step parities)
    double *vprev, *fcprev;          // per candidate, 3 each
    double *cand;                    // per candidate, 6
};
