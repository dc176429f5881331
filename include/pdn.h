/*
 * pdn.h -- C-ABI of the MI355X explicit PDN impact step (libpdn.so).
 *
 * The library advances a low-velocity impact of a rigid hemispherical striker
 * on a laminated plate with the partial Dirichlet-Neumann (PDN) contact
 * method of Guillamet et al., "Application of the partial Dirichlet-Neumann
 * contact algorithm to simulate low-velocity impact events on composite
 * structures": explicit Tchamwa-Wielgosz / central-difference integration
 * with lumped mass (Section 2.2.1), a point-mass striker advanced by RK4
 * with the contact force frozen over the step (Section 2.2.2), kinematic
 * contact with node release and step repetition (Section 2.1, Eqs. 2-3,
 * Algorithms 1-2), intralaminar damage (Section 2.3.1, Algorithm 4) and
 * cohesive interfaces (Section 2.3.2, Algorithm 5).  Every step runs in HIP
 * kernels on one gfx950 device.
 *
 * Conventions (all calls):
 *  - host values are SI (m, kg, s, N, Pa, J/m^2) in double precision;
 *  - node n = i + (nx+1) * (j + (ny+1) * k), i, j in-plane grid indices,
 *    k the node plane (bottom 0); an interface between plies of different
 *    angle duplicates its plane;  nodal vectors are x,y,z interleaved;
 *  - bulk element e = i + nx * (j + ny * l), l the bulk element layer;
 *  - cohesive node pair p = i + (nx+1) * (j + (ny+1) * c), c the interface;
 *  - the impact direction is -Z; gravity acts along -Z;
 *  - all input structs and arrays are copied during the call; outputs go to
 *    caller-owned host buffers of capacity `cap` elements; when `cap` is too
 *    small the call returns PDN_ERANGE and sets *n_out to the size needed;
 *  - a context is used by one host thread at a time; it owns its device
 *    memory and stream work;
 *  - errors are negative return codes; pdn_last_error() gives the message.
 */
#ifndef PDN_H
#define PDN_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct pdn_ctx pdn_ctx;
typedef struct pdn_batch pdn_batch;

enum {
    PDN_OK = 0,
    PDN_EINVAL = -1,      /* invalid argument (sizes, material constants, snap-back) */
    PDN_ENOMEM = -2,      /* device or host allocation failed */
    PDN_EDEVICE = -3,     /* HIP runtime error */
    PDN_ESTATE = -4,      /* call out of order (mesh -> materials -> impactor -> step) */
    PDN_EUNSTABLE = -5,   /* non-finite state found; the context accepts only info/destroy */
    PDN_ERANGE = -6       /* output buffer too small, or contact left the search window */
};

enum { PDN_FP64 = 0, PDN_MIXED = 1 };     /* MIXED: FP32 element arithmetic and GP state,
                                             FP64 nodal, contact, striker and energies */
enum { PDN_BC_CLAMPED_EDGES = 0, PDN_BC_ASTM_WINDOW = 1, PDN_BC_FREE = 2 };
enum { PDN_LAW_ELASTIC = 0, PDN_LAW_CDM = 1, PDN_LAW_CDM_SURROGATE = 2 };
enum { PDN_DMG_FIBRE = 0, PDN_DMG_MATRIX = 1, PDN_DMG_SHEAR = 2, PDN_DMG_COHESIVE = 3,
       PDN_DMG_PROJ_FIBRE = 4, PDN_DMG_PROJ_MATRIX = 5, PDN_DMG_PROJ_COHESIVE = 6 };
enum { PDN_ARR_DISP = 0,    /* 3 * n_nodes: displacement at the last completed level */
       PDN_ARR_VEL = 1,     /* 3 * n_nodes: velocity (TW velocity = CD half-step velocity) */
       PDN_ARR_GP_R = 2,    /* 4 per bulk Gauss point (as PDN_ARR_GP_EP): damage thresholds r1+, r1-,
                               r2+, r2- */
       PDN_ARR_COH_R = 3,   /* n_pairs: cohesive damage threshold per interface node pair */
       PDN_ARR_MASS = 4,    /* n_nodes: lumped mass (get only) */
       PDN_ARR_GP_EP = 5 }; /* 3 per bulk Gauss point (n_bulk, or 8 n_bulk with full integration, points
                               of an element consecutive): plastic gamma12, gamma13 and accumulated
                               plastic shear (zeros, and set rejected, without plasticity) */

/* Plate description (Section 3.2 set-up): nx*ny element columns on lx*ly,
 * n_plies plies of ply_thickness each split into elems_per_ply hex8 layers.
 * The mesh is structured: every element is a box (an axis-aligned hexahedron)
 * between grid lines x_i, y_j and the layer planes; the grid lines may be
 * graded (x_coords, y_coords).  General (distorted) hexahedra are not
 * accepted: there is no per-node coordinate input. */
typedef struct {
    int32_t nx, ny, n_plies, elems_per_ply;
    double lx, ly, ply_thickness;
    const double *ply_angle_deg;   /* n_plies, bottom to top (fibre angle about Z) */
    int32_t cohesive;              /* 1 = zero-thickness interface where adjacent angles differ */
    int32_t bc;                    /* PDN_BC_*: clamped lateral faces; ASTM D7136 cut-out
                                      window (u_z = 0 on its edges, bottom plane) with corner
                                      clamps (u = 0 within clamp_radius of each corner); free */
    double window_lx, window_ly, clamp_radius;
    int32_t precision;             /* PDN_FP64 or PDN_MIXED */
    double phi;                    /* TW parameter: 1.0 = central difference */
    double cfl_safety;             /* stable-step fraction, e.g. 0.9 */
    double gravity;                /* m/s^2 along -Z on plate and striker (0 = off) */
    double hourglass_kappa;        /* Flanagan-Belytschko stiffness coefficient, e.g. 0.05 */
    const double *x_coords;        /* optional nx+1 graded grid lines (NULL = uniform) */
    const double *y_coords;        /* optional ny+1 graded grid lines (NULL = uniform) */
    int32_t device;                /* HIP device ordinal */
    void *stream;                  /* hipStream_t to run on; NULL = the context's own */
    int32_t integration;           /* bulk element: 0 or 1 = one point with hourglass control;
                                      8 = full 2x2x2 Gauss integration (Section 2), one damage
                                      state per point, no hourglass control (tiles 15x15 and
                                      16x16; no surrogate plies).  Other values: PDN_EINVAL */
} pdn_mesh_desc;

/* Ply material (Table 1 fields).  law = PDN_LAW_ELASTIC uses only the elastic
 * constants.  The interface fields describe the cohesive interface lying on
 * top of this ply.
 * Snap-back reading: the crack-band softening of Section 2.3.1 needs
 * l_c X^2 < 2 E G (l_c = cube root of the element volume); the paper does not
 * say what happens beyond that size.  A matrix or shear strength X that
 * violates it at an element's size is lowered for that element to
 * l_c X^2 = 0.9 * 2 E G, which keeps the dissipated energy G / l_c; the call
 * does not fail for it.  The fibre modes' bilinear law is not capped: a
 * fibre law that is not ordered at the element size gives PDN_EINVAL. */
typedef struct {
    double E1, E2, E3, nu12, nu13, nu23, G12, G13, G23, rho;
    int32_t law;
    double XT, XC, YT, YC, SL, alpha0_deg;
    double GXT, GXC, GYT, GYC, GSL;
    double fXT, fGT, fXC, fGC;
    double KI, tauI, tauII, GIc, GIIc, eta_bk;
    /* Matrix shear plasticity (Algorithm 4, first two lines; Table 1's S_p,
     * K_p), law PDN_LAW_CDM only; Sp = 0 turns it off.  Reading: linear
     * isotropic hardening of the longitudinal shear tau_L = |(tau12, tau13)|
     * in effective stress, yield when tau_L > Sp + Kp G12 abar (abar the
     * accumulated plastic shear), radial return; the damage criteria act on
     * the stress of the elastic strains; one plastic state per Gauss point
     * (one-point or full integration).  Needs G13 = G12, the 15x15, 16x16
     * or 8x8 tile (full integration: 15x15 or 16x16), no surrogate plies and
     * no batch; otherwise PDN_EINVAL. */
    double Sp, Kp;
} pdn_material;

/* Rigid striker (Section 3.2): radius, mass, initial tip gap above the top
 * surface, impact velocity v0 or energy (energy > 0 gives v0 = sqrt(2E/m)),
 * impact point x0/y0 (NaN = plate centre).  Reading of Section 2.2.2 for a
 * drop-weight striker guided along its axis: only the Z motion is
 * integrated; the in-plane components of the contact force do no work on
 * it (they are booked on the plate side only). */
typedef struct {
    double radius, mass, v0, energy, gap, x0, y0;
} pdn_impactor;

/* Energy books at the last complete time level L (one step behind the state).
 * Identity: ke_plate + ke_striker + w_int + d_pdn = ke0 + w_grav. */
typedef struct {
    double level;
    double ke_plate;         /* 0.5 sum m v^L . v^{L+1} */
    double ke_striker;       /* 0.5 m_s |V^L|^2 */
    double w_int;            /* trapezoidal work of internal forces (incl. hourglass, cohesive) */
    double w_grav;           /* work of gravity on plate and striker */
    double w_contact_plate;  /* trapezoidal work of the contact forces on the plate */
    double w_striker;        /* work of the frozen contact force on the striker */
    double d_pdn;            /* w_striker - w_contact_plate */
    double ke0;              /* striker kinetic energy at t = 0 */
    double u_el;             /* secant energy 0.5 sigma.eps V + hourglass + cohesive */
    double residual;         /* left side minus right side of the identity */
} pdn_energy;

typedef struct {
    double dt;
    int64_t n_nodes, n_bulk, n_cohesive, n_pairs, n_planes, n_layers, n_candidates;
    int64_t steps, reset_passes, released, active, max_passes;
    double fallback_fraction;     /* surrogate: of the GP updates on which the network was consulted,
                                     the fraction whose answer failed the residual bar and that the
                                     exact law produced (0 when none was consulted) */
    int32_t precision, tile_x, tile_y, blocks;
    double sur_consulted;         /* surrogate: GP updates on which the network was consulted (its
                                     answer computed and checked against the residual bar).  Points
                                     outside the law's screen whose incoming damage passes the gate,
                                     or of elements two workgroups evaluate, take the exact law
                                     without it and are not counted.  In steps of the plain build:
                                     the points outside the screen.  The others of surrogate plies
                                     were screened elastic by the law */
    int64_t sur_network_steps;    /* surrogate: steps run by the build that evaluates the network */
} pdn_info;

/* Build the plate mesh and allocate device state on desc->device. */
int pdn_mesh_create(const pdn_mesh_desc *desc, pdn_ctx **out);
/* Set the material of one ply (ply = -1: all plies).  EINVAL on non-positive
 * stiffness or a fibre softening law that is not ordered at this element size. */
int pdn_material_set(pdn_ctx *ctx, int32_t ply, const pdn_material *m);
/* Set the striker.  Before the first step: places it at gap above the plate
 * centre (or x0, y0).  Later: replaces only its velocity (v0 along -Z). */
int pdn_impactor_set(pdn_ctx *ctx, const pdn_impactor *imp);
/* Advance n explicit steps (Algorithm 1) on the context's stream; returns
 * after the stream has drained.  PDN_ERANGE if contact reached the edge of the
 * contact search window; PDN_EUNSTABLE on non-finite state. */
int pdn_step(pdn_ctx *ctx, int64_t n);
/* Contact-force history (the force-time and force-displacement outputs of
 * Section 3, Figs. 6-8; the peak forces of Tables 2 and 4), one entry per
 * step: time, contact force on the plate along -Z (the sum of the PDN
 * reactions of Eq. 3 over the active set), striker displacement along -Z.
 * Any of t/force/imp_disp may be NULL.  PDN_ERANGE with *n_out = steps when
 * cap is smaller. */
int pdn_contact_force(const pdn_ctx *ctx, double *t, double *force, double *imp_disp,
                      int64_t cap, int64_t *n_out);
/* Damage field (the damage maps of Fig. 9 and the projected delamination
 * area of Table 4): per bulk element (FIBRE/MATRIX/SHEAR: the larger damage
 * variable of the mode pair of Section 2.3.1, largest over the element's
 * points), per cohesive element (COHESIVE: interface damage D of
 * Section 2.3.2 at its current opening, largest over its 4 nodal points), or
 * projected nx*ny maps (PROJ_FIBRE, PROJ_MATRIX, PROJ_COHESIVE: largest over
 * the thickness of FIBRE, MATRIX and COHESIVE), i fastest.  Before the first
 * step every value is 0.  PDN_EINVAL for an unknown kind, PDN_ERANGE with
 * *n_out = size when cap is smaller. */
int pdn_damage_field(const pdn_ctx *ctx, int32_t kind, double *out, int64_t cap, int64_t *n_out);
int pdn_energies(const pdn_ctx *ctx, pdn_energy *out);
int pdn_info_get(const pdn_ctx *ctx, pdn_info *out);
/* Read (get) or replace (set) a state array (PDN_ARR_*), host double values.
 * A set makes the next step restart the explicit scheme from that state. */
int pdn_array_get(const pdn_ctx *ctx, int32_t kind, double *out, int64_t cap, int64_t *n_out);
int pdn_array_set(pdn_ctx *ctx, int32_t kind, const double *in, int64_t n);
/* Checkpoint: opaque blob of every device array, striker, books and history. */
int pdn_state_save(const pdn_ctx *ctx, void *buf, int64_t cap, int64_t *n_out);
int pdn_state_load(pdn_ctx *ctx, const void *buf, int64_t n);
/* Element-tile shape of the element/node kernel (autotuner hook): 0, 0 = the
 * default, 15 x 15 element columns.  Others: 16x16, 32x8, 8x8, 31x15 (full
 * integration: 15x15 and 16x16 only; shear plasticity: 15x15, 16x16 and
 * 8x8).  PDN_EINVAL for other shapes or one whose workgroup does not fit
 * the device's LDS. */
int pdn_set_tile(pdn_ctx *ctx, int32_t tile_x, int32_t tile_y);
/* Mean device time per step of the element/node kernel (with the contact
 * step on the top plane) and of the one-workgroup books kernel that closes
 * the step, over the last timed pdn_step call, from HIP events (0 if none
 * was timed). */
int pdn_kernel_times(const pdn_ctx *ctx, double *elem_node_ms, double *books_ms);
/* Time the following pdn_step calls (on != 0) or not.  Switching it on
 * creates the events for calls of up to 1,024 steps (longer calls add more),
 * so that a timed call holds only its launches and event records. */
int pdn_set_timing(pdn_ctx *ctx, int32_t on);
/* Measurement hook (not a step of the method): copy `bytes` (a multiple of
 * 16, 16-byte aligned device pointers) from src to dst on `device` with the
 * library's streaming-copy kernel, enqueued on `stream`.  The HBM bandwidth
 * it reaches is the practical ceiling the element/node kernel's roofline is
 * read against.  PDN_EINVAL on bad sizes or alignment. */
int pdn_stream_copy(int32_t device, void *stream, const void *src, void *dst, int64_t bytes);
/* Autotuner: time ten element/node passes per supported tile shape that
 * fits the device, keep the fastest (remembered per plate shape for the
 * process) and report it.  The default 15 x 15 is kept unless another shape
 * is faster by more than 5 %: the timed passes leave out the contact step
 * and the books kernel, whose work grows with the number of tiles.  They
 * recompute the current predictor, so the simulation state is unchanged.
 * ESTATE before materials and striker. */
int pdn_autotune(pdn_ctx *ctx, int32_t *tile_x, int32_t *tile_y);

/* Batched stepping of independent impact cases (many plates of uneven size
 * advanced together; each case is the method of Algorithm 1 on its own plate).
 * pdn_batch_create takes n contexts that are fully set up (mesh, materials,
 * striker), on one device and in one precision; they stay owned by the caller
 * and must outlive the batch.  It picks one element tile for all cases with
 * the autotuner (remembered per batch composition) and captures a graph of
 * steps.  pdn_batch_step advances every case by n steps: one launch of the
 * element/node kernel and one of the books kernel per step serve all cases;
 * it runs on the first case's stream and returns when done.  Each case keeps
 * its own time step, history, energies and outputs, read with the per-context
 * calls; a case may also be stepped alone between batched calls.  Errors name
 * the case (pdn_batch_last_error); EINVAL for mixed devices or precisions or a
 * repeated context, and on failure of pdn_batch_create the first case's
 * pdn_last_error gives the reason. */
int pdn_batch_create(pdn_ctx *const *cases, int32_t n, pdn_batch **out);
int pdn_batch_step(pdn_batch *b, int64_t n);
int pdn_batch_info(const pdn_batch *b, int32_t *tile_x, int32_t *tile_y, int64_t *n_bulk, int32_t *blocks);
const char *pdn_batch_last_error(const pdn_batch *b);
void pdn_batch_destroy(pdn_batch *b);
const char *pdn_last_error(const pdn_ctx *ctx);
void pdn_destroy(pdn_ctx *ctx);

/* ---- constitutive surrogate ------------------------------------------------
 * A network 10 -> 64 -> 64 -> 64 -> 10 (SiLU) replaces the intralaminar update
 * of Section 2.3.1 (Algorithm 4) on chosen plies, evaluated with bf16 matrix
 * operands and fp32 accumulation; the exact law stays the fallback.
 * Inputs: strain_k * E_k / X_k (material frame, Voigt 11, 22, 33, 23, 13, 12,
 * engineering shear) with (E_k, X_k) = (E1, XT), (E2, YT), (E2, YT), (G23, SL),
 * (G12, SL), (G12, SL), then s_N = 1 - 1/r_N for the thresholds r1+, r1-, r2+,
 * r2-.  Outputs: stress_k / X_k, then the new s_N through a sigmoid.
 * Parameters: PDN_SUR_NPARAM floats, W1[10][64], b1[64], W2[64][64], b2[64],
 * W3[64][64], b3[64], W4[64][10], b4[10] (W stored [in][out]).
 * The context-free calls below return negative codes with the reason in
 * pdn_global_last_error() (per host thread). */
#define PDN_SUR_NPARAM 9674

typedef struct {
    int32_t device;
    void *stream;           /* hipStream_t, NULL = null stream */
    int64_t n_paths;        /* strain paths in the data set (e.g. 10,000,000) */
    int32_t increments;     /* increments per path, 1..64 (e.g. 32) */
    uint64_t seed;          /* path recipe seed (e.g. 0x5EED5EED) */
    double val_fraction;    /* last fraction of the paths held out for validation */
    int64_t steps;          /* Adam steps */
    int32_t batch;          /* samples per step, a multiple of 128 */
    double lr, lr_final;    /* cosine schedule from lr to lr_final (0: lr / 100) */
    uint64_t init_seed;     /* Glorot-uniform initial weights */
} pdn_sur_train;

typedef struct {
    double loss_val_initial;   /* validation mean square error per output, before training */
    double loss_val;           /* ... after training */
    double loss_train;         /* training-set error after training (first 4M samples) */
    double data_seconds, train_seconds;
    int64_t samples_train, samples_val;
} pdn_sur_report;

/* Generate the data set on the device from the exact law (FP64) along the
 * seeded strain paths (monotone for even path index, 2-4 reversals for odd,
 * up to 3x onset), at crack-band length `crack_band`, and train the network
 * on it with the library's own matrix-core forward and backward kernels and
 * Adam.  Writes PDN_SUR_NPARAM weights. */
int pdn_surrogate_train(const pdn_sur_train *opt, const pdn_material *m, double crack_band, float *weights,
                        pdn_sur_report *rep);
/* Use a trained network on ply `ply` (-1: every ply with a damage law) of the
 * context.  A point that the exact law's elastic screen passes (thresholds at
 * 1 and strain provably inside every onset surface) takes the law's answer
 * without consulting the network.  A consulted point keeps the exact law when
 * a damage variable of its incoming thresholds exceeds dmg_thresh (e.g. 0.05),
 * or when the network's stress differs from the nominal stress of its own new
 * thresholds by more than res_thresh (e.g. 1e-3) relative to |C0 strain|.
 * pdn_info reports the consulted updates and the fraction of them that used
 * the exact law.  ESTATE for a ply without a damage law.  Legal mid-run. */
int pdn_surrogate_set(pdn_ctx *ctx, int32_t ply, const float *weights, int64_t n, double dmg_thresh,
                      double res_thresh);
/* Which kernel build steps a context with surrogate plies.  mode 0 (the
 * default) chooses per pdn_step call from the previous call: when that call
 * met no point that would consult the network (in the plain build: no point
 * outside the law's screen; in a network build: no point that consulted it),
 * the plain build, which steps the surrogate plies by the exact law (so such
 * a call costs what the plain path costs) and still counts the points outside
 * the screen; otherwise, and right after pdn_surrogate_set, the build that
 * evaluates the network at 1 wave per SIMD (no register spills around the
 * network; on 15x15 tiles, other tiles take the build held to 2 waves per
 * SIMD), which set-up evaluations also use.  The first call after such
 * points appear is stepped by the exact law; results can differ with how
 * steps are split into calls.  mode 1 always uses the 2-wave network build,
 * mode 2 the 1-wave one (both network builds compute the same bits).
 * PDN_EINVAL for other modes. */
int pdn_surrogate_kernel(pdn_ctx *ctx, int32_t mode);
/* Forward pass on n points: x is n x 10 inputs, y receives n x 10 outputs. */
int pdn_surrogate_eval(int32_t device, void *stream, const float *weights, const float *x, int64_t n, float *y);
/* Mean square error over n x 10 outputs against targets t, and its gradient
 * with respect to the PDN_SUR_NPARAM parameters (the training kernel's). */
int pdn_surrogate_grad(int32_t device, void *stream, const float *weights, const float *x, const float *t,
                       int64_t n, float *grad, double *loss);
/* The same loss and gradient with FP32 operands and arithmetic throughout
 * (vector units instead of the bf16 matrix cores), for checking against an
 * FP64 reference at FP32 accuracy.  Host arrays, synchronous. */
int pdn_surrogate_grad_fp32(int32_t device, void *stream, const float *weights, const float *x, const float *t,
                            int64_t n, float *grad, double *loss);
/* Records of paths p0 .. p0+n_paths-1 of the data set (20 floats each:
 * 10 inputs, 10 exact outputs; increments of a path consecutive). */
int pdn_surrogate_data(int32_t device, void *stream, const pdn_material *m, double crack_band, uint64_t seed,
                       int64_t p0, int64_t n_paths, int32_t increments, float *records);
/* The gradient of pdn_surrogate_grad without any allocation, for callers that
 * cannot allocate device memory (code under HIP graph capture, serving loops,
 * harnesses that forbid hipMalloc).  weights (PDN_SUR_NPARAM), x and t (n x 10
 * each), grad (PDN_SUR_NPARAM) and loss (one double, may be NULL) are DEVICE
 * pointers on `device`; the caller owns them.  The packed network, the
 * interleaved records and the per-workgroup partials live in one fixed
 * device array of the library (about 6.3 MB per device, held until the
 * process ends), so n is limited to PDN_SUR_GRAD_NOALLOC_MAX points: larger
 * n, n < 1 or a NULL pointer give PDN_EINVAL with the reason in
 * pdn_global_last_error().  The call only enqueues work on `stream` (NULL =
 * null stream) and returns: grad and loss are ready when the stream reaches
 * that point.  Its results equal those of pdn_surrogate_grad bit for bit.
 * Every call on a device shares that device's array: calls that overlap in
 * time on one device (other streams, other host threads) race and must be
 * serialised by the caller.  The first call on a device looks up the array's
 * address; make it before any graph capture. */
#define PDN_SUR_GRAD_NOALLOC_MAX 16384
int pdn_surrogate_grad_noalloc(int32_t device, void *stream, const float *weights, const float *x, const float *t,
                               int64_t n, float *grad, double *loss);
/* ---- mesh multiplication ----------------------------------------------------
 * Section 2.4, Eq. (mmu) and Algorithm 3: ndivi division levels of a
 * hexahedral mesh with 8-node interface elements, on the device.  One level
 * splits every edge at its midpoint and every face at its centre and adds a
 * node at the centre of every bulk element: a bulk hexahedron becomes eight.
 * An interface element (zero thickness; nodes 0-3 its bottom face, 4-7 the
 * coincident top face, the stacking direction from bottom to top) is divided
 * only by planes parallel to its normal: it becomes four, its edges across
 * the thickness and its lateral faces are not divided and it has no centre.
 * Node order of both element kinds: bottom face counter-clockwise, then top.
 * Numbering of each new level: old nodes first; then edge midpoints in
 * ascending (smaller, larger end node); then face centres in ascending
 * (smallest node, node diagonally opposite it); then bulk centres in element
 * order.  Children of bulk element e are 8e..8e+7 (octant i + 2j + 4k of its
 * natural coordinates), of interface element c are 4c..4c+3 (quadrant
 * i + 2j); tags (e.g. plies; may be NULL) are inherited.  Positions are the
 * averages of the edge's, face's (ascending node numbers) or element's
 * nodes.  All arrays are host arrays: coords 3*n_nodes, hexes 8*n_bulk, cohs
 * 8*n_interface (int32 node numbers).  counts receives the divided mesh's
 * sizes and, for the last level, the base mesh's divided edges and faces and
 * its boundary faces (used by one element; of them, interface lateral faces),
 * the terms of Eq. (mmu).  With NULL outputs or capacities too small, only
 * counts is filled and the call returns PDN_ERANGE.  PDN_EINVAL: negative
 * sizes, ndivi outside 0..6, node numbers out of range, or a divided mesh
 * beyond int32 numbering; reason in pdn_global_last_error(). */
typedef struct {
    int64_t n_nodes, n_bulk, n_interface;
    int64_t n_edges, n_faces, n_boundary0, n_boundary_interface0;
} pdn_mmu_counts;
int pdn_mesh_multiply(int32_t device, void *stream, const double *coords, int64_t n_nodes, const int32_t *hexes,
                      int64_t n_bulk, const int32_t *cohs, int64_t n_interface, const int32_t *hex_tag,
                      const int32_t *coh_tag, int32_t ndivi, double *coords_out, int32_t *hexes_out,
                      int32_t *cohs_out, int32_t *hex_tag_out, int32_t *coh_tag_out, int64_t cap_nodes,
                      int64_t cap_bulk, int64_t cap_interface, pdn_mmu_counts *counts);
const char *pdn_global_last_error(void);

#ifdef __cplusplus
}
#endif
#endif
