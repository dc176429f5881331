// pdn_api.cpp -- host side of libpdn: the C-ABI of include/pdn.h.
//
// The host builds the structured plate (grid lines, layer table, support
// masks), the per-ply constants and the time step, owns the device buffers
// and launches the kernels; every step of the method runs on the device.
#include "pdn.h"
#include "pdn_internal.h"
#include "pdn_launch.h"
#include "pdn_mlp.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

namespace {

struct Buf {
    void *p = nullptr;
    size_t n = 0;
};

}  // namespace

struct pdn_ctx {
    std::string err;
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    // description
    int nx = 0, ny = 0, P = 0, epp = 0, NL = 0, K = 0, cohesive = 0, bc = 0, precision = 0;
    double lx = 0, ly = 0, tply = 0, phi = 1, safety = 0.9, grav = 0, kappa = 0.05;
    double wlx = 0, wly = 0, clamp_r = 0;
    std::vector<double> ang, xs, ys, zk;
    std::vector<LayerInfo> layers;
    std::vector<int> bulk_layer, coh_layer;
    int64_t nn = 0, ne = 0, nce = 0, npairs = 0, plane = 0;
    // materials / striker
    std::vector<pdn_material> mat;
    std::vector<int> mat_set;
    bool have_imp = false;
    pdn_impactor imp{};
    double v0 = 0;
    // derived
    double dt = 0;
    std::vector<double> mx, my, mz, imx, imy, imz;
    int ci0 = 0, ci1 = 0, cj0 = 0, cj1 = 0;
    int tile = PDN_TILE_16x16, tiles_x = 1, tiles_y = 1;
    // state
    bool ready = false, needs_init = true, broken = false, loaded_state = false;
    int cur = 0;                      // buffer with the last completed level
    DevGlobals gl{};
    // device buffers
    double *d[2] = {nullptr, nullptr}, *v[2] = {nullptr, nullptr};
    void *r = nullptr, *rd = nullptr;
    void *hx = nullptr, *hy = nullptr, *ihx = nullptr, *ihy = nullptr, *ply = nullptr;
    double *xs_d = nullptr, *ys_d = nullptr, *mx_d = nullptr, *my_d = nullptr, *mz_d = nullptr;
    double *imx_d = nullptr, *imy_d = nullptr, *imz_d = nullptr, *cand_d = nullptr;
    bool cand_dirty = false;          // corrected candidates not yet in the state buffers
    LayerInfo *layers_d = nullptr;
    int *bulk_layer_d = nullptr, *coh_layer_d = nullptr;
    uint8_t *bcb_d = nullptr;
    uint8_t *active_d = nullptr;
    double *vprev_d = nullptr, *fcprev_d = nullptr, *fside_d = nullptr;
    double *partials_d = nullptr;     // two sets (written / read by consecutive passes), then the stage rows
    int prow = 0;                     // rows of one set
    int nblocks = 0;
    DevGlobals *gl_d = nullptr;
    double *hist_d = nullptr;
    int64_t hist_cap = 0;
    double *dmg_d = nullptr;
    size_t dmg_n = 0;
    std::vector<uint8_t> bcb;
    // constitutive surrogate: packed networks, network of each ply (-1 none)
    uint4 *sur_d = nullptr;
    int n_nets = 0;
    bool use_sur = false;             // some ply evaluates a network (kernel variant)
    bool plastic = false;             // some ply has shear plasticity (kernel variant, state ep)
    void *ep = nullptr;               // 4 per bulk GP when plastic: gamma12_p, gamma13_p, abar, -
    int ngp = 1;                      // Gauss points of a bulk element: 1 (hourglass control) or 8
    std::vector<int> ply_net;
    double sur_dmg = 0.05, sur_res = 1e-3;
    // which build steps the surrogate plies in a pdn_step call (0 plain, 1
    // network at 2 waves/SIMD, 2 network at 1 wave/SIMD where built): mode 0
    // picks per call from the previous call (a point outside the law's screen
    // or a network just set: build 2; none: the plain build, which steps those
    // plies by the exact law and counts such points); modes 1 and 2 pin that
    // build.  Build 2 is the faster network build in every case measured on
    // MI355X (1200x800x16 plate: 1.04 against 2.12 ms per step with no point
    // consulting the network, 4.35 against 5.9 with every point; 300x200x8
    // plate, 1.3 % consulting: 0.141 against 0.198 ms)
    int sur_mode = 0;
    int sur_build = 2;                 // also the build of set-up evaluations
    bool sur_fresh = true;
    double sur_gp_mark = 0.0;
    int64_t sur_prev_n = 0;
    int64_t sur_net_steps = 0;
    // timing: events are kept between calls (creating them inside a timed
    // call would add host time to it) and read when the times are asked for
    bool timing = false;
    double t_en_ms = 0, t_bk_ms = 0;
    std::vector<hipEvent_t> tev;       // per step: its start and the point between its two kernels; one more at the end
    int64_t tev_n = 0;                 // steps of the last timed call not yet read
};

namespace {

int set_err(pdn_ctx *c, int code, const char *fmt, ...)
{
    if (c) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        c->err = buf;
    }
    return code;
}

#define HIPCHK(ctx, call)                                                                       \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return set_err(ctx, e_ == hipErrorOutOfMemory ? PDN_ENOMEM : PDN_EDEVICE, "%s: %s", \
                           #call, hipGetErrorString(e_));                                       \
    } while (0)

size_t rsize(const pdn_ctx *c) { return c->precision == PDN_MIXED ? sizeof(float) : sizeof(double); }

int dalloc(pdn_ctx *c, void **p, size_t bytes)
{
    if (bytes == 0) bytes = 8;
    hipError_t e = hipMalloc(p, bytes);
    if (e != hipSuccess) return set_err(c, PDN_ENOMEM, "hipMalloc(%zu bytes) failed: %s", bytes, hipGetErrorString(e));
    return PDN_OK;
}

template <typename T>
int upload(pdn_ctx *c, T *dst, const std::vector<T> &src)
{
    if (src.empty()) return PDN_OK;
    HIPCHK(c, hipMemcpyAsync(dst, src.data(), src.size() * sizeof(T), hipMemcpyHostToDevice, c->stream));
    return PDN_OK;
}

// inverse of the symmetric 3x3 normal compliance block (adjugate / det)
void inv3(const double H[3][3], double C[3][3])
{
    double a00 = H[1][1] * H[2][2] - H[1][2] * H[2][1];
    double a01 = H[0][2] * H[2][1] - H[0][1] * H[2][2];
    double a02 = H[0][1] * H[1][2] - H[0][2] * H[1][1];
    double a11 = H[0][0] * H[2][2] - H[0][2] * H[2][0];
    double a12 = H[0][2] * H[1][0] - H[0][0] * H[1][2];
    double a22 = H[0][0] * H[1][1] - H[0][1] * H[1][0];
    double det = H[0][0] * a00 + H[0][1] * (H[1][2] * H[2][0] - H[1][0] * H[2][2]) + H[0][2] * (H[1][0] * H[2][1] - H[1][1] * H[2][0]);
    C[0][0] = a00 / det; C[0][1] = a01 / det; C[0][2] = a02 / det;
    C[1][0] = C[0][1]; C[1][1] = a11 / det; C[1][2] = a12 / det;
    C[2][0] = C[0][2]; C[2][1] = C[1][2]; C[2][2] = a22 / det;
}

double stiffness_max(const pdn_material &m, double C[3][3])
{
    double H[3][3] = {{1 / m.E1, -m.nu12 / m.E1, -m.nu13 / m.E1},
                      {-m.nu12 / m.E1, 1 / m.E2, -m.nu23 / m.E2},
                      {-m.nu13 / m.E1, -m.nu23 / m.E2, 1 / m.E3}};
    inv3(H, C);
    double mx = std::max({m.G23, m.G13, m.G12});
    for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) mx = std::max(mx, std::fabs(C[i][j]));
    return mx;
}

template <typename R>
PlyC<R> make_ply(const pdn_material &m, double ang_deg, int net = -1, double lc_min = 0.0, double lc_max = 0.0)
{
    PlyC<R> P{};
    double C[3][3];
    double cm = stiffness_max(m, C);
    P.C11 = (R)C[0][0]; P.C12 = (R)C[0][1]; P.C13 = (R)C[0][2];
    P.C22 = (R)C[1][1]; P.C23 = (R)C[1][2]; P.C33 = (R)C[2][2];
    P.G23 = (R)m.G23; P.G13 = (R)m.G13; P.G12 = (R)m.G12;
    P.iE1 = (R)(1 / m.E1); P.iE2 = (R)(1 / m.E2); P.iE3 = (R)(1 / m.E3);
    P.mn12 = (R)(-m.nu12 / m.E1); P.mn13 = (R)(-m.nu13 / m.E1); P.mn23 = (R)(-m.nu23 / m.E2);
    const double th = ang_deg * M_PI / 180.0;
    P.c = (R)std::cos(th);
    P.s = (R)std::sin(th);
    P.cmax = (R)cm;
    P.E1 = (R)m.E1; P.E2 = (R)m.E2; P.G12v = (R)m.G12;
    P.XT = (R)m.XT; P.XC = (R)m.XC; P.YT = (R)m.YT; P.YC = (R)m.YC; P.SL = (R)m.SL;
    P.GXT = (R)m.GXT; P.GXC = (R)m.GXC; P.GYT = (R)m.GYT; P.GYC = (R)m.GYC; P.GSL = (R)m.GSL;
    P.fXT = (R)m.fXT; P.fGT = (R)m.fGT; P.fXC = (R)m.fXC; P.fGC = (R)m.fGC;
    const double a0 = m.alpha0_deg * M_PI / 180.0;
    P.sa0 = (R)std::sin(a0);
    P.ca0 = (R)std::cos(a0);
    P.kST = (R)(std::cos(a0) * (std::sin(a0) + std::cos(a0) / std::tan(2 * a0)));
    P.etaT = (R)(-1.0 / std::tan(2 * a0));
    P.kEtaL = (R)(-std::cos(2 * a0) / (std::cos(a0) * std::cos(a0)));
    P.rho = (R)m.rho;
    // a surrogate ply without a network keeps the exact law
    P.law = m.law == PDN_LAW_ELASTIC ? 0 : (m.law == PDN_LAW_CDM_SURROGATE && net >= 0 ? 2 : 1);
    P.sur = P.law == 2 ? net : 0;
    if (P.law) {
        const double kst = std::cos(a0) * (std::sin(a0) + std::cos(a0) / std::tan(2 * a0));
        const double etat = -1.0 / std::tan(2 * a0);
        P.kE1XT = (R)(m.E1 / m.XT);
        P.iYT = (R)(1.0 / m.YT);
        P.iSL = (R)(1.0 / m.SL);
        P.kT = (R)(std::cos(a0) * (std::sin(a0) + std::fabs(etat) * std::cos(a0)));
        // Screen constants for the crack bands lc_min .. lc_max of the ply's
        // elements.  The crack band caps a strength at sqrt(1.8 E G / lc),
        // which only lowers it as lc grows: the strengths capped at lc_max
        // bound every element's loading functions from above.  eta_L =
        // k SL / YC is taken at its largest magnitude over the range (at an
        // end or where a cap sets in).  A relative margin of 1e-5 keeps a
        // screened point below onset in the law's own rounding too.
        auto capped = [](double X, double E, double G, double lc) {
            const double lim = 1.8 * E * G / lc;
            return lc > 0 && X * X > lim ? std::sqrt(lim) : X;
        };
        const double mg = 1.0 + 1e-5, lhi = lc_max * (1.0 + 1e-6), llo = lc_min * (1.0 - 1e-6);
        const double kel = -std::cos(2 * a0) / (std::cos(a0) * std::cos(a0));
        double rmax = 0.0;
        for (double lc : {llo, lhi, 1.8 * m.G12 * m.GSL / (m.SL * m.SL), 1.8 * m.E2 * m.GYC / (m.YC * m.YC)})
            if (lc >= llo && lc <= lhi)
                rmax = std::max(rmax, capped(m.SL, m.G12, m.GSL, lc) / capped(m.YC, m.E2, m.GYC, lc));
        P.scr_kXT = (R)(mg * m.E1 / m.XT);
        P.scr_kXC = (R)(mg * m.E1 / m.XC);
        P.scr_iYT = (R)(mg / capped(m.YT, m.E2, m.GYT, lhi));
        P.scr_iSL = (R)(mg / capped(m.SL, m.G12, m.GSL, lhi));
        P.scr_iST = (R)(mg / (kst * capped(m.YC, m.E2, m.GYC, lhi)));
        P.scr_etaL = (R)(mg * kel * rmax);
        P.scr_vmax = (R)(lc_max > 0 ? lc_max * lc_max * lc_max * (1.0 + 1e-6) : 0.0);
    }
    P.KI = (R)m.KI;
    const double ksh = (m.tauI > 0 && m.GIIc > 0) ? m.KI * (m.GIc / m.GIIc) * (m.tauII / m.tauI) * (m.tauII / m.tauI) : m.KI;
    P.Ksh = (R)ksh;
    P.tauI = (R)m.tauI; P.GIc = (R)m.GIc; P.GIIc = (R)m.GIIc; P.eta_bk = (R)m.eta_bk;
    P.GIo = (R)(m.KI > 0 ? m.tauI * m.tauI / (2 * m.KI) : 0.0);
    // An undamaged pair below the smallest onset opening over all mode
    // mixities stays undamaged: lambda <= lambda_o(B) for every B when
    // Ksh |d_sh|^2 + KI <d3>^2 <= 2 GIo min(GIc, GIIc) / GIc (a relative margin
    // of 1e-5 covers the rounding of the law's own evaluation).  It needs
    // GIc > GIo (lambda_c > lambda_o); otherwise no pair is screened.
    const double gio = m.KI > 0 ? m.tauI * m.tauI / (2 * m.KI) : 0.0;
    P.den_onset = (R)(m.KI > 0 && m.GIc > gio && m.GIIc > 0
                          ? 2.0 * gio * std::min(m.GIc, m.GIIc) / m.GIc * (1.0 - 1e-5) : -1.0);
    P.plas = (P.law == 1 && m.Sp > 0) ? 1 : 0;
    P.Sp = (R)m.Sp;
    P.Hp = (R)(m.Kp * m.G12);
    return P;
}

bool ply_plastic(const pdn_material &m) { return m.law == PDN_LAW_CDM && m.Sp > 0; }

// device record of Gauss point k = ngp e + g (the order of the exposed
// arrays): record e with one point; with eight, a layer's records point by
// point (point g of every element of the layer, then point g + 1)
int64_t gp_record(const pdn_ctx *c, int64_t k)
{
    if (c->ngp == 1) return k;
    const int64_t pl = (int64_t)c->nx * c->ny, e = k / 8, g = k % 8;
    return 8 * pl * (e / pl) + g * pl + e % pl;
}

bool all_set(const pdn_ctx *c)
{
    for (int p = 0; p < c->P; ++p)
        if (!c->mat_set[p]) return false;
    return true;
}

int window_index(int n, double len, double win)
{
    double q = n * (len - win) / (2.0 * len);
    return (int)std::floor(q + 0.5 + 1e-9);
}

// mass factors, time step, tables, globals; done once before the first step
int prepare(pdn_ctx *c)
{
    const int nx = c->nx, ny = c->ny;
    c->mx.assign(nx + 1, 0.0);
    c->my.assign(ny + 1, 0.0);
    c->mz.assign(c->K, 0.0);
    for (int i = 0; i <= nx; ++i)
        c->mx[i] = 0.5 * ((i > 0 ? c->xs[i] - c->xs[i - 1] : 0.0) + (i < nx ? c->xs[i + 1] - c->xs[i] : 0.0));
    for (int j = 0; j <= ny; ++j)
        c->my[j] = 0.5 * ((j > 0 ? c->ys[j] - c->ys[j - 1] : 0.0) + (j < ny ? c->ys[j + 1] - c->ys[j] : 0.0));
    for (int k = 0; k < c->K; ++k) {
        double s = 0;
        if (k > 0 && c->layers[k - 1].type == 0) s += c->mat[c->layers[k - 1].ply].rho * c->layers[k - 1].hz;
        if (k < c->NL && c->layers[k].type == 0) s += c->mat[c->layers[k].ply].rho * c->layers[k].hz;
        c->mz[k] = 0.5 * s;
    }
    // stable step (Section 2.3.1: l_c / c_D with l_c = V / A_max; 2.3.2: interface springs)
    double hxmin = 1e300, hymin = 1e300;
    for (int i = 0; i < nx; ++i) hxmin = std::min(hxmin, c->xs[i + 1] - c->xs[i]);
    for (int j = 0; j < ny; ++j) hymin = std::min(hymin, c->ys[j + 1] - c->ys[j]);
    double dtb = 1e300, dtc = 1e300;
    for (int l = 0; l < c->NL; ++l) {
        const LayerInfo &L = c->layers[l];
        const pdn_material &m = c->mat[L.ply];
        if (L.type == 0) {
            double C[3][3];
            double cm = stiffness_max(m, C);
            double lc = std::min({hxmin, hymin, L.hz});
            dtb = std::min(dtb, lc * std::sqrt(m.rho / cm));
        } else {
            double a = c->mz[l], b = c->mz[l + 1];
            dtc = std::min(dtc, 2.0 * std::sqrt((a * b / (a + b)) / m.KI));
        }
    }
    c->dt = c->nce > 0 ? c->safety / std::sqrt(1.0 / (dtb * dtb) + 1.0 / (dtc * dtc)) : c->safety * dtb;

    int rc;
    if ((rc = upload(c, c->mx_d, c->mx))) return rc;
    if ((rc = upload(c, c->my_d, c->my))) return rc;
    if ((rc = upload(c, c->mz_d, c->mz))) return rc;
    c->imx.resize(nx + 1);
    c->imy.resize(ny + 1);
    c->imz.resize(c->K);
    for (int i = 0; i <= nx; ++i) c->imx[i] = 1.0 / c->mx[i];
    for (int j = 0; j <= ny; ++j) c->imy[j] = 1.0 / c->my[j];
    for (int k = 0; k < c->K; ++k) c->imz[k] = c->mz[k] > 0 ? 1.0 / c->mz[k] : 0.0;
    if ((rc = upload(c, c->imx_d, c->imx))) return rc;
    if ((rc = upload(c, c->imy_d, c->imy))) return rc;
    if ((rc = upload(c, c->imz_d, c->imz))) return rc;
    c->use_sur = false;
    for (int p = 0; p < c->P; ++p)
        if (c->mat[p].law == PDN_LAW_CDM_SURROGATE && c->ply_net[p] >= 0) c->use_sur = true;
    c->plastic = false;
    for (int p = 0; p < c->P; ++p)
        if (ply_plastic(c->mat[p])) c->plastic = true;
    if (c->plastic) {
        if (c->use_sur) return set_err(c, PDN_EINVAL, "shear plasticity and surrogate plies are not built together");
        if (c->ngp == 1 ? !pdn::tile_has_plas(c->tile) : !pdn::tile_has_full(c->tile))
            return set_err(c, PDN_EINVAL, "shear plasticity is built for the 15x15, 16x16 and 8x8 tiles "
                                          "(with full integration: 15x15 and 16x16)");
        if (!c->ep) {                 // plastic state, zero at the start (Algorithm 4)
            const size_t bytes = 4 * (size_t)c->ngp * (size_t)std::max<int64_t>(1, c->ne) * rsize(c);
            if ((rc = dalloc(c, &c->ep, bytes))) return rc;
            HIPCHK(c, hipMemsetAsync(c->ep, 0, bytes, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
    }
    // crack-band range of each ply's elements (for the screen constants)
    std::vector<double> lcmin(c->P, 0.0), lcmax(c->P, 0.0);
    {
        double hxlo = 1e300, hxhi = 0, hylo = 1e300, hyhi = 0;
        for (int i = 0; i < nx; ++i) { const double h = c->xs[i + 1] - c->xs[i]; hxlo = std::min(hxlo, h); hxhi = std::max(hxhi, h); }
        for (int j = 0; j < ny; ++j) { const double h = c->ys[j + 1] - c->ys[j]; hylo = std::min(hylo, h); hyhi = std::max(hyhi, h); }
        std::vector<double> hzlo(c->P, 1e300), hzhi(c->P, 0.0);
        for (int l = 0; l < c->NL; ++l)
            if (c->layers[l].type == 0) {
                const int p = c->layers[l].ply;
                hzlo[p] = std::min(hzlo[p], c->layers[l].hz);
                hzhi[p] = std::max(hzhi[p], c->layers[l].hz);
            }
        for (int p = 0; p < c->P; ++p)
            if (hzhi[p] > 0) {
                lcmin[p] = std::cbrt(hxlo * hylo * hzlo[p]);
                lcmax[p] = std::cbrt(hxhi * hyhi * hzhi[p]);
            }
    }
    if (c->precision == PDN_MIXED) {
        std::vector<PlyC<float>> pc;
        for (int p = 0; p < c->P; ++p)
            pc.push_back(make_ply<float>(c->mat[p], c->ang[p], c->ply_net[p], lcmin[p], lcmax[p]));
        HIPCHK(c, hipMemcpyAsync(c->ply, pc.data(), pc.size() * sizeof(pc[0]), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else {
        std::vector<PlyC<double>> pc;
        for (int p = 0; p < c->P; ++p)
            pc.push_back(make_ply<double>(c->mat[p], c->ang[p], c->ply_net[p], lcmin[p], lcmax[p]));
        HIPCHK(c, hipMemcpyAsync(c->ply, pc.data(), pc.size() * sizeof(pc[0]), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    c->ready = true;
    return PDN_OK;
}

int ensure_history(pdn_ctx *c, int64_t need)
{
    if (need <= c->hist_cap) return PDN_OK;
    int64_t cap = std::max<int64_t>(need, std::max<int64_t>(2 * c->hist_cap, 4096));
    double *nh = nullptr;
    int rc = dalloc(c, (void **)&nh, 3 * cap * sizeof(double));
    if (rc) return rc;
    if (c->hist_d) {
        HIPCHK(c, hipMemcpyAsync(nh, c->hist_d, 3 * c->hist_cap * sizeof(double), hipMemcpyDeviceToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        HIPCHK(c, hipFree(c->hist_d));
    }
    c->hist_d = nh;
    c->hist_cap = cap;
    c->gl.hist_cap = cap;
    HIPCHK(c, hipMemcpyAsync(&c->gl_d->hist_cap, &cap, sizeof cap, hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));      // the source is a local
    return PDN_OK;
}

// two term-major sets of block partials, then the books stage rows
size_t partials_bytes(int prow) { return (2 * (size_t)PDN_NTERMS * prow + PDN_STAGE * PDN_NTERMS) * sizeof(double); }

// arguments of an element/node pass reading buffer `in` and writing `out`;
// contact = 1: the pass does the contact step on the top plane first
template <typename R>
ElemArgs<R> elem_args(pdn_ctx *c, int in, int out, int contact)
{
    ElemArgs<R> a{};
    a.nx = c->nx; a.ny = c->ny; a.K = c->K; a.NL = c->NL;
    a.tiles_x = c->tiles_x; a.tiles_y = c->tiles_y;
    a.clamp_lateral = c->bc == PDN_BC_CLAMPED_EDGES;
    a.ci0 = c->ci0; a.ci1 = c->ci1; a.cj0 = c->cj0; a.cj1 = c->cj1;
    a.dt = c->dt; a.phi = c->phi; a.grav = c->grav;
    a.kappa = (R)c->kappa;
    a.d_in = c->d[in]; a.v_in = c->v[in]; a.d_out = c->d[out]; a.v_out = c->v[out];
    a.r = (R *)c->r; a.rd = (R *)c->rd;
    a.ep = c->plastic ? (R *)c->ep : nullptr;
    a.hx = (const R *)c->hx; a.hy = (const R *)c->hy;
    a.ihx = (const R *)c->ihx; a.ihy = (const R *)c->ihy;
    a.mx = c->mx_d; a.my = c->my_d; a.mz = c->mz_d;
    a.imx = c->imx_d; a.imy = c->imy_d; a.imz = c->imz_d;
    a.layers = c->layers_d;
    a.ply = (const PlyC<R> *)c->ply;
    a.bc_bottom = c->bcb_d;
    a.fside = c->fside_d;
    // partial sets follow the buffers: a pass writes set `out`, the next pass
    // (which reads buffer `out`) finds them as set `in`
    a.partials = c->partials_d + (size_t)out * PDN_NTERMS * c->prow;
    a.partials_prev = c->partials_d + (size_t)in * PDN_NTERMS * c->prow;
    a.prow = c->prow;
    a.stage = c->partials_d + 2 * (size_t)PDN_NTERMS * c->prow;
    // owner tile of node column g along one axis (tiles overlap by one element
    // column, a tile owns the nodes past its first line), widened by one tile
    const int TX = pdn_tile_dims[c->tile][0], TY = pdn_tile_dims[c->tile][1];
    auto owner = [](int g, int T, int nt) { return std::min(nt - 1, g > 0 ? (g - 1) / (T - 1) : 0); };
    a.wt0 = std::max(0, owner(c->ci0, TX, c->tiles_x) - 1);
    a.wt1 = std::min(c->tiles_x, owner(std::max(c->ci0, c->ci1 - 1), TX, c->tiles_x) + 2);
    a.wu0 = std::max(0, owner(c->cj0, TY, c->tiles_y) - 1);
    a.wu1 = std::min(c->tiles_y, owner(std::max(c->cj0, c->cj1 - 1), TY, c->tiles_y) + 2);
    a.contact = contact;
    a.gl = c->gl_d;
    a.xs = c->xs_d; a.ys = c->ys_d;
    a.ztop = c->zk[c->K - 1];
    const size_t nc = (size_t)(c->ci1 - c->ci0) * (c->cj1 - c->cj0);
    a.active_in = c->active_d + (size_t)in * nc;
    a.active_out = c->active_d + (size_t)out * nc;
    a.vprev = c->vprev_d; a.fcprev = c->fcprev_d;
    a.cand = c->cand_d;
    a.hist = c->hist_d;
    a.mlp = c->sur_d;
    a.sur_dmg = (float)c->sur_dmg;
    a.sur_res = (float)c->sur_res;
    a.count_sur = c->use_sur && c->sur_build == 0 ? 1 : 0;
    return a;
}

ContactArgs contact_args(pdn_ctx *c, int buf)
{
    ContactArgs a{};
    a.d = c->d[buf]; a.v = c->v[buf];
    a.nx = c->nx; a.ny = c->ny; a.K = c->K;
    a.ci0 = c->ci0; a.ci1 = c->ci1; a.cj0 = c->cj0; a.cj1 = c->cj1;
    a.active = c->active_d; a.vprev = c->vprev_d; a.fcprev = c->fcprev_d; a.cand = c->cand_d;
    return a;
}

// at least `need` timing events in the context's pool
int timing_pool(pdn_ctx *c, int64_t need)
{
    while ((int64_t)c->tev.size() < need) {
        hipEvent_t e;
        HIPCHK(c, hipEventCreate(&e));
        c->tev.push_back(e);
    }
    return PDN_OK;
}

// mean kernel times of the last timed call, from its events (complete: the
// call synchronised its stream before returning)
int timing_collect(pdn_ctx *c)
{
    const int64_t n = c->tev_n;
    if (n <= 0) return PDN_OK;
    double a = 0, b = 0;
    for (int64_t s = 0; s < n; ++s) {
        float t = 0, u = 0;
        HIPCHK(c, hipEventElapsedTime(&t, c->tev[2 * s], c->tev[2 * s + 1]));
        HIPCHK(c, hipEventElapsedTime(&u, c->tev[2 * s + 1], c->tev[2 * s + 2]));
        a += t;
        b += u;
    }
    c->t_en_ms = a / n;
    c->t_bk_ms = b / n;
    c->tev_n = 0;
    return PDN_OK;
}

// one pass; a contact pass is closed by the books kernel (an event between
// the two when mid is given)
int launch_en(pdn_ctx *c, int in, int out, int contact, hipEvent_t mid = nullptr)
{
    hipError_t e;
    const bool mx = c->precision == PDN_MIXED;
    const int net = c->use_sur ? c->sur_build : 0;
    if (mx)
        e = pdn::launch_elem_node<float>(elem_args<float>(c, in, out, contact), c->tile, net, c->ngp, c->stream);
    else
        e = pdn::launch_elem_node<double>(elem_args<double>(c, in, out, contact), c->tile, net, c->ngp, c->stream);
    if (e != hipSuccess) return set_err(c, PDN_EDEVICE, "element/node kernel launch: %s", hipGetErrorString(e));
    if (!contact) return PDN_OK;
    if (mid) HIPCHK(c, hipEventRecord(mid, c->stream));
    e = mx ? pdn::launch_books<float>(elem_args<float>(c, in, out, contact), c->stream)
           : pdn::launch_books<double>(elem_args<double>(c, in, out, contact), c->stream);
    if (e != hipSuccess) return set_err(c, PDN_EDEVICE, "books kernel launch: %s", hipGetErrorString(e));
    return PDN_OK;
}

bool tile_fits(pdn_ctx *c, int tile)
{
    int maxlds = 0;
    if (hipDeviceGetAttribute(&maxlds, hipDeviceAttributeMaxSharedMemoryPerBlock, c->device) != hipSuccess) return false;
    const int lds = pdn::elem_node_lds_bytes(c->precision == PDN_MIXED, tile, c->use_sur);
    return lds > 0 && lds <= maxlds;
}

void set_tiles(pdn_ctx *c)
{
    const int TX = pdn_tile_dims[c->tile][0], TY = pdn_tile_dims[c->tile][1];
    c->tiles_x = std::max(1, (c->nx - 1 + TX - 2) / (TX - 1));
    c->tiles_y = std::max(1, (c->ny - 1 + TY - 2) / (TY - 1));
    c->nblocks = c->tiles_x * c->tiles_y;
}

// corrected top-surface candidates of the last contact pass into the state buffers
int materialize(pdn_ctx *c)
{
    if (!c->cand_dirty) return PDN_OK;
    hipError_t e = pdn::launch_cand_scatter(contact_args(c, c->cur), c->stream);
    if (e != hipSuccess) return set_err(c, PDN_EDEVICE, "candidate scatter: %s", hipGetErrorString(e));
    c->cand_dirty = false;
    return PDN_OK;
}

// restart the explicit scheme from the state in buffer c->cur
int init_level(pdn_ctx *c, bool reset_contact)
{
    const int in = c->cur, out = 1 - c->cur;
    int rc = materialize(c);
    if (!rc) rc = launch_en(c, in, out, 0);
    if (rc) return rc;
    if (reset_contact) {
        hipError_t e = pdn::launch_contact_init(contact_args(c, in), 1, c->stream);
        if (e != hipSuccess) return set_err(c, PDN_EDEVICE, "contact init: %s", hipGetErrorString(e));
    }
    c->needs_init = false;
    return PDN_OK;
}

void free_all(pdn_ctx *c)
{
    void *ps[] = {c->d[0], c->d[1], c->v[0], c->v[1], c->r, c->rd, c->hx, c->hy, c->ihx, c->ihy, c->ply, c->xs_d, c->ys_d,
                  c->mx_d, c->my_d, c->mz_d, c->imx_d, c->imy_d, c->imz_d, c->cand_d,
                  c->layers_d, c->bulk_layer_d, c->coh_layer_d, c->bcb_d,
                  c->active_d, c->vprev_d, c->fcprev_d, c->fside_d, c->partials_d, c->gl_d, c->hist_d, c->dmg_d,
                  c->sur_d, c->ep};
    for (void *p : ps)
        if (p) (void)hipFree(p);
}

int alloc_contact_window(pdn_ctx *c)
{
    // candidate window: top-surface node columns within 1.25 R + one element of the impact point
    const double x0 = std::isnan(c->imp.x0) ? 0.5 * (c->xs[0] + c->xs[c->nx]) : c->imp.x0;
    const double y0 = std::isnan(c->imp.y0) ? 0.5 * (c->ys[0] + c->ys[c->ny]) : c->imp.y0;
    double hmax = 0;
    for (int i = 0; i < c->nx; ++i) hmax = std::max(hmax, c->xs[i + 1] - c->xs[i]);
    for (int j = 0; j < c->ny; ++j) hmax = std::max(hmax, c->ys[j + 1] - c->ys[j]);
    const double Rc = 1.25 * c->imp.radius + hmax;
    int ci0 = 0, ci1 = c->nx + 1, cj0 = 0, cj1 = c->ny + 1;
    while (ci0 < c->nx && c->xs[ci0] < x0 - Rc) ++ci0;
    while (ci1 > ci0 + 1 && c->xs[ci1 - 1] > x0 + Rc) --ci1;
    while (cj0 < c->ny && c->ys[cj0] < y0 - Rc) ++cj0;
    while (cj1 > cj0 + 1 && c->ys[cj1 - 1] > y0 + Rc) --cj1;
    c->ci0 = ci0; c->ci1 = ci1; c->cj0 = cj0; c->cj1 = cj1;
    const size_t nc = (size_t)(ci1 - ci0) * (cj1 - cj0);
    int rc;
    if (c->active_d) { (void)hipFree(c->active_d); (void)hipFree(c->vprev_d); (void)hipFree(c->fcprev_d); (void)hipFree(c->fside_d); (void)hipFree(c->cand_d); }
    if ((rc = dalloc(c, (void **)&c->active_d, 2 * nc))) return rc;             // two step parities
    if ((rc = dalloc(c, (void **)&c->vprev_d, 3 * nc * sizeof(double)))) return rc;
    if ((rc = dalloc(c, (void **)&c->fcprev_d, 3 * nc * sizeof(double)))) return rc;
    if ((rc = dalloc(c, (void **)&c->fside_d, 3 * nc * sizeof(double)))) return rc;
    if ((rc = dalloc(c, (void **)&c->cand_d, 6 * nc * sizeof(double)))) return rc;
    HIPCHK(c, hipMemsetAsync(c->active_d, 0, 2 * nc, c->stream));
    HIPCHK(c, hipMemsetAsync(c->fside_d, 0, 3 * nc * sizeof(double), c->stream));
    c->cand_dirty = false;
    return PDN_OK;
}

int sync_globals_from_device(pdn_ctx *c)
{
    HIPCHK(c, hipMemcpyAsync(&c->gl, c->gl_d, sizeof(DevGlobals), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PDN_OK;
}

int push_globals(pdn_ctx *c)
{
    HIPCHK(c, hipMemcpyAsync(c->gl_d, &c->gl, sizeof(DevGlobals), hipMemcpyHostToDevice, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PDN_OK;
}

}  // namespace

// ===========================================================================
// C-ABI
// ===========================================================================

extern "C" {

int pdn_mesh_create(const pdn_mesh_desc *desc, pdn_ctx **out)
{
    if (!desc || !out) return PDN_EINVAL;
    *out = nullptr;
    const pdn_mesh_desc &D = *desc;
    if (D.nx < 1 || D.ny < 1 || D.n_plies < 1 || D.n_plies > PDN_MAX_PLIES || D.elems_per_ply < 1 ||
        !(D.lx > 0) || !(D.ly > 0) || !(D.ply_thickness > 0) || !D.ply_angle_deg ||
        (D.precision != PDN_FP64 && D.precision != PDN_MIXED) || D.bc < 0 || D.bc > 2 ||
        !(D.cfl_safety > 0) || !(D.phi >= 1.0) || D.hourglass_kappa < 0 ||
        (D.integration != 0 && D.integration != 1 && D.integration != 8))
        return PDN_EINVAL;
    pdn_ctx *c = new pdn_ctx();
    c->ngp = D.integration == 8 ? 8 : 1;
    c->device = D.device;
    c->nx = D.nx; c->ny = D.ny; c->P = D.n_plies; c->epp = D.elems_per_ply;
    c->cohesive = D.cohesive; c->bc = D.bc; c->precision = D.precision;
    c->lx = D.lx; c->ly = D.ly; c->tply = D.ply_thickness; c->phi = D.phi; c->safety = D.cfl_safety;
    c->grav = D.gravity; c->kappa = D.hourglass_kappa;
    c->wlx = D.window_lx; c->wly = D.window_ly; c->clamp_r = D.clamp_radius;
    c->ang.assign(D.ply_angle_deg, D.ply_angle_deg + D.n_plies);
    c->mat.assign(c->P, pdn_material{});
    c->mat_set.assign(c->P, 0);
    c->ply_net.assign(c->P, -1);
    // grid lines
    c->xs.resize(c->nx + 1);
    c->ys.resize(c->ny + 1);
    for (int i = 0; i <= c->nx; ++i) c->xs[i] = D.x_coords ? D.x_coords[i] : D.lx * i / D.nx;
    for (int j = 0; j <= c->ny; ++j) c->ys[j] = D.y_coords ? D.y_coords[j] : D.ly * j / D.ny;
    for (int i = 0; i < c->nx; ++i)
        if (!(c->xs[i + 1] > c->xs[i])) { delete c; return PDN_EINVAL; }
    for (int j = 0; j < c->ny; ++j)
        if (!(c->ys[j + 1] > c->ys[j])) { delete c; return PDN_EINVAL; }
    // layers: plies split into elements, interfaces where the angle changes
    const double hz = D.ply_thickness / D.elems_per_ply;
    int nb = 0, ncl = 0;
    for (int p = 0; p < c->P; ++p) {
        for (int e = 0; e < c->epp; ++e) {
            c->layers.push_back(LayerInfo{0, p, nb++, 0, hz, 1.0 / hz});
            c->bulk_layer.push_back((int)c->layers.size() - 1);
        }
        if (p + 1 < c->P && c->cohesive && c->ang[p] != c->ang[p + 1]) {
            c->layers.push_back(LayerInfo{1, p, ncl++, 0, 0.0, 0.0});
            c->coh_layer.push_back((int)c->layers.size() - 1);
        }
    }
    c->NL = (int)c->layers.size();
    c->K = c->NL + 1;
    c->zk.assign(c->K, 0.0);
    for (int l = 0; l < c->NL; ++l) c->zk[l + 1] = c->zk[l] + c->layers[l].hz;
    c->plane = (int64_t)(c->nx + 1) * (c->ny + 1);
    c->nn = c->plane * c->K;
    c->ne = (int64_t)c->nx * c->ny * nb;
    c->nce = (int64_t)c->nx * c->ny * ncl;
    c->npairs = c->plane * ncl;
    // supports of the bottom plane
    c->bcb.assign(c->plane, 0);
    if (c->bc == PDN_BC_ASTM_WINDOW) {
        const int ilo = window_index(c->nx, c->xs[c->nx] - c->xs[0], D.window_lx), ihi = c->nx - ilo;
        const int jlo = window_index(c->ny, c->ys[c->ny] - c->ys[0], D.window_ly), jhi = c->ny - jlo;
        const double r2 = D.clamp_radius * D.clamp_radius * (1.0 + 1e-9);
        for (int j = 0; j <= c->ny; ++j)
            for (int i = 0; i <= c->nx; ++i) {
                uint8_t b = 0;
                if (((i == ilo || i == ihi) && j >= jlo && j <= jhi) || ((j == jlo || j == jhi) && i >= ilo && i <= ihi)) b |= 4;
                const int ci[2] = {ilo, ihi}, cj[2] = {jlo, jhi};
                for (int a = 0; a < 2; ++a)
                    for (int q = 0; q < 2; ++q) {
                        const double dx = c->xs[i] - c->xs[ci[a]], dy = c->ys[j] - c->ys[cj[q]];
                        if (dx * dx + dy * dy <= r2) b = 7;
                    }
                c->bcb[i + (int64_t)(c->nx + 1) * j] = b;
            }
    }
    // device
    hipError_t he = hipSetDevice(c->device);
    if (he != hipSuccess) { set_err(c, PDN_EDEVICE, "hipSetDevice: %s", hipGetErrorString(he)); delete c; return PDN_EDEVICE; }
    if (D.stream) c->stream = (hipStream_t)D.stream;
    else {
        he = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking);
        if (he != hipSuccess) { delete c; return PDN_EDEVICE; }
        c->own_stream = true;
    }
    {   // default element tile: the preferred shape whose workgroup fits the device's LDS
        const int pref_mixed[] = {PDN_TILE_15x15, PDN_TILE_16x16, PDN_TILE_31x15, PDN_TILE_32x8, PDN_TILE_8x8};
        // FP64: at 16x16 the one-point kernel spills 116 VGPRs at 2 waves/SIMD; at 15x15
        // it runs at 1 wave/SIMD without spills, 1.19 against 1.65 ms on 1200x800x16
        const int pref_fp64[] = {PDN_TILE_15x15, PDN_TILE_16x16, PDN_TILE_31x15, PDN_TILE_32x8, PDN_TILE_8x8};
        const int *pref = c->precision == PDN_MIXED ? pref_mixed : pref_fp64;
        c->tile = -1;
        for (int k = 0; k < PDN_TILE_COUNT && c->tile < 0; ++k)
            if (tile_fits(c, pref[k]) && (c->ngp == 1 || pdn::tile_has_full(pref[k]))) c->tile = pref[k];
        if (c->tile < 0) {
            if (c->own_stream) (void)hipStreamDestroy(c->stream);
            delete c;
            return PDN_EDEVICE;
        }
    }
    set_tiles(c);
    int rc = PDN_OK;
    const size_t rs = rsize(c);
    for (int b = 0; b < 2 && !rc; ++b) {
        rc = dalloc(c, (void **)&c->d[b], 3 * c->nn * sizeof(double));
        if (!rc) rc = dalloc(c, (void **)&c->v[b], 3 * c->nn * sizeof(double));
    }
    if (!rc) rc = dalloc(c, &c->r, 4 * c->ngp * c->ne * rs);
    if (!rc) rc = dalloc(c, &c->rd, c->npairs * rs);
    if (!rc) rc = dalloc(c, &c->hx, c->nx * rs);
    if (!rc) rc = dalloc(c, &c->hy, c->ny * rs);
    if (!rc) rc = dalloc(c, &c->ihx, c->nx * rs);
    if (!rc) rc = dalloc(c, &c->ihy, c->ny * rs);
    if (!rc) rc = dalloc(c, &c->ply, c->P * std::max(sizeof(PlyC<float>), sizeof(PlyC<double>)));
    if (!rc) rc = dalloc(c, (void **)&c->xs_d, (c->nx + 1) * sizeof(double));
    if (!rc) rc = dalloc(c, (void **)&c->ys_d, (c->ny + 1) * sizeof(double));
    if (!rc) rc = dalloc(c, (void **)&c->mx_d, (c->nx + 1) * sizeof(double));
    if (!rc) rc = dalloc(c, (void **)&c->my_d, (c->ny + 1) * sizeof(double));
    if (!rc) rc = dalloc(c, (void **)&c->mz_d, c->K * sizeof(double));
    if (!rc) rc = dalloc(c, (void **)&c->imx_d, (c->nx + 1) * sizeof(double));
    if (!rc) rc = dalloc(c, (void **)&c->imy_d, (c->ny + 1) * sizeof(double));
    if (!rc) rc = dalloc(c, (void **)&c->imz_d, c->K * sizeof(double));
    if (!rc) rc = dalloc(c, (void **)&c->layers_d, c->NL * sizeof(LayerInfo));
    if (!rc) rc = dalloc(c, (void **)&c->bulk_layer_d, std::max<size_t>(1, c->bulk_layer.size()) * sizeof(int));
    if (!rc) rc = dalloc(c, (void **)&c->coh_layer_d, std::max<size_t>(1, c->coh_layer.size()) * sizeof(int));
    if (!rc) rc = dalloc(c, (void **)&c->bcb_d, c->plane);
    if (!rc) rc = dalloc(c, (void **)&c->gl_d, sizeof(DevGlobals));
    c->prow = std::max(1, c->nblocks);
    if (!rc) rc = dalloc(c, (void **)&c->partials_d, partials_bytes(c->prow));
    if (rc) { free_all(c); if (c->own_stream) (void)hipStreamDestroy(c->stream); delete c; return rc; }
    // tables
    std::vector<double> hxv(c->nx), hyv(c->ny), ihxv(c->nx), ihyv(c->ny);
    for (int i = 0; i < c->nx; ++i) { hxv[i] = c->xs[i + 1] - c->xs[i]; ihxv[i] = 1.0 / hxv[i]; }
    for (int j = 0; j < c->ny; ++j) { hyv[j] = c->ys[j + 1] - c->ys[j]; ihyv[j] = 1.0 / hyv[j]; }
    if (c->precision == PDN_MIXED) {
        std::vector<float> a(hxv.begin(), hxv.end()), b(hyv.begin(), hyv.end());
        std::vector<float> ia(ihxv.begin(), ihxv.end()), ib(ihyv.begin(), ihyv.end());
        rc = upload(c, (float *)c->hx, a);
        if (!rc) rc = upload(c, (float *)c->hy, b);
        if (!rc) rc = upload(c, (float *)c->ihx, ia);
        if (!rc) rc = upload(c, (float *)c->ihy, ib);
        if (!rc) rc = hipStreamSynchronize(c->stream) == hipSuccess ? PDN_OK : PDN_EDEVICE;
    } else {
        rc = upload(c, (double *)c->hx, hxv);
        if (!rc) rc = upload(c, (double *)c->hy, hyv);
        if (!rc) rc = upload(c, (double *)c->ihx, ihxv);
        if (!rc) rc = upload(c, (double *)c->ihy, ihyv);
        if (!rc) rc = hipStreamSynchronize(c->stream) == hipSuccess ? PDN_OK : PDN_EDEVICE;
    }
    if (!rc) rc = upload(c, c->xs_d, c->xs);
    if (!rc) rc = upload(c, c->ys_d, c->ys);
    if (!rc) rc = upload(c, c->layers_d, c->layers);
    if (!rc) rc = upload(c, c->bulk_layer_d, c->bulk_layer);
    if (!rc) rc = upload(c, c->coh_layer_d, c->coh_layer);
    if (!rc) rc = upload(c, c->bcb_d, c->bcb);
    // zero state, thresholds r = 1 (Algorithm 4 initial state), r_D = 0
    if (!rc) {
        for (int b = 0; b < 2; ++b) {
            (void)hipMemsetAsync(c->d[b], 0, 3 * c->nn * sizeof(double), c->stream);
            (void)hipMemsetAsync(c->v[b], 0, 3 * c->nn * sizeof(double), c->stream);
        }
        (void)hipMemsetAsync(c->rd, 0, std::max<int64_t>(1, c->npairs) * rs, c->stream);
        if (c->ne > 0) {
            if (c->precision == PDN_MIXED) {
                std::vector<float> ones(4 * c->ngp * c->ne, 1.0f);
                rc = upload(c, (float *)c->r, ones);
                if (!rc && hipStreamSynchronize(c->stream) != hipSuccess) rc = PDN_EDEVICE;
            } else {
                std::vector<double> ones(4 * c->ngp * c->ne, 1.0);
                rc = upload(c, (double *)c->r, ones);
                if (!rc && hipStreamSynchronize(c->stream) != hipSuccess) rc = PDN_EDEVICE;
            }
        }
    }
    if (!rc && hipStreamSynchronize(c->stream) != hipSuccess) rc = set_err(c, PDN_EDEVICE, "mesh upload failed");
    if (rc) { free_all(c); if (c->own_stream) (void)hipStreamDestroy(c->stream); delete c; return rc; }
    *out = c;
    return PDN_OK;
}

int pdn_material_set(pdn_ctx *c, int32_t ply, const pdn_material *m)
{
    if (!c || !m) return PDN_EINVAL;
    if (c->broken) return set_err(c, PDN_EUNSTABLE, "context is unstable");
    if (ply < -1 || ply >= c->P) return set_err(c, PDN_EINVAL, "ply index %d out of range", ply);
    if (!(m->E1 > 0 && m->E2 > 0 && m->E3 > 0 && m->G12 > 0 && m->G13 > 0 && m->G23 > 0 && m->rho > 0))
        return set_err(c, PDN_EINVAL, "elastic constants and density must be positive");
    if (m->law < 0 || m->law > 2) return set_err(c, PDN_EINVAL, "unknown law %d", m->law);
    if (m->law != PDN_LAW_ELASTIC) {
        if (!(m->XT > 0 && m->XC > 0 && m->YT > 0 && m->YC > 0 && m->SL > 0 && m->GXT > 0 && m->GXC > 0 &&
              m->GYT > 0 && m->GYC > 0 && m->GSL > 0 && m->fXT > 0 && m->fXC > 0 && m->fGT > 0 && m->fGC > 0 &&
              m->fGT < 1 && m->fGC < 1))
            return set_err(c, PDN_EINVAL, "damage law needs positive strengths, toughness and shape factors");
        // fibre bilinear softening must stay ordered at the largest crack band of the ply
        double hxm = 0, hym = 0;
        for (int i = 0; i < c->nx; ++i) hxm = std::max(hxm, c->xs[i + 1] - c->xs[i]);
        for (int j = 0; j < c->ny; ++j) hym = std::max(hym, c->ys[j + 1] - c->ys[j]);
        const double lc = std::cbrt(hxm * hym * c->tply / c->epp);
        const double X[2] = {m->XT, m->XC}, G[2] = {m->GXT, m->GXC}, fx[2] = {m->fXT, m->fXC}, fg[2] = {m->fGT, m->fGC};
        for (int k = 0; k < 2; ++k) {
            double e0 = X[k] / m->E1, g = G[k] / lc;
            double eB = 2 * fg[k] * g / X[k] + fx[k] * e0, eC = 2 * (1 - fg[k]) * g / (fx[k] * X[k]);
            if (!(eB > e0 && eC > eB)) return set_err(c, PDN_EINVAL, "fibre softening not ordered at element size");
        }
    }
    if (c->cohesive && m->KI < 0) return set_err(c, PDN_EINVAL, "interface penalty must be positive");
    if (!(m->Sp >= 0 && m->Kp >= 0)) return set_err(c, PDN_EINVAL, "plasticity needs Sp >= 0 and Kp >= 0");
    if (m->Sp > 0 && m->law == PDN_LAW_CDM_SURROGATE)
        return set_err(c, PDN_EINVAL, "shear plasticity is built for the exact damage law, not the surrogate");
    if (ply_plastic(*m) && m->G13 != m->G12)
        return set_err(c, PDN_EINVAL, "shear plasticity needs an isotropic longitudinal shear plane (G13 = G12)");
    for (int p = 0; p < c->P; ++p)
        if (ply < 0 || p == ply) { c->mat[p] = *m; c->mat_set[p] = 1; }
    c->ready = false;
    if (c->gl.step > 0) {           // mid-run: re-run the element pass, keep the contact state
        c->needs_init = true;
        c->loaded_state = true;
    }
    return PDN_OK;
}

int pdn_impactor_set(pdn_ctx *c, const pdn_impactor *imp)
{
    if (!c || !imp) return PDN_EINVAL;
    if (c->broken) return set_err(c, PDN_EUNSTABLE, "context is unstable");
    if (!(imp->radius > 0 && imp->mass > 0 && imp->gap >= 0)) return set_err(c, PDN_EINVAL, "bad striker");
    if (!all_set(c)) return set_err(c, PDN_ESTATE, "set the materials of every ply first");
    (void)hipSetDevice(c->device);
    const double v0 = imp->energy > 0 ? std::sqrt(2.0 * imp->energy / imp->mass) : imp->v0;
    if (!c->have_imp || c->gl.step == 0) {
        c->imp = *imp;
        c->have_imp = true;
        int rc = alloc_contact_window(c);
        if (rc) return rc;
        DevGlobals &G = c->gl;
        std::memset(&G, 0, sizeof G);
        const double x0 = std::isnan(imp->x0) ? 0.5 * (c->xs[0] + c->xs[c->nx]) : imp->x0;
        const double y0 = std::isnan(imp->y0) ? 0.5 * (c->ys[0] + c->ys[c->ny]) : imp->y0;
        G.c0[0] = x0; G.c0[1] = y0; G.c0[2] = c->zk[c->K - 1] + imp->radius + imp->gap;
        std::memcpy(G.c, G.c0, sizeof G.c);
        G.V[2] = -v0;
        G.ms = imp->mass; G.R = imp->radius; G.g = c->grav; G.phi = c->phi;
        G.first = 1;
        G.ke0 = 0.5 * imp->mass * v0 * v0;
        G.e_kes = G.ke0;
        G.hist_cap = c->hist_cap;
        c->v0 = v0;
        c->needs_init = true;
        c->loaded_state = false;
        return PDN_OK;
    }
    // mid-run: only the velocity changes
    int rc = sync_globals_from_device(c);
    if (rc) return rc;
    c->gl.V[0] = 0; c->gl.V[1] = 0; c->gl.V[2] = -v0;
    return push_globals(c);
}

int pdn_step(pdn_ctx *c, int64_t n)
{
    if (!c) return PDN_EINVAL;
    if (n < 0) return set_err(c, PDN_EINVAL, "negative step count %lld", (long long)n);
    if (c->broken) return set_err(c, PDN_EUNSTABLE, "context is unstable");
    if (!all_set(c) || !c->have_imp) return set_err(c, PDN_ESTATE, "materials and striker must be set first");
    (void)hipSetDevice(c->device);
    int rc;
    if (!c->ready) {
        if ((rc = prepare(c))) return rc;
        c->gl.dt = c->dt;
        if (c->gl.step == 0 && !c->loaded_state) {
            if ((rc = push_globals(c))) return rc;
        } else {
            // material changed mid-run: keep the device books, refresh dt
            if ((rc = sync_globals_from_device(c))) return rc;
            c->gl.dt = c->dt;
            if ((rc = push_globals(c))) return rc;
        }
    }
    if (c->needs_init) {
        const bool reset_contact = !c->loaded_state;
        if ((rc = init_level(c, reset_contact))) return rc;
        c->loaded_state = false;
    }
    if ((rc = ensure_history(c, c->gl.step + n))) return rc;
    if (c->use_sur && n > 0) {
        // build for this call, from the previous call's points outside the screen
        const double outside = c->gl.sur_gp + c->gl.sur_unscreened;
        if (c->sur_mode != 0)
            c->sur_build = c->sur_mode;
        else
            c->sur_build = c->sur_fresh || c->sur_prev_n <= 0 || outside > c->sur_gp_mark ? 2 : 0;
        c->sur_fresh = false;
        c->sur_gp_mark = outside;
        c->sur_prev_n = n;
        if (c->sur_build != 0) c->sur_net_steps += n;
    }
    if (c->timing && n > 0) {
        if ((rc = timing_collect(c))) return rc;       // the previous call's, before its events are reused
        if ((rc = timing_pool(c, 2 * n + 1))) return rc;
    }
    hipEvent_t *ev = c->tev.data();
    // one pass per step: the element/node update of the whole plate with the
    // contact step (Algorithms 1-2) on its top plane, then the books kernel
    for (int64_t s = 0; s < n; ++s) {
        const int pred = 1 - c->cur;
        // a step's books kernel ends where the next step starts (two events per step)
        if (c->timing) HIPCHK(c, hipEventRecord(ev[2 * s], c->stream));
        if ((rc = launch_en(c, pred, c->cur, 1, c->timing ? ev[2 * s + 1] : nullptr))) return rc;
        c->cur = pred;
        c->cand_dirty = true;
    }
    if (c->timing && n > 0) HIPCHK(c, hipEventRecord(ev[2 * n], c->stream));
    if ((rc = sync_globals_from_device(c))) return rc;
    if (c->timing && n > 0) c->tev_n = n;                  // read by pdn_kernel_times
    if (c->gl.flag_unstable) {
        c->broken = true;
        return set_err(c, PDN_EUNSTABLE, "non-finite displacement at step %lld", (long long)c->gl.step);
    }
    if (c->gl.flag_overflow)
        return set_err(c, PDN_ERANGE, "contact reached the edge of the contact search window");
    return PDN_OK;
}

int pdn_contact_force(const pdn_ctx *c, double *t, double *force, double *disp, int64_t cap, int64_t *n_out)
{
    if (!c) return PDN_EINVAL;
    pdn_ctx *m = const_cast<pdn_ctx *>(c);
    const int64_t n = c->gl.step;
    if (n_out) *n_out = n;
    if (cap < n) return set_err(m, PDN_ERANGE, "history needs %lld entries", (long long)n);
    if (n == 0) return PDN_OK;
    (void)hipSetDevice(c->device);
    std::vector<double> h(3 * n);
    HIPCHK(m, hipMemcpyAsync(h.data(), c->hist_d, 3 * n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(m, hipStreamSynchronize(c->stream));
    for (int64_t i = 0; i < n; ++i) {
        if (t) t[i] = h[3 * i];
        if (force) force[i] = h[3 * i + 1];
        if (disp) disp[i] = h[3 * i + 2];
    }
    return PDN_OK;
}

int pdn_damage_field(const pdn_ctx *cc, int32_t kind, double *out, int64_t cap, int64_t *n_out)
{
    if (!cc) return PDN_EINVAL;
    pdn_ctx *c = const_cast<pdn_ctx *>(cc);
    if (kind < 0 || kind > 6) return set_err(c, PDN_EINVAL, "unknown damage field %d", kind);
    const bool proj = kind >= PDN_DMG_PROJ_FIBRE;
    const int base = proj ? (kind == PDN_DMG_PROJ_COHESIVE ? PDN_DMG_COHESIVE : kind - 4) : kind;
    const int64_t ncol = (int64_t)c->nx * c->ny;
    const int64_t nelem = base == PDN_DMG_COHESIVE ? c->nce : c->ne;
    const int64_t n = proj ? ncol : nelem;
    if (n_out) *n_out = n;
    if (cap < n) return set_err(c, PDN_ERANGE, "damage field needs %lld values", (long long)n);
    if (n == 0) return PDN_OK;
    if (!c->ready) {
        for (int64_t i = 0; i < n; ++i) out[i] = 0;
        return PDN_OK;
    }
    (void)hipSetDevice(c->device);
    const size_t need = (size_t)(nelem + ncol);
    if (c->dmg_n < need) {
        if (c->dmg_d) (void)hipFree(c->dmg_d);
        c->dmg_d = nullptr;
        int rc = dalloc(c, (void **)&c->dmg_d, need * sizeof(double));
        if (rc) return rc;
        c->dmg_n = need;
    }
    hipError_t e;
    if (base == PDN_DMG_COHESIVE) {
        if (c->precision == PDN_MIXED)
            e = pdn::launch_damage_coh<float>((const float *)c->rd, c->d[c->cur], c->layers_d, c->coh_layer_d,
                                              (const PlyC<float> *)c->ply, c->nx, c->ny, nelem, c->dmg_d, c->stream);
        else
            e = pdn::launch_damage_coh<double>((const double *)c->rd, c->d[c->cur], c->layers_d, c->coh_layer_d,
                                               (const PlyC<double> *)c->ply, c->nx, c->ny, nelem, c->dmg_d, c->stream);
    } else {
        if (c->precision == PDN_MIXED)
            e = pdn::launch_damage_bulk<float>((const float *)c->r, c->ngp, c->layers_d, c->bulk_layer_d,
                                               (const PlyC<float> *)c->ply, (const float *)c->hx,
                                               (const float *)c->hy, c->nx, c->ny, nelem, base, c->dmg_d, c->stream);
        else
            e = pdn::launch_damage_bulk<double>((const double *)c->r, c->ngp, c->layers_d, c->bulk_layer_d,
                                                (const PlyC<double> *)c->ply, (const double *)c->hx,
                                                (const double *)c->hy, c->nx, c->ny, nelem, base, c->dmg_d, c->stream);
    }
    if (e != hipSuccess) return set_err(c, PDN_EDEVICE, "damage kernel: %s", hipGetErrorString(e));
    const double *src = c->dmg_d;
    if (proj) {
        const int nl = (int)(nelem / std::max<int64_t>(1, ncol));
        e = pdn::launch_project_max(c->dmg_d, ncol, nl, c->dmg_d + nelem, c->stream);
        if (e != hipSuccess) return set_err(c, PDN_EDEVICE, "projection kernel: %s", hipGetErrorString(e));
        src = c->dmg_d + nelem;
    }
    HIPCHK(c, hipMemcpyAsync(out, src, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PDN_OK;
}

int pdn_energies(const pdn_ctx *c, pdn_energy *o)
{
    if (!c || !o) return PDN_EINVAL;
    const DevGlobals &G = c->gl;
    o->level = G.e_level;
    o->ke_plate = G.e_kep;
    o->ke_striker = G.e_kes;
    o->w_int = G.e_wint;
    o->w_grav = G.e_wgp + G.e_wgs;
    o->w_contact_plate = G.e_wc;
    o->w_striker = G.e_ws;
    o->d_pdn = G.e_ws - G.e_wc;
    o->ke0 = G.ke0;
    o->u_el = G.e_uel;
    o->residual = o->ke_plate + o->ke_striker + o->w_int + o->d_pdn - (o->ke0 + o->w_grav);
    return PDN_OK;
}

int pdn_info_get(const pdn_ctx *c, pdn_info *o)
{
    if (!c || !o) return PDN_EINVAL;
    std::memset(o, 0, sizeof *o);
    o->dt = c->dt;
    o->n_nodes = c->nn; o->n_bulk = c->ne; o->n_cohesive = c->nce; o->n_pairs = c->npairs;
    o->n_planes = c->K; o->n_layers = c->NL;
    o->n_candidates = (int64_t)(c->ci1 - c->ci0) * (c->cj1 - c->cj0);
    o->steps = c->gl.step; o->reset_passes = c->gl.reset_passes; o->released = c->gl.released;
    o->active = c->gl.active; o->max_passes = c->gl.max_passes;
    o->fallback_fraction = c->gl.sur_gp > 0 ? c->gl.fallback_gp / c->gl.sur_gp : 0.0;
    o->precision = c->precision;
    o->sur_consulted = c->gl.sur_gp;
    o->tile_x = pdn_tile_dims[c->tile][0];
    o->tile_y = pdn_tile_dims[c->tile][1];
    o->blocks = c->nblocks;
    o->sur_network_steps = c->sur_net_steps;
    return PDN_OK;
}

int pdn_array_get(const pdn_ctx *cc, int32_t kind, double *out, int64_t cap, int64_t *n_out)
{
    if (!cc) return PDN_EINVAL;
    pdn_ctx *c = const_cast<pdn_ctx *>(cc);
    int64_t n;
    switch (kind) {
    case PDN_ARR_DISP: case PDN_ARR_VEL: n = 3 * c->nn; break;
    case PDN_ARR_GP_R: n = 4 * c->ngp * c->ne; break;
    case PDN_ARR_COH_R: n = c->npairs; break;
    case PDN_ARR_MASS: n = c->nn; break;
    case PDN_ARR_GP_EP: n = 3 * c->ngp * c->ne; break;
    default: return set_err(c, PDN_EINVAL, "unknown array kind %d", kind);
    }
    if (n_out) *n_out = n;
    if (cap < n) return set_err(c, PDN_ERANGE, "array needs %lld values", (long long)n);
    if (n == 0) return PDN_OK;
    (void)hipSetDevice(c->device);
    if (kind == PDN_ARR_MASS) {
        if (!c->ready) return set_err(c, PDN_ESTATE, "mass is known after the first step");
        for (int k = 0; k < c->K; ++k)
            for (int j = 0; j <= c->ny; ++j)
                for (int i = 0; i <= c->nx; ++i)
                    out[i + (int64_t)(c->nx + 1) * (j + (int64_t)(c->ny + 1) * k)] = c->mx[i] * c->my[j] * c->mz[k];
        return PDN_OK;
    }
    if (kind == PDN_ARR_DISP || kind == PDN_ARR_VEL) {
        int rc = materialize(c);
        if (rc) return rc;
        const double *src = kind == PDN_ARR_DISP ? c->d[c->cur] : c->v[c->cur];
        HIPCHK(c, hipMemcpyAsync(out, src, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        return PDN_OK;
    }
    if (kind == PDN_ARR_GP_R || kind == PDN_ARR_GP_EP) {   // 4 words per GP record on the device
        const void *src = kind == PDN_ARR_GP_R ? c->r : c->ep;
        const int w = kind == PDN_ARR_GP_R ? 4 : 3;           // values per GP out
        if (!src) {
            for (int64_t i = 0; i < n; ++i) out[i] = 0.0;
            return PDN_OK;
        }
        const int64_t ng = c->ngp * c->ne;
        std::vector<double> all(4 * ng);
        if (c->precision == PDN_MIXED) {
            std::vector<float> tmp(4 * ng);
            HIPCHK(c, hipMemcpyAsync(tmp.data(), src, tmp.size() * sizeof(float), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
            for (size_t i = 0; i < tmp.size(); ++i) all[i] = tmp[i];
        } else {
            HIPCHK(c, hipMemcpyAsync(all.data(), src, all.size() * sizeof(double), hipMemcpyDeviceToHost, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
        for (int64_t k = 0; k < ng; ++k) {
            const int64_t rec = gp_record(c, k);
            for (int q = 0; q < w; ++q) out[w * k + q] = all[4 * rec + q];
        }
        return PDN_OK;
    }
    const void *src = c->rd;
    if (c->precision == PDN_MIXED) {
        std::vector<float> tmp(n);
        HIPCHK(c, hipMemcpyAsync(tmp.data(), src, n * sizeof(float), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        for (int64_t i = 0; i < n; ++i) out[i] = tmp[i];
    } else {
        HIPCHK(c, hipMemcpyAsync(out, src, n * sizeof(double), hipMemcpyDeviceToHost, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    }
    return PDN_OK;
}

int pdn_array_set(pdn_ctx *c, int32_t kind, const double *in, int64_t n)
{
    if (!c || !in) return PDN_EINVAL;
    if (c->broken) return set_err(c, PDN_EUNSTABLE, "context is unstable");
    int64_t need;
    switch (kind) {
    case PDN_ARR_DISP: case PDN_ARR_VEL: need = 3 * c->nn; break;
    case PDN_ARR_GP_R: need = 4 * c->ngp * c->ne; break;
    case PDN_ARR_COH_R: need = c->npairs; break;
    case PDN_ARR_GP_EP:
        need = 3 * c->ngp * c->ne;
        if (!c->ep) return set_err(c, PDN_EINVAL, "no plastic state: no ply has shear plasticity (or no step yet)");
        break;
    default: return set_err(c, PDN_EINVAL, "array kind %d cannot be set", kind);
    }
    if (n != need) return set_err(c, PDN_EINVAL, "array needs %lld values, got %lld", (long long)need, (long long)n);
    (void)hipSetDevice(c->device);
    if (kind == PDN_ARR_DISP || kind == PDN_ARR_VEL) {
        // first the corrected candidates of the last step into both arrays (the
        // array not replaced here keeps them)
        int rc0 = materialize(c);
        if (rc0) return rc0;
        // supported DOFs stay at rest
        std::vector<double> tmp(in, in + n);
        for (int k = 0; k < c->K; ++k)
            for (int j = 0; j <= c->ny; ++j)
                for (int i = 0; i <= c->nx; ++i) {
                    const int64_t col = i + (int64_t)(c->nx + 1) * j, nd = col + c->plane * k;
                    int bits = (c->bc == PDN_BC_CLAMPED_EDGES && (i == 0 || i == c->nx || j == 0 || j == c->ny)) ? 7 : 0;
                    if (k == 0) bits |= c->bcb[col];
                    for (int q = 0; q < 3; ++q)
                        if ((bits >> q) & 1) tmp[3 * nd + q] = 0.0;
                }
        double *dst = kind == PDN_ARR_DISP ? c->d[c->cur] : c->v[c->cur];
        HIPCHK(c, hipMemcpyAsync(dst, tmp.data(), n * sizeof(double), hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
    } else if (kind == PDN_ARR_GP_R || kind == PDN_ARR_GP_EP) {
        void *dst = kind == PDN_ARR_GP_R ? c->r : c->ep;
        const int w = kind == PDN_ARR_GP_R ? 4 : 3;           // values per GP in
        const int64_t ng = c->ngp * c->ne;
        std::vector<double> all(4 * ng, 0.0);
        for (int64_t k = 0; k < ng; ++k) {
            const int64_t rec = gp_record(c, k);
            for (int q = 0; q < w; ++q) all[4 * rec + q] = in[w * k + q];
        }
        if (c->precision == PDN_MIXED) {
            std::vector<float> tmp(all.begin(), all.end());
            HIPCHK(c, hipMemcpyAsync(dst, tmp.data(), tmp.size() * sizeof(float), hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        } else {
            HIPCHK(c, hipMemcpyAsync(dst, all.data(), all.size() * sizeof(double), hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
    } else {
        if (c->precision == PDN_MIXED) {
            std::vector<float> tmp(in, in + n);
            HIPCHK(c, hipMemcpyAsync(c->rd, tmp.data(), n * sizeof(float), hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        } else {
            HIPCHK(c, hipMemcpyAsync(c->rd, in, n * sizeof(double), hipMemcpyHostToDevice, c->stream));
            HIPCHK(c, hipStreamSynchronize(c->stream));
        }
    }
    c->needs_init = true;
    c->loaded_state = false;
    // the books restart from this state
    if (c->have_imp) {
        int rc = c->gl.step > 0 ? sync_globals_from_device(c) : PDN_OK;
        if (rc) return rc;
        DevGlobals &G = c->gl;
        G.first = 1;
        G.e_wint = G.e_wgp = G.e_wc = G.half_int = 0;
        if (c->ready) return push_globals(c);
    }
    return PDN_OK;
}

// ---- checkpoint ----------------------------------------------------------
namespace {
struct BlobHeader {
    uint64_t magic;
    int64_t nn, ne, npairs, ncand, hist_n;
    int32_t precision, cur;
    int32_t ngp, pad;
};
const uint64_t kMagic = 0x32304b4350444e50ull;   // "PNDPCK02"
}  // namespace

int pdn_state_save(const pdn_ctx *cc, void *buf, int64_t cap, int64_t *n_out)
{
    if (!cc) return PDN_EINVAL;
    pdn_ctx *c = const_cast<pdn_ctx *>(cc);
    if (!c->ready || c->needs_init) return set_err(c, PDN_ESTATE, "checkpoint needs at least one completed step");
    const size_t rs = rsize(c);
    const int64_t ncand = (int64_t)(c->ci1 - c->ci0) * (c->cj1 - c->cj0);
    const int64_t hn = c->gl.step;
    const size_t eps_bytes = c->plastic ? 4 * c->ngp * c->ne * rs : 0;
    const size_t need = sizeof(BlobHeader) + sizeof(DevGlobals) + 2 * 3 * c->nn * sizeof(double) +
                        4 * c->ngp * c->ne * rs + eps_bytes +
                        c->npairs * rs + ncand * (1 + 6 * sizeof(double)) + 3 * hn * sizeof(double);
    if (n_out) *n_out = (int64_t)need;
    if (cap < (int64_t)need || !buf) return set_err(c, PDN_ERANGE, "checkpoint needs %zu bytes", need);
    (void)hipSetDevice(c->device);
    int rc = sync_globals_from_device(c);
    if (!rc) rc = materialize(c);
    if (rc) return rc;
    char *p = (char *)buf;
    BlobHeader h{kMagic, c->nn, c->ne, c->npairs, ncand, hn, c->precision, 0, c->ngp, c->plastic ? 1 : 0};
    std::memcpy(p, &h, sizeof h); p += sizeof h;
    std::memcpy(p, &c->gl, sizeof(DevGlobals)); p += sizeof(DevGlobals);
    auto d2h = [&](const void *src, size_t bytes) -> int {
        if (bytes == 0) return PDN_OK;
        HIPCHK(c, hipMemcpyAsync(p, src, bytes, hipMemcpyDeviceToHost, c->stream));
        p += bytes;
        return PDN_OK;
    };
    if ((rc = d2h(c->d[c->cur], 3 * c->nn * sizeof(double)))) return rc;
    if ((rc = d2h(c->v[c->cur], 3 * c->nn * sizeof(double)))) return rc;
    if ((rc = d2h(c->r, 4 * c->ngp * c->ne * rs))) return rc;
    if (eps_bytes && (rc = d2h(c->ep, eps_bytes))) return rc;
    if ((rc = d2h(c->rd, c->npairs * rs))) return rc;
    if ((rc = d2h(c->active_d + (size_t)(1 - c->cur) * ncand, ncand))) return rc;   // read by the next step
    if ((rc = d2h(c->vprev_d, 3 * ncand * sizeof(double)))) return rc;
    if ((rc = d2h(c->fcprev_d, 3 * ncand * sizeof(double)))) return rc;
    if ((rc = d2h(c->hist_d, 3 * hn * sizeof(double)))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    return PDN_OK;
}

int pdn_state_load(pdn_ctx *c, const void *buf, int64_t n)
{
    if (!c || !buf) return PDN_EINVAL;
    if (!all_set(c) || !c->have_imp) return set_err(c, PDN_ESTATE, "set materials and striker before loading");
    const char *p = (const char *)buf;
    if (n < (int64_t)sizeof(BlobHeader)) return set_err(c, PDN_EINVAL, "checkpoint too short");
    BlobHeader h;
    std::memcpy(&h, p, sizeof h); p += sizeof h;
    const int64_t ncand = (int64_t)(c->ci1 - c->ci0) * (c->cj1 - c->cj0);
    bool plas = false;
    for (int p = 0; p < c->P; ++p) plas = plas || ply_plastic(c->mat[p]);
    if (h.magic != kMagic || h.nn != c->nn || h.ne != c->ne || h.npairs != c->npairs || h.ncand != ncand ||
        h.precision != c->precision || h.ngp != c->ngp || h.pad != (plas ? 1 : 0))
        return set_err(c, PDN_EINVAL, "checkpoint does not match this context");
    // the blob must be exactly what pdn_state_save writes for this context and
    // history length; nothing is read or changed before this holds
    const size_t rs = rsize(c);
    const size_t eps_bytes = plas ? 4 * c->ngp * c->ne * rs : 0;
    const size_t fixed = sizeof(BlobHeader) + sizeof(DevGlobals) + 2 * 3 * c->nn * sizeof(double) +
                         4 * c->ngp * c->ne * rs + eps_bytes + c->npairs * rs + ncand * (1 + 6 * sizeof(double));
    if (h.hist_n < 0 || (uint64_t)h.hist_n > ((uint64_t)INT64_MAX - fixed) / (3 * sizeof(double)))
        return set_err(c, PDN_EINVAL, "checkpoint history length %lld is invalid", (long long)h.hist_n);
    const size_t need = fixed + 3 * (size_t)h.hist_n * sizeof(double);
    if ((uint64_t)n != (uint64_t)need)
        return set_err(c, PDN_EINVAL, "checkpoint has %lld bytes, this context's checkpoint with %lld steps has %zu",
                       (long long)n, (long long)h.hist_n, need);
    DevGlobals g;
    std::memcpy(&g, p, sizeof g); p += sizeof g;
    if (g.step != h.hist_n) return set_err(c, PDN_EINVAL, "checkpoint step count does not match its history");
    (void)hipSetDevice(c->device);
    int rc;
    if (!c->ready && (rc = prepare(c))) return rc;
    if ((rc = ensure_history(c, h.hist_n + 1))) return rc;
    c->gl = g;
    c->gl.hist_cap = c->hist_cap;
    auto h2d = [&](void *dst, size_t bytes) -> int {
        if (bytes == 0) return PDN_OK;
        HIPCHK(c, hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, c->stream));
        p += bytes;
        return PDN_OK;
    };
    c->cur = 0;
    if ((rc = h2d(c->d[0], 3 * c->nn * sizeof(double)))) return rc;
    if ((rc = h2d(c->v[0], 3 * c->nn * sizeof(double)))) return rc;
    if ((rc = h2d(c->r, 4 * c->ngp * c->ne * rs))) return rc;
    if (eps_bytes && (rc = h2d(c->ep, eps_bytes))) return rc;
    if ((rc = h2d(c->rd, c->npairs * rs))) return rc;
    if ((rc = h2d(c->active_d + ncand, ncand))) return rc;            // cur = 0: the next step reads set 1
    if ((rc = h2d(c->vprev_d, 3 * ncand * sizeof(double)))) return rc;
    if ((rc = h2d(c->fcprev_d, 3 * ncand * sizeof(double)))) return rc;
    if ((rc = h2d(c->hist_d, 3 * h.hist_n * sizeof(double)))) return rc;
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if ((rc = push_globals(c))) return rc;
    c->needs_init = true;
    c->loaded_state = true;
    c->cand_dirty = false;
    return PDN_OK;
}

int pdn_set_tile(pdn_ctx *c, int32_t tx, int32_t ty)
{
    if (!c) return PDN_EINVAL;
    int t = -1;
    if (tx == 0 && ty == 0) t = PDN_TILE_15x15;
    for (int k = 0; k < PDN_TILE_COUNT; ++k)
        if (pdn_tile_dims[k][0] == tx && pdn_tile_dims[k][1] == ty) t = k;
    if (t < 0) return set_err(c, PDN_EINVAL, "unsupported tile %dx%d", tx, ty);
    if (c->ngp == 8 && !pdn::tile_has_full(t))
        return set_err(c, PDN_EINVAL, "full integration is built for the 15x15 and 16x16 tiles");
    if (!tile_fits(c, t)) return set_err(c, PDN_EINVAL, "tile %dx%d does not fit the device's LDS", tx, ty);
    const int old = c->nblocks;
    c->tile = t;
    set_tiles(c);
    (void)old;
    if (c->nblocks > c->prow) {
        (void)hipFree(c->partials_d);
        c->partials_d = nullptr;
        c->prow = c->nblocks;
        int rc = dalloc(c, (void **)&c->partials_d, partials_bytes(c->prow));
        if (rc) return rc;
    }
    // a contact pass reduces the partials of the previous pass: recompute them
    // in the new block layout, keeping the contact state
    if (!c->needs_init) {
        c->needs_init = true;
        c->loaded_state = true;
    }
    return PDN_OK;
}

int pdn_kernel_times(const pdn_ctx *cc, double *en, double *bk)
{
    if (!cc) return PDN_EINVAL;
    pdn_ctx *c = const_cast<pdn_ctx *>(cc);
    (void)hipSetDevice(c->device);
    int rc = timing_collect(c);
    if (rc) return rc;
    if (en) *en = c->t_en_ms;
    if (bk) *bk = c->t_bk_ms;
    return PDN_OK;
}

int pdn_set_timing(pdn_ctx *c, int32_t on)
{
    if (!c) return PDN_EINVAL;
    c->timing = on != 0;
    (void)hipSetDevice(c->device);
    return c->timing ? timing_pool(c, 2 * 1024 + 1) : PDN_OK;   // events for calls of up to 1,024 steps
}

const char *pdn_last_error(const pdn_ctx *c) { return c ? c->err.c_str() : "null context"; }

void pdn_destroy(pdn_ctx *c)
{
    if (!c) return;
    (void)hipSetDevice(c->device);
    (void)hipStreamSynchronize(c->stream);
    free_all(c);
    for (hipEvent_t e : c->tev) (void)hipEventDestroy(e);
    if (c->own_stream) (void)hipStreamDestroy(c->stream);
    delete c;
}

}  // extern "C"

// ---- autotuner and batched stepping --------------------------------------
struct pdn_batch {
    std::string err;
    std::vector<pdn_ctx *> cs;
    int device = 0, precision = 0, tile = -1;
    int ngp = 1;                         // element integration shared by all cases
    hipStream_t stream = nullptr;        // stream of the first case; every step runs here
    hipStream_t cap = nullptr;           // private stream used only to capture the step graph
    // 3 x n element-pass arguments: steps of parity 0 and 1 (contact pass), and
    // a restart pass of the current state (no contact) for the autotuner
    void *eargs_d = nullptr;
    // block offsets of the cases (n + 1), then per block its case and its
    // tile within the case (eblocks each)
    int *estart_d = nullptr;
    size_t estart_cap = 0;               // ints allocated at estart_d
    std::vector<int> estart;
    std::vector<unsigned char> eargs_h;
    int eblocks = 0;
    bool sur = false;                    // some case evaluates a surrogate network
    hipGraphExec_t exec = nullptr;       // PDN_BATCH_GRAPH_STEPS steps, built for (tile, sur, eblocks)
    int graph_tile = -1, graph_eblocks = 0;
    bool graph_sur = false;
    const int *graph_estart = nullptr;   // block table the graph's launches read
};

#define PDN_BATCH_GRAPH_STEPS 8          // even: a replay returns every case to the same buffer parity

namespace {

int berr(pdn_batch *b, int code, const char *fmt, ...)
{
    if (b) {
        char buf[512];
        va_list ap;
        va_start(ap, fmt);
        vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        b->err = buf;
    }
    return code;
}

#define BHIPCHK(b, call)                                                                        \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return berr(b, e_ == hipErrorOutOfMemory ? PDN_ENOMEM : PDN_EDEVICE, "%s: %s",     \
                        #call, hipGetErrorString(e_));                                          \
    } while (0)

const int kTileOrder[PDN_TILE_COUNT] = {PDN_TILE_15x15, PDN_TILE_16x16, PDN_TILE_31x15, PDN_TILE_32x8,
                                        PDN_TILE_8x8};

// tile measured fastest, per plate shape (single plates) or per batch composition
std::map<std::string, int> &tune_cache()
{
    static std::map<std::string, int> m;
    return m;
}

std::string shape_key(const pdn_ctx *c)
{
    char k[96];
    snprintf(k, sizeof k, "%d:%d:%d:%d:%d:%d:%d;", c->device, c->precision, (int)c->use_sur, c->ngp, c->nx, c->ny,
             c->K);
    return k;
}

// Put a context in tile layout t and re-run its element pass in that layout
// (the pass recomputes the predictor from the last completed level, so it
// changes no state: running it again gives the same outputs).
int use_tile(pdn_ctx *c, int t)
{
    int rc = pdn_set_tile(c, pdn_tile_dims[t][0], pdn_tile_dims[t][1]);
    if (!rc) rc = pdn_step(c, 0);
    return rc;
}

// mean time of `reps` element passes of one context in its current layout
int time_single(pdn_ctx *c, int reps, float *ms)
{
    hipEvent_t e0, e1;
    HIPCHK(c, hipEventCreate(&e0));
    HIPCHK(c, hipEventCreate(&e1));
    int rc = materialize(c);
    if (!rc) rc = launch_en(c, c->cur, 1 - c->cur, 0);     // warm
    if (!rc) HIPCHK(c, hipEventRecord(e0, c->stream));
    for (int r = 0; r < reps && !rc; ++r) rc = launch_en(c, c->cur, 1 - c->cur, 0);
    if (!rc) HIPCHK(c, hipEventRecord(e1, c->stream));
    if (!rc) HIPCHK(c, hipEventSynchronize(e1));
    if (!rc) HIPCHK(c, hipEventElapsedTime(ms, e0, e1));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (!rc) *ms /= reps;
    return rc;
}

template <typename R>
void fill_eargs(pdn_batch *b)
{
    const size_t n = b->cs.size();
    b->eargs_h.resize(3 * n * sizeof(ElemArgs<R>));
    ElemArgs<R> *ea = reinterpret_cast<ElemArgs<R> *>(b->eargs_h.data());
    for (int p = 0; p < 2; ++p)
        for (size_t i = 0; i < n; ++i) {
            pdn_ctx *c = b->cs[i];
            const int cur = c->cur ^ p, pred = 1 - cur;     // state of case i at a step of parity p
            ea[p * n + i] = elem_args<R>(c, pred, cur, 1);
        }
    for (size_t i = 0; i < n; ++i) ea[2 * n + i] = elem_args<R>(b->cs[i], b->cs[i]->cur, 1 - b->cs[i]->cur, 0);
}

// argument tables and block offsets of the current layout, uploaded to the device
int upload_tables(pdn_batch *b)
{
    const size_t n = b->cs.size();
    b->estart.assign(n + 1, 0);
    for (size_t i = 0; i < n; ++i) b->estart[i + 1] = b->estart[i] + b->cs[i]->nblocks;
    b->eblocks = b->estart[n];
    // Dispatch order of the blocks.  The hardware deals blocks round-robin to
    // the 8 XCDs, and xcd_tile hands each XCD a contiguous eighth of this list.
    // Every eighth holds the same band of every case's tiles, so the XCDs get
    // equal work although the cases differ in thickness (a block's time grows
    // with its layers); within a band a case's tiles stay contiguous, so
    // neighbouring tiles share an L2.
    b->estart.resize(n + 1 + 2 * (size_t)b->eblocks);
    int *bcase = b->estart.data() + n + 1, *btile = bcase + b->eblocks;
    size_t k = 0;
    for (int x = 0; x < 8; ++x)
        for (size_t i = 0; i < n; ++i) {
            const int nb = b->cs[i]->nblocks;
            for (int t = (int)((int64_t)nb * x / 8); t < (int)((int64_t)nb * (x + 1) / 8); ++t) {
                bcase[k] = (int)i;
                btile[k] = t;
                ++k;
            }
        }
    if (k != (size_t)b->eblocks) return berr(b, PDN_EDEVICE, "block table: %zu of %d blocks", k, b->eblocks);
    b->sur = false;
    for (pdn_ctx *c : b->cs) b->sur = b->sur || c->use_sur;
    if (b->precision == PDN_MIXED) fill_eargs<float>(b);
    else fill_eargs<double>(b);
    if (!b->eargs_d) BHIPCHK(b, hipMalloc(&b->eargs_d, b->eargs_h.size()));
    if (b->estart.size() > b->estart_cap) {                // the block count depends on the tile
        BHIPCHK(b, hipStreamSynchronize(b->stream));
        if (b->estart_d) BHIPCHK(b, hipFree(b->estart_d));
        b->estart_d = nullptr;
        BHIPCHK(b, hipMalloc((void **)&b->estart_d, b->estart.size() * sizeof(int)));
        b->estart_cap = b->estart.size();
    }
    BHIPCHK(b, hipMemcpyAsync(b->eargs_d, b->eargs_h.data(), b->eargs_h.size(), hipMemcpyHostToDevice, b->stream));
    BHIPCHK(b, hipMemcpyAsync(b->estart_d, b->estart.data(), b->estart.size() * sizeof(int), hipMemcpyHostToDevice,
                              b->stream));
    BHIPCHK(b, hipStreamSynchronize(b->stream));          // host tables are reused
    return PDN_OK;
}

// table 0, 1: contact passes of the two step parities; table 2: restart passes
hipError_t launch_batch_elem(pdn_batch *b, int table, hipStream_t s)
{
    const int n = (int)b->cs.size();
    const bool contact = table < 2;
    if (b->precision == PDN_MIXED)
        return pdn::launch_elem_node_batch<float>(reinterpret_cast<ElemArgs<float> *>(b->eargs_d) + table * n,
                                                  b->estart_d, n, b->eblocks, b->tile, b->sur, b->ngp, contact, s);
    return pdn::launch_elem_node_batch<double>(reinterpret_cast<ElemArgs<double> *>(b->eargs_d) + table * n,
                                               b->estart_d, n, b->eblocks, b->tile, b->sur, b->ngp, contact, s);
}

// one step of every case: a contact + element/node pass
hipError_t launch_batch_step(pdn_batch *b, int parity, hipStream_t s) { return launch_batch_elem(b, parity, s); }

// Mean time of `reps` batched element passes.  The passes use the restart
// tables (no contact), which read the last completed level and write the next
// predictor (what the pass after a step already wrote), so no state changes.
int time_batch(pdn_batch *b, int reps, float *ms)
{
    hipEvent_t e0, e1;
    BHIPCHK(b, hipEventCreate(&e0));
    BHIPCHK(b, hipEventCreate(&e1));
    hipError_t e = launch_batch_elem(b, 2, b->stream);      // warm
    if (e == hipSuccess) e = hipEventRecord(e0, b->stream);
    for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_batch_elem(b, 2, b->stream);
    if (e == hipSuccess) e = hipEventRecord(e1, b->stream);
    if (e == hipSuccess) e = hipEventSynchronize(e1);
    if (e == hipSuccess) e = hipEventElapsedTime(ms, e0, e1);
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    if (e != hipSuccess) return berr(b, PDN_EDEVICE, "batch timing: %s", hipGetErrorString(e));
    *ms /= reps;
    return PDN_OK;
}

int batch_case_err(pdn_batch *b, size_t i, int rc)
{
    return berr(b, rc, "case %zu: %s", i, b->cs[i]->err.c_str());
}

// all cases in tile layout t, ready to step, tables uploaded
int batch_use_tile(pdn_batch *b, int t)
{
    for (size_t i = 0; i < b->cs.size(); ++i) {
        int rc = use_tile(b->cs[i], t);
        if (rc) return batch_case_err(b, i, rc);
    }
    b->tile = t;
    return upload_tables(b);
}

int build_graph(pdn_batch *b)
{
    if (b->exec) {
        (void)hipGraphExecDestroy(b->exec);
        b->exec = nullptr;
    }
    hipGraph_t g = nullptr;
    BHIPCHK(b, hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    hipError_t e = hipSuccess;
    for (int s = 0; s < PDN_BATCH_GRAPH_STEPS && e == hipSuccess; ++s) e = launch_batch_step(b, s & 1, b->cap);
    hipError_t e2 = hipStreamEndCapture(b->cap, &g);
    if (e != hipSuccess || e2 != hipSuccess) {
        if (g) (void)hipGraphDestroy(g);
        return berr(b, PDN_EDEVICE, "step graph capture: %s",
                    hipGetErrorString(e != hipSuccess ? e : e2));
    }
    e = hipGraphInstantiateWithFlags(&b->exec, g, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) return berr(b, PDN_EDEVICE, "step graph instantiation: %s", hipGetErrorString(e));
    b->graph_tile = b->tile;
    b->graph_sur = b->sur;
    b->graph_eblocks = b->eblocks;
    b->graph_estart = b->estart_d;
    return PDN_OK;
}

}  // namespace

extern "C" {

int pdn_autotune(pdn_ctx *c, int32_t *tile_x, int32_t *tile_y)
{
    if (!c) return PDN_EINVAL;
    if (c->broken) return set_err(c, PDN_EUNSTABLE, "context is unstable");
    if (!all_set(c) || !c->have_imp) return set_err(c, PDN_ESTATE, "materials and striker must be set first");
    (void)hipSetDevice(c->device);
    bool plas = false;
    for (int p = 0; p < c->P; ++p) plas = plas || ply_plastic(c->mat[p]);
    const std::string key = std::string(plas ? "1p|" : "1|") + shape_key(c);
    auto it = tune_cache().find(key);
    int best = -1, rc;
    if (it != tune_cache().end()) {
        best = it->second;
    } else {
        // The passes timed are restart passes (no contact step, no books
        // kernel, whose work grows with the number of tiles): another shape
        // replaces the default 15 x 15 only when it is faster by a margin.
        float best_ms = 0, dflt_ms = -1;
        for (int t : kTileOrder) {
            if (!tile_fits(c, t) || (c->ngp == 8 && !pdn::tile_has_full(t)) || (plas && !pdn::tile_has_plas(t)))
                continue;
            float ms = 0;
            if ((rc = use_tile(c, t)) || (rc = time_single(c, 10, &ms))) return rc;
            if (t == PDN_TILE_15x15) dflt_ms = ms;
            if (best < 0 || ms < best_ms) { best = t; best_ms = ms; }
        }
        if (best < 0) return set_err(c, PDN_EINVAL, "no element tile fits this device");
        if (dflt_ms > 0 && best != PDN_TILE_15x15 && best_ms > 0.95f * dflt_ms) best = PDN_TILE_15x15;
        tune_cache()[key] = best;
    }
    if ((rc = use_tile(c, best))) return rc;
    if (tile_x) *tile_x = pdn_tile_dims[best][0];
    if (tile_y) *tile_y = pdn_tile_dims[best][1];
    return PDN_OK;
}

int pdn_batch_create(pdn_ctx *const *cases, int32_t n, pdn_batch **out)
{
    if (!out) return PDN_EINVAL;
    *out = nullptr;
    if (!cases || n < 1) return PDN_EINVAL;
    for (int32_t i = 0; i < n; ++i) {
        // the reason goes to the first case's error message
        pdn_ctx *c = cases[i];
        if (!c) return set_err(cases[0], PDN_EINVAL, "case %d is null", i);
        for (int32_t j = 0; j < i; ++j)
            if (cases[j] == c) return set_err(cases[0], PDN_EINVAL, "case %d repeats case %d", i, j);
        if (c->broken) return set_err(cases[0], PDN_EUNSTABLE, "case %d is unstable", i);
        if (!all_set(c) || !c->have_imp)
            return set_err(cases[0], PDN_ESTATE, "case %d: materials and striker must be set first", i);
        if (c->device != cases[0]->device || c->precision != cases[0]->precision || c->ngp != cases[0]->ngp)
            return set_err(cases[0], PDN_EINVAL,
                           "case %d: batched cases must share device, precision and element integration", i);
        for (int p = 0; p < c->P; ++p)
            if (ply_plastic(c->mat[p]))
                return set_err(cases[0], PDN_EINVAL, "case %d: shear plasticity is not built for batches", i);
    }
    pdn_batch *b = new pdn_batch;
    b->cs.assign(cases, cases + n);
    b->device = cases[0]->device;
    b->precision = cases[0]->precision;
    b->ngp = cases[0]->ngp;
    b->stream = cases[0]->stream;
    (void)hipSetDevice(b->device);
    if (hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) {
        delete b;
        return PDN_EDEVICE;
    }
    for (pdn_ctx *c : b->cs) (void)hipStreamSynchronize(c->stream);
    // autotuner: time one batched element pass per tile shape that fits
    std::string key = "B|";
    for (pdn_ctx *c : b->cs) key += shape_key(c);
    int rc = PDN_OK, best = -1;
    auto it = tune_cache().find(key);
    if (it != tune_cache().end()) {
        best = it->second;
    } else {
        float best_ms = 0;
        for (int t : kTileOrder) {
            bool fits = b->ngp == 1 || pdn::tile_has_full(t);
            for (pdn_ctx *c : b->cs) fits = fits && tile_fits(c, t);
            if (!fits) continue;
            float ms = 0;
            if ((rc = batch_use_tile(b, t)) || (rc = time_batch(b, 3, &ms))) break;
            if (best < 0 || ms < best_ms) { best = t; best_ms = ms; }
        }
        if (!rc && best < 0) rc = berr(b, PDN_EINVAL, "no element tile fits this device");
        if (!rc) tune_cache()[key] = best;
    }
    if (!rc) rc = batch_use_tile(b, best);
    if (!rc) rc = build_graph(b);
    if (rc) {
        set_err(cases[0], rc, "batch: %s", b->err.c_str());      // the batch is gone; keep the reason
        pdn_batch_destroy(b);
        return rc;
    }
    *out = b;
    return PDN_OK;
}

int pdn_batch_step(pdn_batch *b, int64_t n)
{
    if (!b || n < 0) return PDN_EINVAL;
    (void)hipSetDevice(b->device);
    int rc;
    for (size_t i = 0; i < b->cs.size(); ++i) {
        pdn_ctx *c = b->cs[i];
        if (c->broken) return berr(b, PDN_EUNSTABLE, "case %zu is unstable", i);
        if (c->tile != b->tile) {
            if ((rc = use_tile(c, b->tile))) return batch_case_err(b, i, rc);
        } else if ((rc = pdn_step(c, 0))) {          // pending (re)initialisation, if any
            return batch_case_err(b, i, rc);
        }
        if ((rc = ensure_history(c, c->gl.step + n))) return batch_case_err(b, i, rc);
        (void)hipStreamSynchronize(c->stream);
    }
    if ((rc = upload_tables(b))) return rc;
    if (b->graph_tile != b->tile || b->graph_sur != b->sur || b->graph_eblocks != b->eblocks ||
        b->graph_estart != b->estart_d)
        if ((rc = build_graph(b))) return rc;
    int64_t s = 0;
    for (; s + PDN_BATCH_GRAPH_STEPS <= n; s += PDN_BATCH_GRAPH_STEPS)
        BHIPCHK(b, hipGraphLaunch(b->exec, b->stream));
    for (; s < n; ++s) {
        hipError_t e = launch_batch_step(b, (int)(s & 1), b->stream);
        if (e != hipSuccess) return berr(b, PDN_EDEVICE, "batched step launch: %s", hipGetErrorString(e));
    }
    BHIPCHK(b, hipStreamSynchronize(b->stream));
    rc = PDN_OK;
    for (size_t i = 0; i < b->cs.size(); ++i) {
        pdn_ctx *c = b->cs[i];
        if (n & 1) c->cur ^= 1;
        if (n > 0) c->cand_dirty = true;
        int r2 = sync_globals_from_device(c);
        if (r2) return batch_case_err(b, i, r2);
        if (c->gl.flag_unstable) {
            c->broken = true;
            set_err(c, PDN_EUNSTABLE, "non-finite displacement at step %lld", (long long)c->gl.step);
            if (!rc) rc = berr(b, PDN_EUNSTABLE, "case %zu: non-finite state", i);
        } else if (c->gl.flag_overflow && !rc) {
            set_err(c, PDN_ERANGE, "contact reached the edge of the contact search window");
            rc = berr(b, PDN_ERANGE, "case %zu: contact reached the edge of the search window", i);
        }
    }
    return rc;
}

int pdn_batch_info(const pdn_batch *b, int32_t *tile_x, int32_t *tile_y, int64_t *n_bulk, int32_t *blocks)
{
    if (!b) return PDN_EINVAL;
    int64_t ne = 0;
    for (const pdn_ctx *c : b->cs) ne += c->ne;
    if (tile_x) *tile_x = b->tile >= 0 ? pdn_tile_dims[b->tile][0] : 0;
    if (tile_y) *tile_y = b->tile >= 0 ? pdn_tile_dims[b->tile][1] : 0;
    if (n_bulk) *n_bulk = ne;
    if (blocks) *blocks = b->eblocks;
    return PDN_OK;
}

const char *pdn_batch_last_error(const pdn_batch *b) { return b ? b->err.c_str() : "null batch"; }

void pdn_batch_destroy(pdn_batch *b)
{
    if (!b) return;
    (void)hipSetDevice(b->device);
    if (b->stream) (void)hipStreamSynchronize(b->stream);
    if (b->exec) (void)hipGraphExecDestroy(b->exec);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    if (b->eargs_d) (void)hipFree(b->eargs_d);
    if (b->estart_d) (void)hipFree(b->estart_d);
    delete b;
}

}  // extern "C"

// ---- constitutive surrogate ----------------------------------------------
namespace {

thread_local std::string g_err;

int gerr(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

#define GHIPCHK(call)                                                                           \
    do {                                                                                        \
        hipError_t e_ = (call);                                                                 \
        if (e_ != hipSuccess)                                                                   \
            return gerr(e_ == hipErrorOutOfMemory ? PDN_ENOMEM : PDN_EDEVICE, "%s: %s", #call,  \
                        hipGetErrorString(e_));                                                 \
    } while (0)

// device buffers released on scope exit
struct DevMem {
    std::vector<void *> ps;
    ~DevMem()
    {
        for (void *p : ps) (void)hipFree(p);
    }
    template <typename T>
    hipError_t get(T **p, size_t bytes)
    {
        *p = nullptr;
        hipError_t e = hipMalloc((void **)p, bytes ? bytes : 1);
        if (e == hipSuccess) ps.push_back((void *)*p);
        return e;
    }
};

// Glorot-uniform weights from SplitMix64(seed), zero biases
void sur_init(uint64_t seed, std::vector<float> &w)
{
    w.assign(SUR_NPARAM, 0.f);
    uint64_t st = seed;
    auto uni = [&]() {
        st += 0x9E3779B97F4A7C15ull;
        uint64_t z = st;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        z ^= z >> 31;
        return (double)(z >> 11) * (1.0 / 9007199254740992.0);
    };
    const int offs[4] = {SUR_W1, SUR_W2, SUR_W3, SUR_W4};
    const int fin[4] = {SUR_NIN, SUR_NH, SUR_NH, SUR_NH}, fout[4] = {SUR_NH, SUR_NH, SUR_NH, SUR_NOUT};
    for (int l = 0; l < 4; ++l) {
        const double a = std::sqrt(6.0 / (fin[l] + fout[l]));
        for (int i = 0; i < fin[l] * fout[l]; ++i) w[offs[l] + i] = (float)(a * (2.0 * uni() - 1.0));
    }
}

PlyC<double> sur_ply(const pdn_material &m)
{
    pdn_material e = m;
    e.law = PDN_LAW_CDM;
    return make_ply<double>(e, 0.0);
}

bool sur_material_ok(const pdn_material *m)
{
    return m && m->E1 > 0 && m->E2 > 0 && m->G12 > 0 && m->G23 > 0 && m->XT > 0 && m->XC > 0 && m->YT > 0 &&
           m->YC > 0 && m->SL > 0 && m->GXT > 0 && m->GXC > 0 && m->GYT > 0 && m->GYC > 0 && m->GSL > 0;
}

int sur_loss_host(const void *pk, const float *data, int64_t i0, int64_t n, double *part, hipStream_t s, double *out)
{
    if (n <= 0) { *out = 0.0; return PDN_OK; }
    GHIPCHK(pdn::launch_sur_loss(pk, data, i0, n, part, s));
    std::vector<double> h(pdn::sur_loss_blocks(n));
    GHIPCHK(hipMemcpyAsync(h.data(), part, h.size() * sizeof(double), hipMemcpyDeviceToHost, s));
    GHIPCHK(hipStreamSynchronize(s));
    double t = 0;
    for (double v : h) t += v;
    *out = t / ((double)n * SUR_NOUT);
    return PDN_OK;
}

}  // namespace

extern "C" {

const char *pdn_global_last_error(void) { return g_err.c_str(); }

int pdn_surrogate_data(int32_t device, void *stream, const pdn_material *m, double crack_band, uint64_t seed,
                       int64_t p0, int64_t n_paths, int32_t increments, float *records)
{
    if (!sur_material_ok(m) || !(crack_band > 0) || p0 < 0 || n_paths < 1 || increments < 1 || increments > 64 ||
        !records)
        return gerr(PDN_EINVAL, "surrogate data: invalid argument");
    GHIPCHK(hipSetDevice(device));
    hipStream_t s = (hipStream_t)stream;
    DevMem mem;
    float *out;
    const size_t bytes = (size_t)n_paths * increments * 20 * sizeof(float);
    GHIPCHK(mem.get(&out, bytes));
    const double vol = crack_band * crack_band * crack_band;
    GHIPCHK(pdn::launch_sur_data(sur_ply(*m), vol, seed, p0, n_paths, increments, out, s));
    GHIPCHK(hipMemcpyAsync(records, out, bytes, hipMemcpyDeviceToHost, s));
    GHIPCHK(hipStreamSynchronize(s));
    return PDN_OK;
}

int pdn_surrogate_eval(int32_t device, void *stream, const float *weights, const float *x, int64_t n, float *y)
{
    if (!weights || !x || !y || n < 0) return gerr(PDN_EINVAL, "surrogate eval: invalid argument");
    if (n == 0) return PDN_OK;
    GHIPCHK(hipSetDevice(device));
    hipStream_t s = (hipStream_t)stream;
    DevMem mem;
    float *w, *xd, *yd;
    void *pk;
    GHIPCHK(mem.get(&w, SUR_NPARAM * sizeof(float)));
    GHIPCHK(mem.get(&pk, SUR_PACK_BYTES));
    GHIPCHK(mem.get(&xd, n * SUR_NIN * sizeof(float)));
    GHIPCHK(mem.get(&yd, n * SUR_NOUT * sizeof(float)));
    GHIPCHK(hipMemcpyAsync(w, weights, SUR_NPARAM * sizeof(float), hipMemcpyHostToDevice, s));
    GHIPCHK(hipMemcpyAsync(xd, x, n * SUR_NIN * sizeof(float), hipMemcpyHostToDevice, s));
    GHIPCHK(pdn::launch_sur_pack(w, pk, s));
    GHIPCHK(pdn::launch_sur_eval(pk, xd, n, yd, s));
    GHIPCHK(hipMemcpyAsync(y, yd, n * SUR_NOUT * sizeof(float), hipMemcpyDeviceToHost, s));
    GHIPCHK(hipStreamSynchronize(s));
    return PDN_OK;
}

int pdn_surrogate_grad(int32_t device, void *stream, const float *weights, const float *x, const float *t,
                       int64_t n, float *grad, double *loss)
{
    if (!weights || !x || !t || !grad || n < 1) return gerr(PDN_EINVAL, "surrogate grad: invalid argument");
    GHIPCHK(hipSetDevice(device));
    hipStream_t s = (hipStream_t)stream;
    std::vector<float> rec((size_t)n * 20);
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 10; ++k) {
            rec[i * 20 + k] = x[i * 10 + k];
            rec[i * 20 + 10 + k] = t[i * 10 + k];
        }
    const int nwg = pdn::sur_grad_blocks(n, 1);
    DevMem mem;
    float *w, *data, *part;
    void *pk;
    GHIPCHK(mem.get(&w, SUR_NPARAM * sizeof(float)));
    GHIPCHK(mem.get(&pk, SUR_PACK_BYTES));
    GHIPCHK(mem.get(&data, rec.size() * sizeof(float)));
    GHIPCHK(mem.get(&part, (size_t)nwg * (SUR_NPARAM + 1) * sizeof(float)));
    GHIPCHK(hipMemcpyAsync(w, weights, SUR_NPARAM * sizeof(float), hipMemcpyHostToDevice, s));
    GHIPCHK(hipMemcpyAsync(data, rec.data(), rec.size() * sizeof(float), hipMemcpyHostToDevice, s));
    GHIPCHK(pdn::launch_sur_pack(w, pk, s));
    GHIPCHK(pdn::launch_sur_grad(pk, data, n, 0, n, 1, 0, 0, (float)(1.0 / ((double)n * SUR_NOUT)), part, s));
    std::vector<float> h((size_t)nwg * (SUR_NPARAM + 1));
    GHIPCHK(hipMemcpyAsync(h.data(), part, h.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    GHIPCHK(hipStreamSynchronize(s));
    double l = 0;
    for (int p = 0; p <= SUR_NPARAM; ++p) {
        double g = 0;
        for (int b = 0; b < nwg; ++b) g += h[(size_t)b * (SUR_NPARAM + 1) + p];
        if (p < SUR_NPARAM) grad[p] = (float)g;
        else l = g;
    }
    if (loss) *loss = l / ((double)n * SUR_NOUT);
    return PDN_OK;
}

int pdn_mesh_multiply(int32_t device, void *stream, const double *coords, int64_t n_nodes, const int32_t *hexes,
                      int64_t n_bulk, const int32_t *cohs, int64_t n_interface, const int32_t *hex_tag,
                      const int32_t *coh_tag, int32_t ndivi, double *coords_out, int32_t *hexes_out,
                      int32_t *cohs_out, int32_t *hex_tag_out, int32_t *coh_tag_out, int64_t cap_nodes,
                      int64_t cap_bulk, int64_t cap_interface, pdn_mmu_counts *counts)
{
    if (!counts || n_nodes < 0 || n_bulk < 0 || n_interface < 0 || ndivi < 0 || ndivi > 6 ||
        (n_nodes > 0 && !coords) || (n_bulk > 0 && !hexes) || (n_interface > 0 && !cohs) || n_nodes > INT32_MAX)
        return gerr(PDN_EINVAL, "mesh multiplication: invalid argument");
    for (int64_t i = 0; i < 8 * n_bulk; ++i)
        if (hexes[i] < 0 || hexes[i] >= n_nodes) return gerr(PDN_EINVAL, "mesh multiplication: bulk node out of range");
    for (int64_t i = 0; i < 8 * n_interface; ++i)
        if (cohs[i] < 0 || cohs[i] >= n_nodes)
            return gerr(PDN_EINVAL, "mesh multiplication: interface node out of range");
    std::memset(counts, 0, sizeof *counts);
    GHIPCHK(hipSetDevice(device));
    hipStream_t s = (hipStream_t)stream;
    // current level on the device (freed as levels are replaced)
    struct Level {
        double *X = nullptr;
        int32_t *H = nullptr, *C = nullptr, *ht = nullptr, *ct = nullptr;
        void release()
        {
            for (void *p : {(void *)X, (void *)H, (void *)C, (void *)ht, (void *)ct})
                if (p) (void)hipFree(p);
            X = nullptr; H = C = ht = ct = nullptr;
        }
        ~Level() { release(); }
    } cur, nxt;
    auto up = [&](void **d, const void *h, size_t bytes) -> hipError_t {
        hipError_t e = hipMalloc(d, bytes ? bytes : 1);
        if (e == hipSuccess && bytes) e = hipMemcpyAsync(*d, h, bytes, hipMemcpyHostToDevice, s);
        return e;
    };
    GHIPCHK(up((void **)&cur.X, coords, 3 * n_nodes * sizeof(double)));
    GHIPCHK(up((void **)&cur.H, hexes, 8 * n_bulk * sizeof(int32_t)));
    GHIPCHK(up((void **)&cur.C, cohs, 8 * n_interface * sizeof(int32_t)));
    if (hex_tag) GHIPCHK(up((void **)&cur.ht, hex_tag, n_bulk * sizeof(int32_t)));
    if (coh_tag) GHIPCHK(up((void **)&cur.ct, coh_tag, n_interface * sizeof(int32_t)));
    int64_t nn = n_nodes, nh = n_bulk, nc = n_interface;
    for (int lv = 0; lv < ndivi; ++lv) {
        pdn::MmuLevel info{};
        const hipError_t e = pdn::mmu_divide(cur.X, nn, cur.H, nh, cur.C, nc, cur.ht, cur.ct, &nxt.X, &nxt.H, &nxt.C,
                                             &nxt.ht, &nxt.ct, &info, s);
        if (e == hipErrorInvalidValue) return gerr(PDN_EINVAL, "mesh multiplication: the divided mesh exceeds int32 numbering");
        GHIPCHK(e);
        cur.release();
        std::swap(cur.X, nxt.X); std::swap(cur.H, nxt.H); std::swap(cur.C, nxt.C);
        std::swap(cur.ht, nxt.ht); std::swap(cur.ct, nxt.ct);
        nn = info.nn; nh = info.nh; nc = info.nc;
        counts->n_edges = info.n_edges;
        counts->n_faces = info.n_faces;
        counts->n_boundary0 = info.nb0;
        counts->n_boundary_interface0 = info.nb_int0;
    }
    counts->n_nodes = nn;
    counts->n_bulk = nh;
    counts->n_interface = nc;
    if (!coords_out || !hexes_out || !cohs_out || cap_nodes < nn || cap_bulk < nh || cap_interface < nc ||
        (hex_tag && !hex_tag_out) || (coh_tag && !coh_tag_out))
        return gerr(PDN_ERANGE, "mesh multiplication: outputs need %lld nodes, %lld bulk and %lld interface elements",
                    (long long)nn, (long long)nh, (long long)nc);
    if (nn) GHIPCHK(hipMemcpyAsync(coords_out, cur.X, 3 * nn * sizeof(double), hipMemcpyDeviceToHost, s));
    if (nh) GHIPCHK(hipMemcpyAsync(hexes_out, cur.H, 8 * nh * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (nc) GHIPCHK(hipMemcpyAsync(cohs_out, cur.C, 8 * nc * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (hex_tag && nh) GHIPCHK(hipMemcpyAsync(hex_tag_out, cur.ht, nh * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    if (coh_tag && nc) GHIPCHK(hipMemcpyAsync(coh_tag_out, cur.ct, nc * sizeof(int32_t), hipMemcpyDeviceToHost, s));
    GHIPCHK(hipStreamSynchronize(s));
    return PDN_OK;
}

int pdn_surrogate_grad_fp32(int32_t device, void *stream, const float *weights, const float *x, const float *t,
                            int64_t n, float *grad, double *loss)
{
    if (!weights || !x || !t || !grad || n < 1) return gerr(PDN_EINVAL, "surrogate grad (fp32): invalid argument");
    GHIPCHK(hipSetDevice(device));
    hipStream_t s = (hipStream_t)stream;
    std::vector<float> rec((size_t)n * 20);
    for (int64_t i = 0; i < n; ++i)
        for (int k = 0; k < 10; ++k) {
            rec[i * 20 + k] = x[i * 10 + k];
            rec[i * 20 + 10 + k] = t[i * 10 + k];
        }
    const int nwg = pdn::sur_grad32_blocks(n);
    DevMem mem;
    float *w, *data, *part;
    GHIPCHK(mem.get(&w, SUR_NPARAM * sizeof(float)));
    GHIPCHK(mem.get(&data, rec.size() * sizeof(float)));
    GHIPCHK(mem.get(&part, (size_t)nwg * (SUR_NPARAM + 1) * sizeof(float)));
    GHIPCHK(hipMemcpyAsync(w, weights, SUR_NPARAM * sizeof(float), hipMemcpyHostToDevice, s));
    GHIPCHK(hipMemcpyAsync(data, rec.data(), rec.size() * sizeof(float), hipMemcpyHostToDevice, s));
    GHIPCHK(pdn::launch_sur_grad32(w, data, n, (float)(1.0 / ((double)n * SUR_NOUT)), part, s));
    std::vector<float> h((size_t)nwg * (SUR_NPARAM + 1));
    GHIPCHK(hipMemcpyAsync(h.data(), part, h.size() * sizeof(float), hipMemcpyDeviceToHost, s));
    GHIPCHK(hipStreamSynchronize(s));
    for (int p = 0; p <= SUR_NPARAM; ++p) {
        double g = 0;
        for (int b = 0; b < nwg; ++b) g += h[(size_t)b * (SUR_NPARAM + 1) + p];
        if (p < SUR_NPARAM) grad[p] = (float)g;
        else if (loss) *loss = g;
    }
    return PDN_OK;
}

int pdn_surrogate_grad_noalloc(int32_t device, void *stream, const float *weights, const float *x, const float *t,
                               int64_t n, float *grad, double *loss)
{
    if (!weights || !x || !t || !grad || n < 1)
        return gerr(PDN_EINVAL, "surrogate grad (no allocation): invalid argument");
    if (n > PDN_SUR_GRAD_NOALLOC_MAX)
        return gerr(PDN_EINVAL, "surrogate grad (no allocation): %lld points exceed the fixed scratch's %d",
                    (long long)n, PDN_SUR_GRAD_NOALLOC_MAX);
    const int nwg = pdn::sur_grad_blocks(n, 1);
    if (nwg > PDN_SUR_NOALLOC_PARTS) return gerr(PDN_EINVAL, "surrogate grad (no allocation): scratch layout");
    GHIPCHK(hipSetDevice(device));
    void *scr = nullptr;
    GHIPCHK(pdn::sur_noalloc_scratch(device, &scr));
    hipStream_t s = (hipStream_t)stream;
    char *base = (char *)scr;
    void *pk = base;
    float *rec = (float *)(base + PDN_SUR_NOALLOC_OFF_REC);
    float *part = (float *)(base + PDN_SUR_NOALLOC_OFF_PART);
    GHIPCHK(pdn::launch_sur_pack(weights, pk, s));
    GHIPCHK(pdn::launch_sur_interleave(x, t, n, rec, s));
    GHIPCHK(pdn::launch_sur_grad(pk, rec, n, 0, n, 1, 0, 0, (float)(1.0 / ((double)n * SUR_NOUT)), part, s));
    GHIPCHK(pdn::launch_sur_grad_reduce(part, nwg, (double)n * SUR_NOUT, grad, loss, s));
    return PDN_OK;
}

int pdn_surrogate_train(const pdn_sur_train *o, const pdn_material *m, double crack_band, float *weights,
                        pdn_sur_report *rep)
{
    if (!o || !sur_material_ok(m) || !(crack_band > 0) || !weights || o->n_paths < 2 || o->increments < 1 ||
        o->increments > 64 || o->steps < 0 || o->batch < 128 || o->batch % 128 || !(o->lr > 0) ||
        !(o->val_fraction > 0 && o->val_fraction < 1))
        return gerr(PDN_EINVAL, "surrogate training: invalid argument");
    GHIPCHK(hipSetDevice(o->device));
    hipStream_t s = (hipStream_t)o->stream;
    const int64_t n_val_paths = std::max<int64_t>(1, (int64_t)(o->n_paths * o->val_fraction));
    const int64_t n_train_paths = o->n_paths - n_val_paths;
    if (n_train_paths < 1) return gerr(PDN_EINVAL, "surrogate training: no training paths");
    const int64_t n_all = o->n_paths * o->increments, n_train = n_train_paths * o->increments;
    const int nblk = std::max(1, o->batch / (128 * 256));
    const int nwg = pdn::sur_grad_blocks(o->batch, nblk);
    DevMem mem;
    float *data, *w, *mm, *vv, *part, *lossd;
    double *lpart;
    void *pk;
    GHIPCHK(mem.get(&data, (size_t)n_all * 20 * sizeof(float)));
    GHIPCHK(mem.get(&w, SUR_NPARAM * sizeof(float)));
    GHIPCHK(mem.get(&mm, SUR_NPARAM * sizeof(float)));
    GHIPCHK(mem.get(&vv, SUR_NPARAM * sizeof(float)));
    GHIPCHK(mem.get(&pk, SUR_PACK_BYTES));
    GHIPCHK(mem.get(&part, (size_t)nwg * (SUR_NPARAM + 1) * sizeof(float)));
    GHIPCHK(mem.get(&lossd, std::max<int64_t>(1, o->steps) * sizeof(float)));
    GHIPCHK(mem.get(&lpart, (size_t)pdn::sur_loss_blocks(std::max(n_all - n_train, n_train)) * sizeof(double)));
    hipEvent_t e0, e1, e2;
    GHIPCHK(hipEventCreate(&e0));
    GHIPCHK(hipEventCreate(&e1));
    GHIPCHK(hipEventCreate(&e2));
    GHIPCHK(hipEventRecord(e0, s));
    GHIPCHK(pdn::launch_sur_data(sur_ply(*m), crack_band * crack_band * crack_band, o->seed, 0, o->n_paths,
                                 o->increments, data, s));
    GHIPCHK(hipEventRecord(e1, s));
    std::vector<float> w0;
    sur_init(o->init_seed, w0);
    GHIPCHK(hipMemcpyAsync(w, w0.data(), SUR_NPARAM * sizeof(float), hipMemcpyHostToDevice, s));
    GHIPCHK(hipMemsetAsync(mm, 0, SUR_NPARAM * sizeof(float), s));
    GHIPCHK(hipMemsetAsync(vv, 0, SUR_NPARAM * sizeof(float), s));
    GHIPCHK(pdn::launch_sur_pack(w, pk, s));
    double val0 = 0;
    int rc = sur_loss_host(pk, data, n_train, n_all - n_train, lpart, s, &val0);
    if (rc) return rc;
    const float b1 = 0.9f, b2 = 0.999f;
    double p1 = 1, p2 = 1;
    const double lr_end = o->lr_final > 0 ? o->lr_final : 0.01 * o->lr;
    GHIPCHK(hipEventRecord(e1, s));
    for (int64_t t = 0; t < o->steps; ++t) {
        p1 *= b1;
        p2 *= b2;
        const double lr = lr_end + 0.5 * (o->lr - lr_end) * (1.0 + std::cos(M_PI * (double)t / (double)o->steps));
        GHIPCHK(pdn::launch_sur_grad(pk, data, n_train, t * (int64_t)o->batch, o->batch, nblk, 1,
                                     o->seed ^ 0x5A17C0DEull, (float)(1.0 / ((double)o->batch * SUR_NOUT)), part, s));
        GHIPCHK(pdn::launch_sur_adam(part, nwg, w, mm, vv, (float)lr, b1, b2, 1e-8f, (float)(1 - p1), (float)(1 - p2),
                                     lossd + t, s));
        GHIPCHK(pdn::launch_sur_pack(w, pk, s));
    }
    GHIPCHK(hipEventRecord(e2, s));
    double val = 0;
    if ((rc = sur_loss_host(pk, data, n_train, n_all - n_train, lpart, s, &val))) return rc;
    double tr = 0;
    if ((rc = sur_loss_host(pk, data, 0, std::min<int64_t>(n_train, 1 << 22), lpart, s, &tr))) return rc;
    GHIPCHK(hipMemcpyAsync(weights, w, SUR_NPARAM * sizeof(float), hipMemcpyDeviceToHost, s));
    GHIPCHK(hipStreamSynchronize(s));
    float tdata = 0, ttrain = 0;
    GHIPCHK(hipEventElapsedTime(&tdata, e0, e1));
    GHIPCHK(hipEventElapsedTime(&ttrain, e1, e2));
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    (void)hipEventDestroy(e2);
    if (rep) {
        rep->loss_val_initial = val0;
        rep->loss_val = val;
        rep->loss_train = tr;
        rep->data_seconds = 1e-3 * tdata;
        rep->train_seconds = 1e-3 * ttrain;
        rep->samples_train = n_train;
        rep->samples_val = n_all - n_train;
    }
    return PDN_OK;
}

int pdn_surrogate_kernel(pdn_ctx *c, int32_t mode)
{
    if (!c) return PDN_EINVAL;
    if (mode < 0 || mode > 2) return set_err(c, PDN_EINVAL, "surrogate kernel mode must be 0, 1 or 2");
    c->sur_mode = mode;
    c->sur_build = mode != 0 ? mode : 2;
    return PDN_OK;
}

int pdn_surrogate_set(pdn_ctx *c, int32_t ply, const float *weights, int64_t n, double dmg_thresh,
                      double res_thresh)
{
    if (!c) return PDN_EINVAL;
    if (c->broken) return set_err(c, PDN_EUNSTABLE, "context is unstable");
    if (!weights || n != SUR_NPARAM) return set_err(c, PDN_EINVAL, "surrogate needs %d parameters", SUR_NPARAM);
    if (ply < -1 || ply >= c->P) return set_err(c, PDN_EINVAL, "ply index %d out of range", ply);
    if (!(dmg_thresh >= 0) || !(res_thresh >= 0)) return set_err(c, PDN_EINVAL, "thresholds must be >= 0");
    if (c->ngp != 1) return set_err(c, PDN_EINVAL, "surrogate plies need one-point integration");
    for (int p = 0; p < c->P; ++p)
        if ((ply < 0 || p == ply) && (!c->mat_set[p] || c->mat[p].law == PDN_LAW_ELASTIC))
            return set_err(c, PDN_ESTATE, "ply %d has no damage law to replace", p);
    for (int p = 0; p < c->P; ++p)
        if (c->mat_set[p] && c->mat[p].Sp > 0)
            return set_err(c, PDN_EINVAL, "surrogate plies and shear plasticity are not built together (ply %d)", p);
    (void)hipSetDevice(c->device);
    // grow the network table by one
    uint4 *nd = nullptr;
    int rc = dalloc(c, (void **)&nd, (size_t)(c->n_nets + 1) * SUR_PACK_BYTES);
    if (rc) return rc;
    if (c->sur_d) {
        HIPCHK(c, hipMemcpyAsync(nd, c->sur_d, (size_t)c->n_nets * SUR_PACK_BYTES, hipMemcpyDeviceToDevice, c->stream));
    }
    float *w = nullptr;
    if ((rc = dalloc(c, (void **)&w, SUR_NPARAM * sizeof(float)))) return rc;
    HIPCHK(c, hipMemcpyAsync(w, weights, SUR_NPARAM * sizeof(float), hipMemcpyHostToDevice, c->stream));
    hipError_t e = pdn::launch_sur_pack(w, reinterpret_cast<char *>(nd) + (size_t)c->n_nets * SUR_PACK_BYTES,
                                        c->stream);
    HIPCHK(c, hipStreamSynchronize(c->stream));
    (void)hipFree(w);
    if (e != hipSuccess) return set_err(c, PDN_EDEVICE, "surrogate packing: %s", hipGetErrorString(e));
    if (c->sur_d) (void)hipFree(c->sur_d);
    c->sur_d = nd;
    for (int p = 0; p < c->P; ++p)
        if (ply < 0 || p == ply) {
            c->ply_net[p] = c->n_nets;
            c->mat[p].law = PDN_LAW_CDM_SURROGATE;
        }
    c->n_nets += 1;
    c->sur_fresh = true;
    c->sur_dmg = dmg_thresh;
    c->sur_res = res_thresh;
    c->ready = false;
    if (c->gl.step > 0) {
        c->needs_init = true;
        c->loaded_state = true;
    }
    return PDN_OK;
}

}  // extern "C"

