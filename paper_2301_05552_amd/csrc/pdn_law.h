// pdn_law.h -- constitutive laws of the plate (device code, internal).
//
//  cdm_*   : intralaminar damage of a ply (Section 2.3.1, Algorithm 4),
//            elastic-damage reading with crack-band regularisation;
//  czm_*   : cohesive interface law (Section 2.3.2, Algorithm 5).
#pragma once
#include "pdn_internal.h"

namespace pdn {

template <typename R>
__device__ __forceinline__ R rmax(R a, R b) { return a > b ? a : b; }
template <typename R>
__device__ __forceinline__ R rmin(R a, R b) { return a < b ? a : b; }

// ---------------------------------------------------------------------------
// intralaminar law (Section 2.3.1, Algorithm 4; elastic-damage reading)
// ---------------------------------------------------------------------------

// crack-band strength: lowered when the softening would snap back at size lc
template <typename R>
__device__ __forceinline__ R cap_strength(R X, R E, R G, R lc)
{
    R lim = R(1.8) * E * G / lc;
    return (X * X > lim) ? sqrt(lim) : X;
}

// exponential softening of a matrix / shear mode: d = 1 - exp(A (1 - r)) / r
template <typename R>
__device__ R damage_exp(R r, R X, R E, R G, R lc)
{
    if (r <= R(1)) return R(0);
    R A = R(2) * lc * X * X / (R(2) * E * G - lc * X * X);
    R d = R(1) - exp(A * (R(1) - r)) / r;
    return rmin(rmax(d, R(0)), R(1) - R(1e-6));
}

// bilinear softening of a fibre mode, secant at the strain r * X / E
template <typename R>
__device__ R damage_bilinear(R r, R X, R E, R G, R fX, R fG, R lc)
{
    if (r <= R(1)) return R(0);
    R e0 = X / E, g = G / lc;
    R eB = R(2) * fG * g / X + fX * e0;
    R eC = R(2) * (R(1) - fG) * g / (fX * X);
    R e = r * e0, sg;
    if (e <= e0) sg = E * e;
    else if (e <= eB) sg = X + (fX * X - X) * (e - e0) / (eB - e0);
    else if (e <= eC) sg = fX * X * (eC - e) / (eC - eB);
    else sg = R(0);
    R d = R(1) - sg / (E * e);
    return rmin(rmax(d, R(0)), R(1) - R(1e-6));
}

// Damage variables of the thresholds and the nominal stress: the inverse of
// the damaged compliance applied to the strain (normal block by cofactors).
// s0, s1 are the effective stresses 11, 22 (their signs pick tension or
// compression); YT, YC, SL the crack-band strengths at length lc.
template <typename R>
__device__ __forceinline__ void cdm_nominal(const PlyC<R> &P, R lc, R YT, R YC, R SL, R r0, R r1, R r2, R r3,
                                            R s0, R s1, const R e[6], R sg[6])
{
    R d1p = damage_bilinear(r0, P.XT, P.E1, P.GXT, P.fXT, P.fGT, lc);
    R d1m = damage_bilinear(r1, P.XC, P.E1, P.GXC, P.fXC, P.fGC, lc);
    R d2p = damage_exp(r2, YT, P.E2, P.GYT, lc);
    R d2m = damage_exp(r3, YC, P.E2, P.GYC, lc);
    R d6 = damage_exp(r2, SL, P.G12v, P.GSL, lc);
    R d1 = s0 >= R(0) ? d1p : d1m;
    R d2 = s1 >= R(0) ? d2p : d2m;
    R h00 = P.iE1 / (R(1) - d1), h11 = P.iE2 / (R(1) - d2), h22 = P.iE3;
    R h01 = P.mn12, h02 = P.mn13, h12 = P.mn23;
    R c00 = h11 * h22 - h12 * h12, c01 = h02 * h12 - h01 * h22, c02 = h01 * h12 - h02 * h11;
    R c11 = h00 * h22 - h02 * h02, c12 = h01 * h02 - h00 * h12, c22 = h00 * h11 - h01 * h01;
    R inv = R(1) / (h00 * c00 + h01 * c01 + h02 * c02);
    sg[0] = (c00 * e[0] + c01 * e[1] + c02 * e[2]) * inv;
    sg[1] = (c01 * e[0] + c11 * e[1] + c12 * e[2]) * inv;
    sg[2] = (c02 * e[0] + c12 * e[1] + c22 * e[2]) * inv;
    // crack closure acts on the normal terms only: the transverse shear keeps
    // the tensile matrix damage, so no closed strain cycle returns energy
    // (thermodynamic consistency, Section 2.3.1)
    sg[3] = (R(1) - d2p) * P.G23 * e[3];
    sg[4] = (R(1) - d6) * P.G13 * e[4];
    sg[5] = (R(1) - d6) * P.G12 * e[5];
}

// largest of the five damage variables of thresholds r
template <typename R>
__device__ __forceinline__ R cdm_max_damage(const PlyC<R> &P, R lc, R YT, R YC, R SL, const R r[4])
{
    R d = rmax(damage_bilinear(r[0], P.XT, P.E1, P.GXT, P.fXT, P.fGT, lc),
               damage_bilinear(r[1], P.XC, P.E1, P.GXC, P.fXC, P.fGC, lc));
    d = rmax(d, damage_exp(r[2], YT, P.E2, P.GYT, lc));
    d = rmax(d, damage_exp(r[3], YC, P.E2, P.GYC, lc));
    return rmax(d, damage_exp(r[2], SL, P.G12v, P.GSL, lc));
}

// Undamaged stress s = C0 e, and the screen: true when the point is provably
// elastic for the law, i.e. its thresholds are all at 1 and upper bounds of
// its loading functions (without roots) show that none can exceed them.  The
// law then returns s and leaves the thresholds unchanged, exactly as its full
// evaluation would.  The bounds use the ply's screen constants, which hold for
// every element of the ply (strengths capped at its largest crack band, with
// a rounding margin).
template <typename R>
__device__ __forceinline__ bool cdm_screen(const PlyC<R> &P, R vol, const R e[6], const R r[4], R s[6])
{
    s[0] = P.C11 * e[0] + P.C12 * e[1] + P.C13 * e[2];
    s[1] = P.C12 * e[0] + P.C22 * e[1] + P.C23 * e[2];
    s[2] = P.C13 * e[0] + P.C23 * e[1] + P.C33 * e[2];
    s[3] = P.G23 * e[3]; s[4] = P.G13 * e[4]; s[5] = P.G12 * e[5];
    if (vol > P.scr_vmax) return false;                  // beyond the elements the constants were made for
    const R s1 = s[1];
    const R t2 = s[5] * s[5] + s[4] * s[4];              // tau_L^2
    bool grow = rmax(e[0], R(0)) * P.scr_kXT > r[0] || rmax(-e[0], R(0)) * P.scr_kXC > r[1];
    if (s1 >= R(0)) {
        const R a = s1 * P.scr_iYT;
        grow |= a * a + t2 * P.scr_iSL * P.scr_iSL > r[2] * r[2];
    } else {
        const R el = P.scr_etaL * s1;                    // eta_L sigma22
        const R qL = el > R(0) ? R(2) * (t2 + el * el) : t2;
        grow |= qL * P.scr_iSL * P.scr_iSL > r[2] * r[2];
        const R bT = -s1 * P.kT * P.scr_iST;
        const R elc = el * P.ca0;
        const R qL2 = R(2) * P.ca0 * P.ca0 * (t2 + elc * elc);
        grow |= bT * bT + qL2 * P.scr_iSL * P.scr_iSL > r[3] * r[3];
    }
    return !grow && r[0] <= R(1) && r[1] <= R(1) && r[2] <= R(1) && r[3] <= R(1);
}

// Algorithm 4, first two lines: the plastic strains of the longitudinal shear
// (linear isotropic hardening in effective stress: yield when tau_L >
// Sp + Hp abar, tau_L = |(tau12, tau13)|, G13 = G12; radial return), then the
// elastic strains e - e_p in place.  ep = {gamma12_p, gamma13_p, abar, -}.
// The flow test has a rounding allowance, and the elastic strains are formed
// from the updated plastic strains: evaluating the point again from its
// updated state then gives the same answer bit for bit (a rim element is
// evaluated by two workgroups, one of which may read the updated state).
// Returns true when the plastic state changed.
template <typename R>
__device__ __forceinline__ bool plastic_return(const PlyC<R> &P, R e[6], R ep[4])
{
    const R G = P.G12;
    const R t12 = G * (e[5] - ep[0]), t13 = G * (e[4] - ep[1]);
    const R tL = sqrt(t12 * t12 + t13 * t13);
    const R Y = P.Sp + P.Hp * ep[2];
    const R F = tL - Y;
    const bool flow = F > (sizeof(R) == 4 ? R(1e-5) : R(1e-12)) * Y;
    if (flow) {
        const R dl = F / (G + P.Hp);
        ep[0] += dl * t12 / tL;
        ep[1] += dl * t13 / tL;
        ep[2] += dl;
    }
    e[5] = e[5] - ep[0];
    e[4] = e[4] - ep[1];
    return flow;
}

// eps: material-frame Green strain (Voigt 11,22,33,23,13,12, engineering shear)
// r: thresholds r1+, r1-, r2+, r2- (in/out).  Returns nominal PK2 stress in sg,
// and true when the screen passed the point (it is provably elastic).
template <typename R>
__device__ bool cdm_update(const PlyC<R> &P, R vol, const R e[6], R r[4], R sg[6], bool &changed)
{
    changed = false;
    R sc[6];
    const bool elastic = cdm_screen(P, vol, e, r, sc);
    const R s0 = sc[0], s1 = sc[1], s2 = sc[2], s3 = sc[3], s4 = sc[4], s5 = sc[5];
    if (P.law == 0 || elastic) {
        sg[0] = s0; sg[1] = s1; sg[2] = s2; sg[3] = s3; sg[4] = s4; sg[5] = s5;
        return elastic;
    }
    const R lc = cbrt(vol);                              // crack-band length
    const R YT = cap_strength(P.YT, P.E2, P.GYT, lc);
    const R YC = cap_strength(P.YC, P.E2, P.GYC, lc);
    const R SL = cap_strength(P.SL, P.G12v, P.GSL, lc);
    // loading functions: maximum strain (fibre), LaRC-type (matrix)
    R p1p = rmax(e[0], R(0)) * P.E1 / P.XT;
    R p1m = rmax(-e[0], R(0)) * P.E1 / P.XC;
    R tL = sqrt(s5 * s5 + s4 * s4);
    R etaL = P.kEtaL * SL / YC;
    R p2p, p2m = R(0);
    if (s1 >= R(0)) {
        R a = s1 / YT, b = tL / SL;
        p2p = sqrt(a * a + b * b);
    } else {
        p2p = rmax(tL + etaL * s1, R(0)) / SL;
        R ST = P.kST * YC;
        R a = -s1 * P.sa0;                           // > 0
        R hyp = sqrt(a * a + tL * tL);
        R ct = a / hyp, st = tL / hyp;               // fracture-plane angle theta
        R tte = rmax(-s1 * P.ca0 * (P.sa0 - P.etaT * P.ca0 * ct), R(0));
        R tle = rmax(P.ca0 * (tL + etaL * s1 * P.ca0 * st), R(0));
        R u = tte / ST, w = tle / SL;
        p2m = sqrt(u * u + w * w);
    }
    R r0 = rmax(r[0], p1p), r1 = rmax(r[1], p1m), r2 = rmax(r[2], p2p), r3 = rmax(r[3], p2m);
    r0 = rmax(r0, r1);
    r2 = rmax(r2, r3);
    changed = (r0 != r[0]) | (r1 != r[1]) | (r2 != r[2]) | (r3 != r[3]);
    r[0] = r0; r[1] = r1; r[2] = r2; r[3] = r3;
    if (r0 <= R(1) && r1 <= R(1) && r2 <= R(1) && r3 <= R(1)) {   // undamaged
        sg[0] = s0; sg[1] = s1; sg[2] = s2; sg[3] = s3; sg[4] = s4; sg[5] = s5;
        return false;
    }
    cdm_nominal(P, lc, YT, YC, SL, r0, r1, r2, r3, s0, s1, e, sg);
    return false;
}

// ---------------------------------------------------------------------------
// cohesive law (Section 2.3.2, Algorithm 5; Turon mixed-mode variables)
// ---------------------------------------------------------------------------
template <typename R>
__device__ R czm_update(const PlyC<R> &P, R d1, R d2, R d3, R &rd, R tau[3], bool &changed)
{
    R sh2 = d1 * d1 + d2 * d2;
    R d3p = rmax(d3, R(0));
    R den = P.Ksh * sh2 + P.KI * d3p * d3p;
    // screen: an undamaged pair whose opening is below onset at every mode
    // mixity keeps D = 0, which is what the evaluation below gives for it
    // (with D = 0 the tractions are K d exactly)
    if (rd == R(0) && den <= P.den_onset) {
        changed = false;
        tau[0] = P.Ksh * d1;
        tau[1] = P.Ksh * d2;
        tau[2] = P.KI * d3;
        return R(0);
    }
    R B = den > R(0) ? P.Ksh * sh2 / den : R(0);
    R KB = (R(1) - B) * P.KI + B * P.Ksh;
    R lam = sqrt(den / KB);
    R Gc = P.GIc + (P.GIIc - P.GIc) * pow(B, P.eta_bk);
    R lo = sqrt(R(2) * P.GIo * Gc / (P.GIc * KB));
    R lc = R(2) * Gc / (KB * lo);
    R H = rmin((lam - lo) / (lc - lo), R(1));
    R rn = rmax(rd, H);
    changed = rn != rd;
    rd = rn;
    R D = rn * lc / (rn * lc + (R(1) - rn) * lo);
    tau[0] = (R(1) - D) * P.Ksh * d1;
    tau[1] = (R(1) - D) * P.Ksh * d2;
    tau[2] = d3 >= R(0) ? (R(1) - D) * P.KI * d3 : P.KI * d3;
    return D;
}

}  // namespace pdn
