// pdn_elem.h -- the fused element / node kernel (device code, internal),
// instantiated without the surrogate in pdn_kernels.hip and with it in
// pdn_elem_sur.hip.
#pragma once
#include "pdn_internal.h"
#include "pdn_launch.h"
#include "pdn_law.h"
#include "pdn_mlp.h"

#include <type_traits>

namespace pdn {

// ---------------------------------------------------------------------------
// intralaminar update by the surrogate network with the exact law as fallback
//
// A point that the law's screen proves elastic takes the law's exact answer
// (C0 e, thresholds unchanged) without the network; a wave made of such
// points does not run the network at all.  Of the other points, one keeps
// the exact law when any damage variable of its incoming thresholds exceeds
// dmg_thr, or when the network's stress disagrees with the nominal stress of
// the network's own new thresholds by more than res_thr (relative to |C0 e|,
// at least 1e-3 Y_T).  A point of an element that two workgroups evaluate
// (shared) keeps the exact law too: the other workgroup may read its
// thresholds before or after their owner updates them, which the exact law's
// idempotent update tolerates and the network would not.  Every lane of the
// wave must call it together (the network runs on the matrix cores).  exact:
// 0 the network's result; 1 the exact law after the network was consulted
// and its answer failed the residual bar; 2 screened elastic; 3 the exact law
// without consulting the network (incoming damage past dmg_thr, or a shared
// element).
// ---------------------------------------------------------------------------
template <typename R>
__device__ void sur_update(const PlyC<R> &P, R vol, const R e[6], R r[4], R sg[6], bool &changed,
                           const uint4 *__restrict__ pk, float dmg_thr, float res_thr, int &exact, bool shared)
{
    R sel[6];
    const bool el = cdm_screen(P, vol, e, r, sel);
    if (__ballot(!el) == 0) {                                   // uniform across the wave
#pragma unroll
        for (int k = 0; k < 6; ++k) sg[k] = sel[k];
        changed = false;
        exact = 2;
        return;
    }
    const R lc = cbrt(vol);
    const R YT = cap_strength(P.YT, P.E2, P.GYT, lc);
    const R YC = cap_strength(P.YC, P.E2, P.GYC, lc);
    const R SL = cap_strength(P.SL, P.G12v, P.GSL, lc);
    const R X[6] = {P.XT, P.YT, P.YT, P.SL, P.SL, P.SL};
    const R kx[6] = {P.kE1XT, P.E2 * P.iYT, P.E2 * P.iYT, P.G23 * P.iSL, P.G12 * P.iSL, P.G12 * P.iSL};
    float x[SUR_NIN], y[SUR_NOUT];
#pragma unroll
    for (int k = 0; k < 6; ++k) x[k] = (float)(e[k] * kx[k]);
#pragma unroll
    for (int k = 0; k < 4; ++k) x[6 + k] = (float)(R(1) - R(1) / r[k]);
    bool fb = shared || ((r[0] > R(1) || r[1] > R(1) || r[2] > R(1) || r[3] > R(1)) &&
                         cdm_max_damage(P, lc, YT, YC, SL, r) > (R)dmg_thr);
    const bool gated = fb;                                      // the network is not consulted
    if (__ballot(!fb && !el) != 0) sur_forward_wave(pk, x, y);  // uniform across the wave
    if (el) {
#pragma unroll
        for (int k = 0; k < 6; ++k) sg[k] = sel[k];
        changed = false;
        exact = 2;
        return;
    }
    R rs[4], ss[6];
    if (!fb) {
#pragma unroll
        for (int k = 0; k < 6; ++k) ss[k] = (R)y[k] * X[k];
#pragma unroll
        for (int k = 0; k < 4; ++k) {
            const R so = rmin(rmax((R)x[6 + k], (R)y[6 + k]), R(1) - R(1e-6));
            rs[k] = rmax(r[k], R(1) / (R(1) - so));               // thresholds never decrease
        }
        rs[0] = rmax(rs[0], rs[1]);
        rs[2] = rmax(rs[2], rs[3]);
        // nominal stress of the predicted thresholds, and the effective stress
        const R s0 = P.C11 * e[0] + P.C12 * e[1] + P.C13 * e[2];
        const R s1 = P.C12 * e[0] + P.C22 * e[1] + P.C23 * e[2];
        const R s2 = P.C13 * e[0] + P.C23 * e[1] + P.C33 * e[2];
        const R s3 = P.G23 * e[3], s4 = P.G13 * e[4], s5 = P.G12 * e[5];
        R sc[6];
        if (rs[0] <= R(1) && rs[1] <= R(1) && rs[2] <= R(1) && rs[3] <= R(1)) {
            sc[0] = s0; sc[1] = s1; sc[2] = s2; sc[3] = s3; sc[4] = s4; sc[5] = s5;
        } else {
            cdm_nominal(P, lc, YT, YC, SL, rs[0], rs[1], rs[2], rs[3], s0, s1, e, sc);
        }
        R num = R(0);
#pragma unroll
        for (int k = 0; k < 6; ++k) num += (ss[k] - sc[k]) * (ss[k] - sc[k]);
        const R den = rmax(s0 * s0 + s1 * s1 + s2 * s2 + s3 * s3 + s4 * s4 + s5 * s5, R(1e-6) * P.YT * P.YT);
        fb = num > (R)res_thr * (R)res_thr * den;
    }
    exact = gated ? 3 : fb ? 1 : 0;
    if (fb) {
        cdm_update(P, vol, e, r, sg, changed);
        return;
    }
    changed = (rs[0] != r[0]) | (rs[1] != r[1]) | (rs[2] != r[2]) | (rs[3] != r[3]);
#pragma unroll
    for (int k = 0; k < 4; ++k) r[k] = rs[k];
#pragma unroll
    for (int k = 0; k < 6; ++k) sg[k] = ss[k];
}

// ---------------------------------------------------------------------------
// 1-point hex8 on a box element (Section 2, total Lagrangian, Eq. 3 form)
//
// For an axis-aligned box the mean gradient is b_a = (xi_a/4hx, eta_a/4hy,
// zeta_a/4hz) and the Flanagan-Belytschko vectors are gamma = h/8, so the
// 8 nodal values of each displacement component are projected on the
// orthogonal corner basis {xi, eta, zeta, eta.zeta, xi.zeta, xi.eta,
// xi.eta.zeta} (a Walsh-Hadamard transform, 24 adds) and the nodal forces are
// the inverse transform of the stress and hourglass coefficients.
// Node order: bottom face (-,-), (+,-), (+,+), (-,+), then the top face.
// ---------------------------------------------------------------------------
template <typename R>
struct Modes { R xi, eta, zeta, ez, xz, xe, xez; };

template <typename R>
__device__ __forceinline__ Modes<R> fwd8(const R u[8])
{
    R p0 = u[0] + u[4], p1 = u[1] + u[5], p2 = u[2] + u[6], p3 = u[3] + u[7];
    R m0 = u[4] - u[0], m1 = u[5] - u[1], m2 = u[6] - u[2], m3 = u[7] - u[3];
    R pa = p0 + p2, pb = p1 + p3, pc = p2 - p0, pd = p1 - p3;
    R ma = m0 + m2, mb = m1 + m3, mc = m2 - m0, md = m1 - m3;
    Modes<R> s;
    s.xi = pc + pd; s.eta = pc - pd; s.xe = pa - pb;
    s.zeta = ma + mb; s.xz = mc + md; s.ez = mc - md; s.xez = ma - mb;
    return s;
}

template <typename R>
__device__ __forceinline__ void inv8(const Modes<R> &c, R f[8])
{
    R q0 = -c.xi - c.eta + c.xe, q1 = c.xi - c.eta - c.xe;
    R q2 = c.xi + c.eta + c.xe, q3 = -c.xi + c.eta - c.xe;
    R r0 = c.zeta - c.xz - c.ez + c.xez, r1 = c.zeta + c.xz - c.ez - c.xez;
    R r2 = c.zeta + c.xz + c.ez + c.xez, r3 = c.zeta - c.xz + c.ez - c.xez;
    f[0] = q0 - r0; f[1] = q1 - r1; f[2] = q2 - r2; f[3] = q3 - r3;
    f[4] = q0 + r0; f[5] = q1 + r1; f[6] = q2 + r2; f[7] = q3 + r3;
}

template <typename R>
__device__ __forceinline__ void load_state(const R *r, int64_t e, R out[4])
{
    const R *p = r + 4 * e;
    out[0] = p[0]; out[1] = p[1]; out[2] = p[2]; out[3] = p[3];
}
template <>
__device__ __forceinline__ void load_state<float>(const float *r, int64_t e, float out[4])
{
    float4 v = reinterpret_cast<const float4 *>(r)[e];
    out[0] = v.x; out[1] = v.y; out[2] = v.z; out[3] = v.w;
}
template <typename R>
__device__ __forceinline__ void store_state(R *r, int64_t e, const R in[4])
{
    R *p = r + 4 * e;
    p[0] = in[0]; p[1] = in[1]; p[2] = in[2]; p[3] = in[3];
}
template <>
__device__ __forceinline__ void store_state<float>(float *r, int64_t e, const float in[4])
{
    reinterpret_cast<float4 *>(r)[e] = make_float4(in[0], in[1], in[2], in[3]);
}

// One point of a box element: Green strain of the displacement gradient G
// (= F - I, row-major), ply frame, law (thresholds r), back to the global
// frame, nominal stress Pn = F S (row-major).  Returns S:E in the ply frame
// (twice the secant energy density).  exact: in, 1 for an element that two
// workgroups evaluate (the surrogate then keeps the exact law); out, as
// sur_update reports it.
template <typename R, bool SUR, bool PLAS = false>
__device__ __forceinline__ R box_point(const R G[9], const PlyC<R> &P, R vol, R r[4], bool &changed, R Pn[9],
                                       const uint4 *sur_pk, float sur_dmg, float sur_res, int &exact,
                                       R *ep = nullptr, bool *pchanged = nullptr)
{
    const R G00 = G[0], G01 = G[1], G02 = G[2], G10 = G[3], G11 = G[4], G12 = G[5];
    const R G20 = G[6], G21 = G[7], G22 = G[8];
    // Green strain E = (G + G^T + G^T G)/2, formed without the 1 + small - 1 cancellation
    R E00 = G00 + R(0.5) * (G00 * G00 + G10 * G10 + G20 * G20);
    R E11 = G11 + R(0.5) * (G01 * G01 + G11 * G11 + G21 * G21);
    R E22 = G22 + R(0.5) * (G02 * G02 + G12 * G12 + G22 * G22);
    R E01 = R(0.5) * (G01 + G10 + G00 * G01 + G10 * G11 + G20 * G21);
    R E02 = R(0.5) * (G02 + G20 + G00 * G02 + G10 * G12 + G20 * G22);
    R E12 = R(0.5) * (G12 + G21 + G01 * G02 + G11 * G12 + G21 * G22);
    // to the ply frame (fibre at angle theta about Z)
    const R c = P.c, s = P.s, cc = c * c, ss = s * s, cs = c * s;
    R e[6];
    e[0] = cc * E00 + R(2) * cs * E01 + ss * E11;
    e[1] = ss * E00 - R(2) * cs * E01 + cc * E11;
    e[2] = E22;
    e[3] = R(2) * (-s * E02 + c * E12);
    e[4] = R(2) * (c * E02 + s * E12);
    e[5] = R(2) * (-cs * E00 + (cc - ss) * E01 + cs * E11);
    R sg[6];
    const bool shared = exact == 1;
    exact = 0;
    if constexpr (PLAS) {
        // plastic strains first; e becomes the elastic strain (its energy is
        // the recoverable one returned below)
        *pchanged = P.plas ? plastic_return(P, e, ep) : false;
    }
    if constexpr (SUR) {
        if (P.law == 2)
            sur_update(P, vol, e, r, sg, changed, sur_pk + (int64_t)P.sur * (SUR_PACK_BYTES / 16), sur_dmg, sur_res,
                       exact, shared);
        else
            cdm_update(P, vol, e, r, sg, changed);
    } else {
        // a surrogate ply keeps the exact law in this build; its unscreened
        // points are counted (those the surrogate build would consult)
        const bool scr = cdm_update(P, vol, e, r, sg, changed);
        if (P.law == 2) exact = scr ? 2 : 1;
    }
    // back to the global frame
    R S00 = cc * sg[0] - R(2) * cs * sg[5] + ss * sg[1];
    R S11 = ss * sg[0] + R(2) * cs * sg[5] + cc * sg[1];
    R S22 = sg[2];
    R S01 = cs * sg[0] + (cc - ss) * sg[5] - cs * sg[1];
    R S02 = c * sg[4] - s * sg[3];
    R S12 = s * sg[4] + c * sg[3];
    // nominal stress P = F S (index form (F S)_{iJ})
    R F00 = R(1) + G00, F11 = R(1) + G11, F22 = R(1) + G22;
    Pn[0] = F00 * S00 + G01 * S01 + G02 * S02;
    Pn[1] = F00 * S01 + G01 * S11 + G02 * S12;
    Pn[2] = F00 * S02 + G01 * S12 + G02 * S22;
    Pn[3] = G10 * S00 + F11 * S01 + G12 * S02;
    Pn[4] = G10 * S01 + F11 * S11 + G12 * S12;
    Pn[5] = G10 * S02 + F11 * S12 + G12 * S22;
    Pn[6] = G20 * S00 + G21 * S01 + F22 * S02;
    Pn[7] = G20 * S01 + G21 * S11 + F22 * S12;
    Pn[8] = G20 * S02 + G21 * S12 + F22 * S22;
    return sg[0] * e[0] + sg[1] * e[1] + sg[2] * e[2] + sg[3] * e[3] + sg[4] * e[4] + sg[5] * e[5];
}

// One point with hourglass control.  Returns the force coefficients on the
// corner basis (forces = inv8 of each).  PLAS: ep is the point's plastic state.
template <typename R, bool SUR, bool PLAS = false>
__device__ void hex_box_force(const R ux[8], const R uy[8], const R uz[8], R hx, R hy, R hz,
                              R ihx, R ihy, R ihz, const PlyC<R> &P, R kappa, R r[4], bool &changed,
                              Modes<R> &cx, Modes<R> &cy, Modes<R> &cz, R &uel,
                              const uint4 *sur_pk, float sur_dmg, float sur_res, int &exact,
                              R *ep = nullptr, bool *pchanged = nullptr)
{
    Modes<R> sx = fwd8(ux), sy = fwd8(uy), sz = fwd8(uz);
    const R gx = R(0.25) * ihx, gy = R(0.25) * ihy, gz = R(0.25) * ihz;
    // displacement gradient G = F - I (mean gradient)
    const R G[9] = {sx.xi * gx, sx.eta * gy, sx.zeta * gz, sy.xi * gx, sy.eta * gy, sy.zeta * gz,
                    sz.xi * gx, sz.eta * gy, sz.zeta * gz};
    const R vol = hx * hy * hz;
    R Pn[9];
    const R w = box_point<R, SUR, PLAS>(G, P, vol, r, changed, Pn, sur_pk, sur_dmg, sur_res, exact, ep, pchanged);
    const R ax = R(0.25) * hy * hz, ay = R(0.25) * hx * hz, az = R(0.25) * hx * hy;
    // hourglass: k = kappa Cmax V sum b^2 / 3, q = s/8, force coefficient k s / 64
    const R khg = kappa * P.cmax * vol * (ihx * ihx + ihy * ihy + ihz * ihz) * R(1.0 / 6.0);
    const R kh = khg * R(1.0 / 64.0);
    cx.xi = Pn[0] * ax; cx.eta = Pn[1] * ay; cx.zeta = Pn[2] * az;
    cy.xi = Pn[3] * ax; cy.eta = Pn[4] * ay; cy.zeta = Pn[5] * az;
    cz.xi = Pn[6] * ax; cz.eta = Pn[7] * ay; cz.zeta = Pn[8] * az;
    cx.ez = kh * sx.ez; cx.xz = kh * sx.xz; cx.xe = kh * sx.xe; cx.xez = kh * sx.xez;
    cy.ez = kh * sy.ez; cy.xz = kh * sy.xz; cy.xe = kh * sy.xe; cy.xez = kh * sy.xez;
    cz.ez = kh * sz.ez; cz.xz = kh * sz.xz; cz.xe = kh * sz.xe; cz.xez = kh * sz.xez;
    R q2 = sx.ez * sx.ez + sx.xz * sx.xz + sx.xe * sx.xe + sx.xez * sx.xez
         + sy.ez * sy.ez + sy.xz * sy.xz + sy.xe * sy.xe + sy.xez * sy.xez
         + sz.ez * sz.ez + sz.xz * sz.xz + sz.xe * sz.xe + sz.xez * sz.xez;
    uel = R(0.5) * vol * w + R(0.5) * khg * q2 * R(1.0 / 64.0);
}

// Full 2x2x2 Gauss integration of the same box (the paper's element,
// Section 2).  At the point (xi, eta, zeta) = (+-g, +-g, +-g), g = 1/sqrt(3),
// the gradient of the trilinear field is the mean gradient plus the mixed
// corner modes weighted by the point's coordinates, e.g.
//   du/dx = (s.xi + eta s.xe + zeta s.xz + eta zeta s.xez) / (4 hx);
// each point calls the law with its own thresholds r[g], and its virtual work
// (weight det J = V/8) lands on all seven corner-basis coefficients.  There
// is no hourglass control.  The thresholds of point g are record e8 + g gs of
// rstate (with plasticity, also its plastic state in epstate), read one point
// ahead and written back (by the owning lane) when they changed, so at most
// two points' states are live at a time.
template <typename R, bool PLAS = false>
__device__ void hex_box_force_full(const R ux[8], const R uy[8], const R uz[8], R hx, R hy, R hz,
                                   R ihx, R ihy, R ihz, const PlyC<R> &P, R *rstate, int64_t e8, int64_t gs,
                                   bool own, Modes<R> &cx, Modes<R> &cy, Modes<R> &cz, R &uel,
                                   R *epstate = nullptr)
{
    const Modes<R> sx = fwd8(ux), sy = fwd8(uy), sz = fwd8(uz);
    const R gx = R(0.25) * ihx, gy = R(0.25) * ihy, gz = R(0.25) * ihz;
    const R vol = hx * hy * hz, wq = R(0.125) * vol;
    const R gp = R(0.57735026918962576451);
    const R ax = wq * gx, ay = wq * gy, az = wq * gz;
    cx = cy = cz = Modes<R>{R(0), R(0), R(0), R(0), R(0), R(0), R(0)};
    R wsum = R(0);
    // the next point's thresholds (and plastic state) are loaded while this
    // point is computed
    R rn[4], epn[4];
    load_state(rstate, e8, rn);
    if constexpr (PLAS) load_state(epstate, e8, epn);
#pragma unroll 1
    for (int g = 0; g < 8; ++g) {
        R rg[4] = {rn[0], rn[1], rn[2], rn[3]};
        const int64_t nxt = e8 + (g < 7 ? g + 1 : 7) * gs;
        load_state(rstate, nxt, rn);
        R epg[4];
        if constexpr (PLAS) {
#pragma unroll
            for (int q = 0; q < 4; ++q) epg[q] = epn[q];
            load_state(epstate, nxt, epn);
        }
        const R xi = (g & 1) ? gp : -gp, eta = (g & 2) ? gp : -gp, zeta = (g & 4) ? gp : -gp;
        const R ez = eta * zeta, xz = xi * zeta, xe = xi * eta;
        R G[9];
        const Modes<R> *sm[3] = {&sx, &sy, &sz};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const Modes<R> &m = *sm[c];
            G[3 * c + 0] = gx * (m.xi + eta * m.xe + zeta * m.xz + ez * m.xez);
            G[3 * c + 1] = gy * (m.eta + xi * m.xe + zeta * m.ez + xz * m.xez);
            G[3 * c + 2] = gz * (m.zeta + xi * m.xz + eta * m.ez + xe * m.xez);
        }
        R Pn[9];
        bool ch = false, pch = false;
        int ex = 0;
        // The law's element-size terms (crack band, capped strengths) are
        // needed only where a point leaves the elastic screen: an empty asm
        // on the volume keeps the compiler from hoisting them out of this
        // loop, where every element would compute them whether used or not.
        R volg = vol;
        asm volatile("" : "+v"(volg));
        wsum += box_point<R, false, PLAS>(G, P, volg, rg, ch, Pn, nullptr, 0.f, 0.f, ex, epg, &pch);
        if (own && ch) store_state(rstate, e8 + g * gs, rg);
        if constexpr (PLAS) {
            if (own && pch) store_state(epstate, e8 + g * gs, epg);
        }
        Modes<R> *cm[3] = {&cx, &cy, &cz};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            Modes<R> &m = *cm[c];
            const R q0 = ax * Pn[3 * c], q1 = ay * Pn[3 * c + 1], q2 = az * Pn[3 * c + 2];
            m.xi += q0; m.eta += q1; m.zeta += q2;
            m.xe += eta * q0 + xi * q1;
            m.xz += zeta * q0 + xi * q2;
            m.ez += zeta * q1 + eta * q2;
            m.xez += ez * q0 + xz * q1 + xe * q2;
        }
    }
    uel = R(0.5) * wq * wsum;
}

// ---------------------------------------------------------------------------
// fused element / node kernel
// ---------------------------------------------------------------------------

__device__ __forceinline__ int xcd_tile(int b, int nb)
{
    // consecutive tiles on one XCD: blocks are dealt round-robin to 8 XCDs
    const int per = nb / 8, rem = nb % 8, x = b % 8, loc = b / 8;
    return x < rem ? x * (per + 1) + loc : rem * (per + 1) + (x - rem) * per + loc;
}

// Read-only tables (plies, layers, per-plane factors) are read through the
// constant address space: the kernel never writes them, and loads from a
// uniform address then use the scalar cache, whose waits do not drain the
// vector loads in flight (the next node plane).
// a whole read-only record through the constant address space (word by word)
template <typename T>
__device__ __forceinline__ T cload(const T *p)
{
    static_assert(sizeof(T) % 4 == 0, "record of whole words");
    T v;
    const __attribute__((address_space(4))) int *src = (const __attribute__((address_space(4))) int *)p;
    int *dst = reinterpret_cast<int *>(&v);
#pragma unroll
    for (int i = 0; i < (int)(sizeof(T) / 4); ++i) dst[i] = src[i];
    return v;
}

// Values that are the same in every lane, made visibly so: addresses built
// from them stay scalar (constants then come through the scalar cache, whose
// waits do not drain the vector loads in flight).
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ float uni(float x)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_readfirstlane(__builtin_bit_cast(int, x)));
}
__device__ __forceinline__ double uni(double x)
{
    const int2 v = __builtin_bit_cast(int2, x);
    return __builtin_bit_cast(double, make_int2(__builtin_amdgcn_readfirstlane(v.x), __builtin_amdgcn_readfirstlane(v.y)));
}


// A node's xyz (24 bytes, 8-byte aligned) as a 16-byte and an 8-byte access:
// two memory instructions per node and array instead of three.
typedef unsigned U4a __attribute__((ext_vector_type(4), aligned(4)));
typedef unsigned U2a __attribute__((ext_vector_type(2), aligned(4)));
__device__ __forceinline__ void load_xyz(const double *p, double (&o)[3])
{
    const U4a a = *reinterpret_cast<const U4a *>(p);
    const U2a b = *reinterpret_cast<const U2a *>(p + 2);
    o[0] = __hiloint2double((int)a.y, (int)a.x);
    o[1] = __hiloint2double((int)a.w, (int)a.z);
    o[2] = __hiloint2double((int)b.y, (int)b.x);
}
__device__ __forceinline__ void store_xyz(double *p, const double (&v)[3])
{
    U4a a;
    U2a b;
    a.x = (unsigned)__double2loint(v[0]); a.y = (unsigned)__double2hiint(v[0]);
    a.z = (unsigned)__double2loint(v[1]); a.w = (unsigned)__double2hiint(v[1]);
    b.x = (unsigned)__double2loint(v[2]); b.y = (unsigned)__double2hiint(v[2]);
    *reinterpret_cast<U4a *>(p) = a;
    *reinterpret_cast<U2a *>(p + 2) = b;
}

// stage rows of the books reduction: 64 or more tiles each, at most PDN_STAGE
__device__ __forceinline__ int books_stage_rows(int nblk) { return rmax(1, rmin(PDN_STAGE, nblk / 64)); }

// a double moved between lanes by a DPP lane pattern (both words alike)
template <int CTRL>
__device__ __forceinline__ double dpp_f64(double v)
{
    const int2 w = __builtin_bit_cast(int2, v);
    int2 r;
    r.x = __builtin_amdgcn_update_dpp(0, w.x, CTRL, 0xF, 0xF, true);
    r.y = __builtin_amdgcn_update_dpp(0, w.y, CTRL, 0xF, 0xF, true);
    return __builtin_bit_cast(double, r);
}

// a float of the lane to the left within a row of 16 lanes (0 in the row's first lane)
__device__ __forceinline__ float row_left(float v)
{
    return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(0, __builtin_bit_cast(int, v), 0x111, 0xF, 0xF, true));
}

// a double of lane l, uniform
__device__ __forceinline__ double lane_f64(double v, int l)
{
    const int2 w = __builtin_bit_cast(int2, v);
    int2 r;
    r.x = __builtin_amdgcn_readlane(w.x, l);
    r.y = __builtin_amdgcn_readlane(w.y, l);
    return __builtin_bit_cast(double, r);
}

// sum over the 64 lanes of a wave in a fixed order: pairs, quads, half rows
// and rows of 16 lanes by DPP lane patterns (commutative steps, so every lane
// of a row holds the same row sum), then the four row sums in order
__device__ __forceinline__ double wave_sum(double v)
{
    v += dpp_f64<0xB1>(v);                   // quad_perm [1,0,3,2]
    v += dpp_f64<0x4E>(v);                   // quad_perm [2,3,0,1]
    v += dpp_f64<0x141>(v);                  // row_half_mirror
    v += dpp_f64<0x140>(v);                  // row_mirror
    return (lane_f64(v, 0) + lane_f64(v, 16)) + (lane_f64(v, 32) + lane_f64(v, 48));
}

// Sum of acc over the workgroup, deterministic (fixed lane pattern per wave,
// waves in order); the NTM totals land in out[0], out[stride], ... from threads 0..NTM-1.
template <int NT, int NTM = PDN_NTERMS>
__device__ void block_reduce_store(const double *acc, double *out, int stride, double *sh)
{
    // deterministic: fixed lane pattern inside each wave, waves summed in order
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NW = NT / 64;
#pragma unroll
    for (int k = 0; k < NTM; ++k) {
        const double v = wave_sum(acc[k]);
        if (lane == 0) sh[k * NW + wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < NTM) {
        double v = 0;
        for (int w = 0; w < NW; ++w) v += sh[threadIdx.x * NW + w];
        out[threadIdx.x * stride] = v;
    }
}

// Closing a contact pass (one workgroup of NT threads, after the pass):
// fixed-order sums of the previous pass's element partials and this pass's
// contact partials give the energy books of the last complete level
// (reported one step late), the striker is advanced and the history row of
// the step written.
template <int NT, typename R>
__device__ void contact_books(const ElemArgs<R> &A, double *sh)
{
    __shared__ double tot[PDN_NTERMS];
    const int t = threadIdx.x, nblk = A.tiles_x * A.tiles_y;
    double q[PDN_NTERMS];
#pragma unroll
    for (int k = 0; k < PDN_NTERMS; ++k) q[k] = 0.0;
    // element terms of the previous pass: its stage rows; contact terms of
    // this pass: the tiles around the candidate window (others add zeros)
    const int ns = books_stage_rows(nblk), wtx = A.wt1 - A.wt0, nw = wtx * (A.wu1 - A.wu0);
    for (int b = t; b < ns; b += NT) {
#pragma unroll
        for (int k = 0; k < T_FC; ++k) q[k] += A.stage[b * PDN_NTERMS + k];
    }
    for (int b = t; b < nw; b += NT) {
        const int tile = A.wt0 + b % wtx + A.tiles_x * (A.wu0 + b / wtx);
#pragma unroll
        for (int k = T_FC; k < PDN_NTERMS; ++k) q[k] += A.partials[(int64_t)k * A.prow + tile];
    }
    block_reduce_store<NT>(q, tot, 1, sh);
    __syncthreads();
    if (t != 0) return;
    // every update is made on a register copy, loaded and stored back at once
    DevGlobals G = *A.gl;
    const double *P = tot;
    const double dt = A.dt, g = A.grav, ms = G.ms;
    // the striker prediction of the pass (same arithmetic as its workgroups)
    const double Fz = G.Fprev[2];
    const double az = -g - Fz / ms;
    const double cz_old = G.c[2], Vz_old = G.V[2];
    const double cz = cz_old + dt * Vz_old + 0.5 * dt * dt * az;
    const double kes_level = 0.5 * ms * (G.V[0] * G.V[0] + G.V[1] * G.V[1] + G.V[2] * G.V[2]);
    // books of level s (= completed steps), final now
    if (!G.first) {
        G.e_wint += G.half_int + P[T_WA];
        G.e_wc += P[T_WCP];
    } else {
        G.mz0 = P[T_MZ];
    }
    // gravity is constant: its work is -g (sum m d_z - initial), the
    // trapezoidal sum telescoped (phi = 1)
    G.e_wgp = -g * (P[T_MZ] - G.mz0);
    G.half_int = P[T_WB] + P[T_WIC];
    G.e_kep = P[T_KE] + P[T_KEC];
    G.e_uel = P[T_UEL];
    G.e_kes = kes_level;
    G.e_ws = G.ws_acc;
    G.e_wgs = G.wgs_acc;
    G.e_level = (double)G.step;
    // the element terms are those of the previous pass: its build decides
    // whether its points consulted the network
    if (G.plain_prev) {
        G.sur_unscreened += P[T_SURN];      // the plain build: no point consulted the network
    } else {
        G.fallback_gp += P[T_AUX];
        G.sur_gp += P[T_SURN];
    }
    G.plain_prev = A.count_sur;
    // a non-finite displacement or velocity propagates into these sums
    if (!(isfinite(P[T_KE]) && isfinite(P[T_WA]) && isfinite(P[T_WB]) && isfinite(P[T_MZ])))
        G.flag_unstable = 1;
    if (P[T_OVF] > 0.0) G.flag_overflow = 1;
    // striker update and its works (force frozen over the step)
    const double dz = cz - cz_old;
    G.ws_acc += Fz * dz;
    G.wgs_acc += ms * g * (-dz);
    G.c[2] = cz;
    G.V[2] = Vz_old + dt * az;
    G.Fprev[0] = P[T_FC]; G.Fprev[1] = P[T_FC + 1]; G.Fprev[2] = P[T_FC + 2];
    const int passes = P[T_REL] > 0.0 ? 2 : 1;
    G.reset_passes += passes;
    G.released += (int64_t)P[T_REL];
    if (passes > G.max_passes) G.max_passes = passes;
    G.active = (int64_t)P[T_ACT];
    if (G.step < G.hist_cap) {
        A.hist[3 * G.step + 0] = (double)(G.step + 1) * dt;
        A.hist[3 * G.step + 1] = -P[T_FC + 2];
        A.hist[3 * G.step + 2] = -(cz - G.c0[2]);
    }
    G.step += 1;
    G.first = 0;
    *A.gl = G;
}

// one workgroup's tile of one plate; block partials go to A.partials[tile].
// SUR: plies with law 2 use the surrogate network (a separate instantiation,
// so that the plain path keeps its register budget); PLAS: plies with shear
// plasticity carry their plastic state (another instantiation, one point)
template <typename R, int TX, int TY, bool SUR, int NGP, bool PLAS = false>
__device__ __forceinline__ void elem_node_tile(const ElemArgs<R> &A, const int tile)
{
    // element slots follow the node rows: element (a, b) is slot a + NCX b,
    // the thread whose node is the element's corner 0 (the last slot of a row
    // has no element), so that a wave's LDS accesses are consecutive words
    constexpr int NCX = TX + 1, NCY = TY + 1, NC = NCX * NCY, NE = NCX * TY;
    constexpr int NT = PDN_TILE_THREADS(TX, TY);
    constexpr bool F32 = sizeof(R) == 4;
    __shared__ R U[2][3][NC];               // node planes k-1, k in the element type (slot k & 1)
    // With rows of 16 element slots (one DPP row, FP32) an element lane adds
    // its left neighbour's corner forces by a lane move: the LDS then holds,
    // per node column, the part of row b (corners 0 + 1) and of row b - 1
    // (corners 3 + 2) of each face instead of the four corners.
    constexpr bool RD = F32 && NCX == 16;
    __shared__ R Fs[2][RD ? 2 : 4][3][NE];  // [bottom/top][corner or row part][xyz][slot]
    __shared__ double red[PDN_NTERMS * (NT / 64)];

    const int t = threadIdx.x;
    const int tx = tile % A.tiles_x, ty = tile / A.tiles_x;
    const int e0x = tx * (TX - 1), e0y = ty * (TY - 1);
    const bool lastx = tx == A.tiles_x - 1, lasty = ty == A.tiles_y - 1;
    const int nx = A.nx, ny = A.ny;
    const int64_t plane = (int64_t)(nx + 1) * (ny + 1);

    // element role: one element column per thread; ewave: the thread's wave has some
    const int ea = t % NCX, eb = t / NCX;
    const bool erole = t < NE && ea < TX;
    const bool ewave = (t & ~63) < NE;
    const int ie = e0x + ea, je = e0y + eb;
    const bool evalid = erole && ie < nx && je < ny;
    const bool eown = evalid && (ea < TX - 1 || lastx) && (eb < TY - 1 || lasty);
    const int s0 = ea + NCX * eb;

    // node role: one node column per thread
    const bool nrole = t < NC;
    const int np = t % NCX, nq = t / NCX;
    const int gi = e0x + np, gj = e0y + nq;
    const bool nvalid = nrole && gi <= nx && gj <= ny;
    const int lox = tx == 0 ? 0 : e0x + 1, hix = lastx ? nx + 1 : e0x + TX;
    const int loy = ty == 0 ? 0 : e0y + 1, hiy = lasty ? ny + 1 : e0y + TY;
    const bool nown = nvalid && gi >= lox && gi < hix && gj >= loy && gj < hiy;
    const int64_t col = nvalid ? gi + (int64_t)(nx + 1) * gj : 0;

    // per-thread constants of the march, loaded once (inside the loop their
    // loads could not move past the state stores and would stall every layer)
    const int iv = rmin(ie, nx - 1), jv = rmin(je, ny - 1);
    const R ehx = A.hx[iv], ehy = A.hy[jv], eihx = A.ihx[iv], eihy = A.ihy[jv];
    const double mxy = nvalid ? A.mx[gi] * A.my[gj] : 0.0;
    const double imxy = nvalid ? A.imx[gi] * A.imy[gj] : 0.0;

    double carry[3] = {0, 0, 0}, fin[3];
    double acc[PDN_NTERMS];
#pragma unroll
    for (int k = 0; k < PDN_NTERMS; ++k) acc[k] = 0.0;

    // node plane k is fetched from HBM two iterations ahead into one of two
    // register sets (the loop is unrolled by two so that a set is never
    // touched while its loads are in flight), then staged in LDS
    double pdA[3] = {0, 0, 0}, pvA[3] = {0, 0, 0}, pdB[3] = {0, 0, 0}, pvB[3] = {0, 0, 0};
    // Every lane issues the same loads in every layer (clamped addresses for
    // lanes without a node, a repeat of the top plane past it): the waits for
    // a load then count only loads issued after it, and the plane in flight
    // is never drained early.
    // Velocities are used for owned nodes only: other lanes read the nearest
    // owned node's, a line the wave reads anyway.
    const int64_t vcol = rmin(rmax(gi, lox), hix - 1) + (int64_t)(nx + 1) * rmin(rmax(gj, loy), hiy - 1);
    auto fetch_plane = [&](int k, double (&pd)[3], double (&pv)[3]) {
        const int64_t kk = plane * (int64_t)rmin(k, A.K - 1);
        const int64_t nk = (nvalid ? col : 0) + kk, nv = vcol + kk;
        load_xyz(A.d_in + 3 * nk, pd);
        load_xyz(A.v_in + 3 * nv, pv);
    };
    // FP64 displacement and velocity of the thread's own node in the last two
    // staged planes, in registers: slot S of a call site is a compile-time
    // parity (the loop is unrolled by two), so the arrays stay in registers
    double sd[2][3] = {{0, 0, 0}, {0, 0, 0}}, sv[2][3] = {{0, 0, 0}, {0, 0, 0}};
    auto stage_plane = [&](auto S, int k, const double (&pd)[3], const double (&pv)[3]) {
        constexpr int s = decltype(S)::value;
        const int p = k & 1;
        if (nvalid) {
#pragma unroll
            for (int c = 0; c < 3; ++c) U[p][c][t] = (R)pd[c];
        } else if (nrole) {
            U[p][0][t] = U[p][1][t] = U[p][2][t] = R(0);
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            sd[s][c] = pd[c];
            sv[s][c] = pv[c];
        }
    };
    // damage thresholds of the element in layer l, fetched one layer ahead
    // and the interface damage threshold of the node pair, for a cohesive layer.
    R rn[4] = {R(1), R(1), R(1), R(1)};
    // Both are loaded for every layer (the other one from a fixed address):
    // the same two loads per lane and layer keep the wait counts static.
    // Values of lanes without an element or node pair, or of an elastic ply,
    // are not used.
    R rdn = R(0);
    R epn[4] = {R(0), R(0), R(0), R(0)};   // plastic state of the element in layer l (PLAS)
    auto fetch_r = [&](int l) {
        const LayerInfo Lr = cload(A.layers + rmin(l, A.NL - 1));
        const int lt = uni(Lr.type), li = uni(Lr.index);
        const int64_t eidx = lt == 0 ? iv + (int64_t)nx * (jv + (int64_t)ny * li) : 0;
        const int64_t pidx = lt == 0 ? 0 : (nvalid ? col : 0) + plane * li;
        if constexpr (NGP == 1) load_state(A.r, eidx, rn);
        if constexpr (PLAS && NGP == 1) load_state(A.ep, eidx, epn);
        rdn = A.rd[pidx];
    };

    // lumped-mass integration of plane kp with total internal force f; next predictor
    // fixed-DOF bits: lateral clamp, and the bottom plane's support bits
    // (read once; the loop then needs neither the flag nor the table)
    const int fix_lat = (A.clamp_lateral && (gi == 0 || gi == nx || gj == 0 || gj == ny)) ? 7 : 0;
    const int fix_bot = fix_lat | (nvalid ? (int)A.bc_bottom[col] : 0);
    auto update_node = [&](auto S, int kp, const double f[3]) {
        constexpr int s = decltype(S)::value;
        const int64_t n = col + plane * kp;
        const int bits = kp == 0 ? fix_bot : fix_lat;
        const double m = mxy * cload(A.mz + kp);
        const double im = imxy * cload(A.imz + kp);
        const double dt = A.dt, g = A.grav;
        acc[T_MZ] += m * sd[s][2];             // gravity work = -g (sum m d_z - its initial value)
        double dn[3], vn[3], vvn = 0.0, vf = 0.0, vnf = 0.0;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double d = sd[s][c], v = sv[s][c];
            const bool fx = (bits >> c) & 1;
            const double fe = c == 2 ? -m * g : 0.0;
            const double a = fx ? 0.0 : (fe - f[c]) * im;
            vn[c] = fx ? 0.0 : v + dt * a;
            dn[c] = fx ? d : d + dt * v + A.phi * dt * dt * a;
            vvn += v * vn[c];
            vf += v * f[c];
            vnf += vn[c] * f[c];
        }
        // half-step kinetic energy and the two halves of the trapezoidal internal work
        acc[T_KE] += 0.5 * m * vvn;
        acc[T_WA] += 0.5 * dt * vf;
        acc[T_WB] += 0.5 * dt * vnf;
        store_xyz(A.d_out + 3 * n, dn);
        store_xyz(A.v_out + 3 * n, vn);
    };

    // ---- contact step (Section 2.1, Eqs. 2-3, Algorithms 1-2) ----
    // Detection on the predictor of a top-surface candidate, projection onto
    // the sphere, reaction, release of adhesion nodes (Eq. 2) with the repeated
    // pass.  A node's correction depends on that node only, so every workgroup
    // that reads it (its owner and the neighbours reading it as halo) corrects
    // its copy identically; the owner alone stores state and sums.
    auto contact_correct = [&](double (&pd)[3], double (&pv)[3]) {
        // Rigid body first (Gauss-Seidel): every workgroup advances the striker
        // with the force of the plate's last step frozen over the step (the
        // books kernel repeats this arithmetic and stores it).  Lateral motion
        // of the striker is constrained.
        const DevGlobals *G = A.gl;
        const double Fz = G->Fprev[2];
        const double az = -A.grav - Fz / G->ms;
        const double cz = G->c[2] + A.dt * G->V[2] + 0.5 * A.dt * A.dt * az;
        const double cx = G->c[0], cy = G->c[1], Rs = G->R;
        if (!nvalid || gi < A.ci0 || gi >= A.ci1 || gj < A.cj0 || gj >= A.cj1) return;
        const int64_t j = (gi - A.ci0) + (int64_t)(A.ci1 - A.ci0) * (gj - A.cj0);
        const double dt = A.dt, phi = A.phi;
        const bool lat = A.clamp_lateral && (gi == 0 || gi == nx || gj == 0 || gj == ny);
        const double m = mxy * cload(A.mz + (A.K - 1));
        const double rx = A.xs[gi] + pd[0] - cx, ry = A.ys[gj] + pd[1] - cy, rz = A.ztop + pd[2] - cz;
        const double dist = sqrt(rx * rx + ry * ry + rz * rz);
        const double gap = dist - Rs;
        double nv[3] = {0.0, 0.0, -1.0};
        if (dist > 0.0) { nv[0] = rx / dist; nv[1] = ry / dist; nv[2] = rz / dist; }
        bool act = A.active_in[j] != 0 || (gap < 0.0 && rz <= 0.0);
        double fc[3] = {0, 0, 0};
        int passes = 0, released = 0;
        for (;;) {
            ++passes;
            bool rel = false;
            if (act) {
                double fn = 0;
                for (int c = 0; c < 3; ++c) {
                    const double d1 = lat ? 0.0 : -gap * nv[c];
                    fc[c] = m * d1 / (phi * dt * dt);
                    fn += fc[c] * nv[c];
                }
                if (fn < 0.0) { act = false; rel = true; ++released; fc[0] = fc[1] = fc[2] = 0.0; }
            }
            if (!rel || passes >= 8) break;
        }
        double dv[3] = {0, 0, 0};
        if (act) {
            for (int c = 0; c < 3; ++c) {
                const double da = fc[c] / m;
                dv[c] = dt * da;
                pd[c] = pd[c] + phi * dt * dt * da;
                pv[c] += dv[c];
            }
        }
        if (!nown) return;
        A.active_out[j] = act ? 1 : 0;
        if (act) {
            acc[T_ACT] += 1.0;
            const bool ring = (gi == A.ci0 && gi > 0) || (gi == A.ci1 - 1 && gi < nx) ||
                              (gj == A.cj0 && gj > 0) || (gj == A.cj1 - 1 && gj < ny);
            if (ring) acc[T_OVF] += 1.0;                          // left the search window
        }
        acc[T_REL] += (double)released;
        for (int c = 0; c < 3; ++c) {
            const double vpv = A.vprev[3 * j + c];
            acc[T_FC + c] += fc[c];                               // reaction sum
            acc[T_KEC] += 0.5 * m * vpv * dv[c];                  // kinetic-energy correction
            acc[T_WIC] += 0.5 * dt * dv[c] * A.fside[3 * j + c];  // internal-work correction
            acc[T_WCP] += 0.5 * dt * vpv * (A.fcprev[3 * j + c] + fc[c]);   // contact work on the plate
            A.vprev[3 * j + c] = pv[c];
            A.fcprev[3 * j + c] = fc[c];
            A.cand[6 * j + c] = pd[c];
            A.cand[6 * j + 3 + c] = pv[c];
        }
    };

    // layer k-1 (between node planes k-1 and k), then the update of plane k-1
    // S: register slot of plane k (plane k - 1 is in the other one)
    auto layer_step = [&](auto S, int k, double (&pd)[3], double (&pv)[3]) {
        constexpr int s = decltype(S)::value;
        const std::integral_constant<int, 1 - s> S1{};
        const LayerInfo Lk = cload(A.layers + (k - 1));
        const int ltype = uni(Lk.type), lply = uni(Lk.ply), lidx = uni(Lk.index);
        const R lhz = (R)uni(Lk.hz), lihz = (R)uni(Lk.ihz);
        stage_plane(S, k, pd, pv);
        R r[4] = {rn[0], rn[1], rn[2], rn[3]};
        R ep[4] = {epn[0], epn[1], epn[2], epn[3]};
        const R rdl = rdn;
        // thresholds first: the wait for them next layer then leaves the plane
        // loads (issued after them) in flight
        fetch_r(k);
        fetch_plane(k + 2, pd, pv);
        if (ltype == 0) {
            __syncthreads();
            if (ewave) {
                // every lane of a wave with element columns evaluates one (lanes
                // without a valid element take a stand-in and discard it), so
                // that wave-wide operations of the law see the whole wave
                const int kb = (k - 1) & 1, kt = k & 1;
                const int sb = erole ? s0 : 0;
                const int sl[4] = {sb, sb + 1, sb + 1 + NCX, sb + NCX};
                R ux[8], uy[8], uz[8];
#pragma unroll
                for (int q = 0; q < 4; ++q) {
                    ux[q] = U[kb][0][sl[q]]; uy[q] = U[kb][1][sl[q]]; uz[q] = U[kb][2][sl[q]];
                    ux[q + 4] = U[kt][0][sl[q]]; uy[q + 4] = U[kt][1][sl[q]]; uz[q + 4] = U[kt][2][sl[q]];
                }
                const PlyC<R> P = cload(A.ply + lply);
                bool changed = false;
                R uel;
                // an element on the rim of this tile that the neighbouring tile evaluates too
                int exact = ((ea == 0 && tx > 0) || (ea == TX - 1 && !lastx) || (eb == 0 && ty > 0) ||
                             (eb == TY - 1 && !lasty)) ? 1 : 0;
                Modes<R> cm[3];
                if constexpr (NGP == 8) {
                    // lanes without an element read a valid record (clamped) and write nothing
                    // a layer's records point by point: point g of every element of the
                    // layer, then point g + 1 (a wave's record loads are contiguous)
                    const int64_t gs = (int64_t)nx * ny;
                    const int64_t e8 = 8 * gs * lidx + iv + (int64_t)nx * jv;
                    hex_box_force_full<R, PLAS>(ux, uy, uz, ehx, ehy, lhz, eihx, eihy, lihz, P, A.r, e8, gs,
                                                eown, cm[0], cm[1], cm[2], uel, A.ep);
                    if (eown) acc[T_UEL] += (double)uel;
                } else {
                    bool pchanged = false;
                    hex_box_force<R, SUR, PLAS>(ux, uy, uz, ehx, ehy, lhz, eihx, eihy, lihz, P, A.kappa, r,
                                                changed, cm[0], cm[1], cm[2], uel, A.mlp, A.sur_dmg, A.sur_res,
                                                exact, ep, &pchanged);
                    if (eown) {
                        if (changed) store_state(A.r, ie + (int64_t)nx * (je + (int64_t)ny * lidx), r);
                        if constexpr (PLAS) {
                            if (pchanged) store_state(A.ep, ie + (int64_t)nx * (je + (int64_t)ny * lidx), ep);
                        }
                        acc[T_UEL] += (double)uel;
                        if (P.law == 2) {
                            if constexpr (SUR) {
                                // consulted: the network's answer was computed and checked
                                acc[T_AUX] += exact == 1 ? 1.0 : 0.0;  // checked and rejected: exact law
                                acc[T_SURN] += (exact == 0 || exact == 1) ? 1.0 : 0.0;
                            } else {
                                // points outside the screen (those a network build would consider)
                                acc[T_AUX] += exact == 1 ? 1.0 : 0.0;
                                acc[T_SURN] += exact != 2 ? 1.0 : 0.0;
                            }
                        }
                    }
                }
                if constexpr (RD) {
                    // every lane of the wave takes part in the lane moves
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        R f[8];
                        inv8(cm[c], f);
#pragma unroll
                        for (int q = 0; q < 8; ++q) f[q] = evalid ? f[q] : R(0);
                        // corners 1, 2 (bottom) and 5, 6 (top) of the element to the left
                        const R l1 = row_left(f[1]), l2 = row_left(f[2]), l5 = row_left(f[5]), l6 = row_left(f[6]);
                        if (t < NE) {
                            Fs[0][0][c][t] = f[0] + l1;                // node (a, b), bottom face
                            Fs[0][1][c][t] = f[3] + l2;                // node (a, b + 1), bottom face
                            Fs[1][0][c][t] = f[4] + l5;                // node (a, b), top face
                            Fs[1][1][c][t] = f[7] + l6;                // node (a, b + 1), top face
                        }
                    }
                } else if (erole) {
                    R *F0 = &Fs[0][0][0][t];
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        R f[8];
                        inv8(cm[c], f);
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            F0[(q * 3 + c) * NE] = evalid ? f[q] : R(0);                  // bottom corners
                            F0[((4 + q) * 3 + c) * NE] = evalid ? f[q + 4] : R(0);        // top corners
                        }
                    }
                }
            }
            __syncthreads();
            if (nown) {
                // node (np, nq) is corner 0 of element (np, nq), 1 of (np-1, nq),
                // 2 of (np-1, nq-1) and 3 of (np, nq-1); the four corner forces of
                // one layer are summed in the element type as (c0 + c1) + (c3 + c2),
                // for every tile shape
                R fb[3] = {R(0), R(0), R(0)}, ft[3] = {R(0), R(0), R(0)};
                if constexpr (RD) {
                    // rows nq (corners 0 + 1) and nq - 1 (corners 3 + 2), in this order
                    if (nq < TY) {
                        const int e = np + NCX * nq;
#pragma unroll
                        for (int c = 0; c < 3; ++c) { fb[c] += Fs[0][0][c][e]; ft[c] += Fs[1][0][c][e]; }
                    }
                    if (nq >= 1) {
                        const int e = np + NCX * (nq - 1);
#pragma unroll
                        for (int c = 0; c < 3; ++c) { fb[c] += Fs[0][1][c][e]; ft[c] += Fs[1][1][c][e]; }
                    }
                } else {
                    // the same sums from the four corners: row nq (corner 0, then
                    // corner 1 of the element to the left), then row nq - 1
                    // (corner 3, then corner 2 of the element to the left)
                    if (nq < TY) {
                        R pb[3] = {R(0), R(0), R(0)}, pt[3] = {R(0), R(0), R(0)};
                        if (np < TX) {
                            const int e = np + NCX * nq;
#pragma unroll
                            for (int c = 0; c < 3; ++c) { pb[c] = Fs[0][0][c][e]; pt[c] = Fs[1][0][c][e]; }
                        }
                        if (np >= 1) {
                            const int e = np - 1 + NCX * nq;
#pragma unroll
                            for (int c = 0; c < 3; ++c) { pb[c] += Fs[0][1][c][e]; pt[c] += Fs[1][1][c][e]; }
                        }
#pragma unroll
                        for (int c = 0; c < 3; ++c) { fb[c] += pb[c]; ft[c] += pt[c]; }
                    }
                    if (nq >= 1) {
                        R qb[3] = {R(0), R(0), R(0)}, qt[3] = {R(0), R(0), R(0)};
                        if (np < TX) {
                            const int e = np + NCX * (nq - 1);
#pragma unroll
                            for (int c = 0; c < 3; ++c) { qb[c] = Fs[0][3][c][e]; qt[c] = Fs[1][3][c][e]; }
                        }
                        if (np >= 1) {
                            const int e = np - 1 + NCX * (nq - 1);
#pragma unroll
                            for (int c = 0; c < 3; ++c) { qb[c] += Fs[0][2][c][e]; qt[c] += Fs[1][2][c][e]; }
                        }
#pragma unroll
                        for (int c = 0; c < 3; ++c) { fb[c] += qb[c]; ft[c] += qt[c]; }
                    }
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) { fin[c] = carry[c] + (double)fb[c]; carry[c] = (double)ft[c]; }
            }
        } else if (nown) {
            // zero-thickness interface, nodal (Newton-Cotes) points: the points of
            // the four elements sharing a node pair coincide, so the pair carries
            // one state and the summed tributary area
            const PlyC<R> P = cload(A.ply + lply);
            const int64_t pi = col + plane * lidx;
            R rd = rdl;                              // fetched one layer ahead
            R tau[3];
            bool changed;
            const R d1 = (R)(sd[s][0] - sd[1 - s][0]);
            const R d2 = (R)(sd[s][1] - sd[1 - s][1]);
            const R d3 = (R)(sd[s][2] - sd[1 - s][2]);
            czm_update(P, d1, d2, d3, rd, tau, changed);
            if (changed) A.rd[pi] = rd;
            const double ap = mxy;                   // (sum of adjacent widths / 2)(... / 2)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double ftc = ap * (double)tau[c];
                fin[c] = carry[c] - ftc;
                carry[c] = ftc;
            }
            acc[T_UEL] += 0.5 * ap * (double)(tau[0] * d1 + tau[1] * d2 + tau[2] * d3);
        }
        if (nown) update_node(S1, k - 1, fin);
    };
    const std::integral_constant<int, 0> S0{};
    const std::integral_constant<int, 1> S1{};

    fetch_plane(0, pdA, pvA);
    stage_plane(S0, 0, pdA, pvA);
    fetch_plane(1, pdB, pvB);
    fetch_plane(2, pdA, pvA);
    fetch_r(0);
    // layers below the top plane in pairs; the top plane is staged by one
    // call site after the contact step (its predictor is moved to set B)
    const int top = A.K - 1;
    int k = 1;
    for (; k + 1 < top; k += 2) {
        layer_step(S1, k, pdB, pvB);
        layer_step(S0, k + 1, pdA, pvA);
    }
    if (k < top) {
        layer_step(S1, k, pdB, pvB);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            pdB[c] = pdA[c];
            pvB[c] = pvA[c];
        }
    }
    // only workgroups whose node columns (halo included) meet the candidate
    // window have contact work (the others would load the striker for nothing)
    if (A.contact && e0x < A.ci1 && e0x + TX >= A.ci0 && e0y < A.cj1 && e0y + TY >= A.cj0)
        contact_correct(pdB, pvB);
    // the top call site stages into register slot 1: plane top - 1 must be in
    // slot 0, where an even top finds it in slot 1
    if ((top & 1) == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double a = sd[0][c], b = sv[0][c];
            sd[0][c] = sd[1][c];
            sv[0][c] = sv[1][c];
            sd[1][c] = a;
            sv[1][c] = b;
        }
    }
    layer_step(S1, top, pdB, pvB);
    if (nown) {
        update_node(S1, A.K - 1, carry);
        // internal force of a top-plane candidate (the contact step's internal-work correction)
        if (gi >= A.ci0 && gi < A.ci1 && gj >= A.cj0 && gj < A.cj1) {
            const int64_t ci = (gi - A.ci0) + (int64_t)(A.ci1 - A.ci0) * (gj - A.cj0);
            A.fside[3 * ci + 0] = carry[0];
            A.fside[3 * ci + 1] = carry[1];
            A.fside[3 * ci + 2] = carry[2];
        }
    }
    // Block partials: the element terms from every tile; the contact terms only
    // from the tiles whose contact terms the books read (those around the
    // candidate window, in a contact pass); the surrogate counters are zero
    // unless the surrogate is built in.
    if (A.contact && tx >= A.wt0 && tx < A.wt1 && ty >= A.wu0 && ty < A.wu1) {
        block_reduce_store<NT>(acc, A.partials + tile, A.prow, red);
    } else if constexpr (SUR) {
        block_reduce_store<NT, T_FC>(acc, A.partials + tile, A.prow, red);
    } else if (A.count_sur) {
        // surrogate plies stepped by this build: their unscreened points are counted
        block_reduce_store<NT, T_FC>(acc, A.partials + tile, A.prow, red);
    } else {
        block_reduce_store<NT, T_AUX>(acc, A.partials + tile, A.prow, red);
        if (t == 0) {
            A.partials[tile + (int64_t)T_AUX * A.prow] = 0.0;
            A.partials[tile + (int64_t)T_SURN * A.prow] = 0.0;
        }
    }
    // first stage of the books of this pass: the element terms of the
    // previous pass over a contiguous range of its tiles
    const int nblk = A.tiles_x * A.tiles_y, ns = books_stage_rows(nblk);
    if (A.contact && tile < ns) {
        const int lo = (int)((int64_t)nblk * tile / ns), hi = (int)((int64_t)nblk * (tile + 1) / ns);
        double q[T_FC];
#pragma unroll
        for (int k = 0; k < T_FC; ++k) q[k] = 0.0;
        for (int b = lo + t; b < hi; b += NT) {
#pragma unroll
            for (int k = 0; k < T_FC; ++k) q[k] += A.partials_prev[(int64_t)k * A.prow + b];
        }
        __syncthreads();                    // red is reused
        block_reduce_store<NT, T_FC>(q, A.stage + tile * PDN_NTERMS, 1, red);
    }
}

// The surrogate build is held to 2 waves per SIMD (256 registers): left
// alone, the network code takes 430 VGPRs and AGPRs and the whole kernel
// runs at 1 wave per SIMD even where no point reaches the network.  The
// spills this costs sit around the network evaluation; the plain build
// (bound 1, the default) is unaffected.  The FP32 build with full
// integration and plasticity is held to 2 waves as well: it needs one
// register more than 256.
template <typename R, int TX, int TY, bool SUR, int NGP = 1, bool PLAS = false>
__global__ __launch_bounds__(PDN_TILE_THREADS(TX, TY))
__attribute__((amdgpu_waves_per_eu((SUR || (PLAS && NGP == 8 && sizeof(R) == 4)) ? 2 : 1)))
void k_elem_node(ElemArgs<R> A)
{
    elem_node_tile<R, TX, TY, SUR, NGP, PLAS>(A, xcd_tile(blockIdx.x, gridDim.x));
}

// The surrogate build without the 2-waves bound (about 430 VGPRs and AGPRs,
// 1 wave per SIMD, no spills): faster where most points reach the network,
// slower where few do (the march then runs at half the occupancy).
template <typename R, int TX, int TY>
__global__ __launch_bounds__(PDN_TILE_THREADS(TX, TY)) __attribute__((amdgpu_waves_per_eu(1)))
void k_elem_node_sur_wide(ElemArgs<R> A)
{
    elem_node_tile<R, TX, TY, true, 1, false>(A, xcd_tile(blockIdx.x, gridDim.x));
}

// many plates in one launch: case c has start[c+1] - start[c] tiles.  After
// the ncase + 1 offsets, the table holds for each block (after the XCD remap)
// its case and its tile within the case (gridDim.x entries each), in the
// order the host chose: one lookup per block.
template <typename R, int TX, int TY, bool SUR, int NGP = 1>
__global__ __launch_bounds__(PDN_TILE_THREADS(TX, TY)) __attribute__((amdgpu_waves_per_eu(SUR ? 2 : 1)))
void k_elem_node_batch(const ElemArgs<R> *__restrict__ args, const int *__restrict__ start, int ncase)
{
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int *bcase = start + ncase + 1, *btile = bcase + gridDim.x;
    const ElemArgs<R> A = args[bcase[b]];
    elem_node_tile<R, TX, TY, SUR, NGP>(A, btile[b]);
}

#define PDN_BOOKS_THREADS 256
template <typename R>
__global__ __launch_bounds__(PDN_BOOKS_THREADS) void k_books(ElemArgs<R> A)
{
    __shared__ double red[PDN_NTERMS * (PDN_BOOKS_THREADS / 64)];
    contact_books<PDN_BOOKS_THREADS>(A, red);
}

// one workgroup per case
template <typename R>
__global__ __launch_bounds__(PDN_BOOKS_THREADS) void k_books_batch(const ElemArgs<R> *__restrict__ args)
{
    __shared__ double red[PDN_NTERMS * (PDN_BOOKS_THREADS / 64)];
    const ElemArgs<R> A = args[blockIdx.x];
    contact_books<PDN_BOOKS_THREADS>(A, red);
}

// ---------------------------------------------------------------------------
// launchers of one variant
// ---------------------------------------------------------------------------
template <typename R, int TX, int TY, bool SUR, int NGP = 1, bool PLAS = false>
static hipError_t launch_en(const ElemArgs<R> &a, hipStream_t s)
{
    const int nb = a.tiles_x * a.tiles_y;
    hipLaunchKernelGGL((k_elem_node<R, TX, TY, SUR, NGP, PLAS>), dim3(nb), dim3(PDN_TILE_THREADS(TX, TY)), 0, s, a);
    return hipGetLastError();
}

template <typename R, bool SUR>
static hipError_t launch_elem_node_v(const ElemArgs<R> &a, int tile, hipStream_t s)
{
    switch (tile) {
    case PDN_TILE_16x16: return launch_en<R, 16, 16, SUR>(a, s);
    case PDN_TILE_32x8: return launch_en<R, 32, 8, SUR>(a, s);
    case PDN_TILE_8x8: return launch_en<R, 8, 8, SUR>(a, s);
    case PDN_TILE_15x15: return launch_en<R, 15, 15, SUR>(a, s);
    case PDN_TILE_31x15: return launch_en<R, 31, 15, SUR>(a, s);
    default: return hipErrorInvalidValue;
    }
}

// the surrogate build at 1 wave per SIMD: built for the 15x15 tile (a
// workgroup of 16x16 node columns is four waves, one per SIMD; the larger
// tiles' workgroups put two waves on a SIMD)
template <typename R>
static hipError_t launch_elem_node_sur_wide_v(const ElemArgs<R> &a, int tile, hipStream_t s)
{
    const int nb = a.tiles_x * a.tiles_y;
    switch (tile) {
    case PDN_TILE_15x15:
        hipLaunchKernelGGL((k_elem_node_sur_wide<R, 15, 15>), dim3(nb), dim3(PDN_TILE_THREADS(15, 15)), 0, s, a);
        return hipGetLastError();
    default: return hipErrorInvalidValue;
    }
}

template <typename R, int TX, int TY, bool SUR, int NGP = 1>
static int lds_of()
{
    hipFuncAttributes at;
    if (hipFuncGetAttributes(&at, reinterpret_cast<const void *>(&k_elem_node<R, TX, TY, SUR, NGP>)) != hipSuccess)
        return -1;
    return (int)at.sharedSizeBytes;
}

template <typename R, bool SUR>
static int lds_v(int tile)
{
    switch (tile) {
    case PDN_TILE_16x16: return lds_of<R, 16, 16, SUR>();
    case PDN_TILE_32x8: return lds_of<R, 32, 8, SUR>();
    case PDN_TILE_8x8: return lds_of<R, 8, 8, SUR>();
    case PDN_TILE_15x15: return lds_of<R, 15, 15, SUR>();
    case PDN_TILE_31x15: return lds_of<R, 31, 15, SUR>();
    default: return -1;
    }
}

template <typename R, int TX, int TY, bool SUR, int NGP = 1>
static hipError_t launch_enb(const ElemArgs<R> *args, const int *start, int ncase, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_elem_node_batch<R, TX, TY, SUR, NGP>), dim3(nblocks), dim3(PDN_TILE_THREADS(TX, TY)), 0, s,
                       args, start, ncase);
    return hipGetLastError();
}

template <typename R, bool SUR>
static hipError_t launch_elem_node_batch_v(const ElemArgs<R> *args, const int *start, int ncase, int nblocks,
                                           int tile, hipStream_t s)
{
    if (ncase < 1 || nblocks < 1) return hipErrorInvalidValue;
    switch (tile) {
    case PDN_TILE_16x16: return launch_enb<R, 16, 16, SUR>(args, start, ncase, nblocks, s);
    case PDN_TILE_32x8: return launch_enb<R, 32, 8, SUR>(args, start, ncase, nblocks, s);
    case PDN_TILE_8x8: return launch_enb<R, 8, 8, SUR>(args, start, ncase, nblocks, s);
    case PDN_TILE_15x15: return launch_enb<R, 15, 15, SUR>(args, start, ncase, nblocks, s);
    case PDN_TILE_31x15: return launch_enb<R, 31, 15, SUR>(args, start, ncase, nblocks, s);
    default: return hipErrorInvalidValue;
    }
}

// shear plasticity (one point): the tiles it is built for
template <typename R>
static hipError_t launch_elem_node_plas_v(const ElemArgs<R> &a, int tile, hipStream_t s)
{
    switch (tile) {
    case PDN_TILE_16x16: return launch_en<R, 16, 16, false, 1, true>(a, s);
    case PDN_TILE_15x15: return launch_en<R, 15, 15, false, 1, true>(a, s);
    case PDN_TILE_8x8: return launch_en<R, 8, 8, false, 1, true>(a, s);
    default: return hipErrorInvalidValue;
    }
}

// full integration (PLAS: with shear plasticity): the tiles it is built for
template <typename R, bool PLAS = false>
static hipError_t launch_elem_node_full_v(const ElemArgs<R> &a, int tile, hipStream_t s)
{
    switch (tile) {
    case PDN_TILE_16x16: return launch_en<R, 16, 16, false, 8, PLAS>(a, s);
    case PDN_TILE_15x15: return launch_en<R, 15, 15, false, 8, PLAS>(a, s);
    default: return hipErrorInvalidValue;
    }
}

template <typename R>
static hipError_t launch_elem_node_batch_full_v(const ElemArgs<R> *args, const int *start, int ncase, int nblocks,
                                                int tile, hipStream_t s)
{
    if (ncase < 1 || nblocks < 1) return hipErrorInvalidValue;
    switch (tile) {
    case PDN_TILE_16x16: return launch_enb<R, 16, 16, false, 8>(args, start, ncase, nblocks, s);
    case PDN_TILE_15x15: return launch_enb<R, 15, 15, false, 8>(args, start, ncase, nblocks, s);
    default: return hipErrorInvalidValue;
    }
}

}  // namespace pdn
