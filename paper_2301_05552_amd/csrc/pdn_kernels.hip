// pdn_kernels.hip -- gfx950 kernels of the explicit PDN impact step.
//
//  k_elem_node : element internal force + damage update, nodal assembly,
//                lumped-mass integration and the next predictor, fused.  One
//                workgroup owns an in-plane tile of element columns and marches
//                through every node plane of the plate (bottom to top); node
//                planes are staged in LDS, element corner forces are summed per
//                node in a fixed order (deterministic), tiles overlap by one
//                element column (owner-computes: rim elements are evaluated by
//                both neighbours, state is written by one).
//  k_contact   : PDN contact step (Algorithms 1-2): striker update, detection,
//                projection, reaction, node release with the repeat flag, one
//                thread per candidate node; the last workgroup to finish sums
//                the reaction and the energy books in a fixed order.
//  k_damage_*  : damage-field outputs.
#include "pdn_internal.h"
#include "pdn_launch.h"

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

// eps: material-frame Green strain (Voigt 11,22,33,23,13,12, engineering shear)
// r: thresholds r1+, r1-, r2+, r2- (in/out).  Returns nominal PK2 stress.
template <typename R>
__device__ void cdm_update(const PlyC<R> &P, R vol, const R e[6], R r[4], R sg[6], bool &changed)
{
    R s0 = P.C11 * e[0] + P.C12 * e[1] + P.C13 * e[2];
    R s1 = P.C12 * e[0] + P.C22 * e[1] + P.C23 * e[2];
    R s2 = P.C13 * e[0] + P.C23 * e[1] + P.C33 * e[2];
    R s3 = P.G23 * e[3], s4 = P.G13 * e[4], s5 = P.G12 * e[5];
    changed = false;
    if (P.law == 0) {
        sg[0] = s0; sg[1] = s1; sg[2] = s2; sg[3] = s3; sg[4] = s4; sg[5] = s5;
        return;
    }
    if (vol <= P.vol_nocap) {
        // Screen: upper bounds of the loading functions without roots or
        // divisions.  When none can exceed its threshold the thresholds keep
        // their values, exactly as the full evaluation below would leave them.
        const R t2 = s5 * s5 + s4 * s4;                  // tau_L^2
        bool grow = rmax(e[0], R(0)) * P.kE1XT > r[0] || rmax(-e[0], R(0)) * P.kE1XC > r[1];
        if (s1 >= R(0)) {
            const R a = s1 * P.iYT;
            grow |= a * a + t2 * P.iSL * P.iSL > r[2] * r[2];
        } else {
            const R el = P.etaL0 * s1;                   // eta_L sigma22
            const R qL = el > R(0) ? R(2) * (t2 + el * el) : t2;
            grow |= qL * P.iSL * P.iSL > r[2] * r[2];
            const R bT = -s1 * P.kT * P.iST;
            const R elc = el * P.ca0;
            const R qL2 = R(2) * P.ca0 * P.ca0 * (t2 + elc * elc);
            grow |= bT * bT + qL2 * P.iSL * P.iSL > r[3] * r[3];
        }
        if (!grow) {
            if (r[0] <= R(1) && r[1] <= R(1) && r[2] <= R(1) && r[3] <= R(1)) {
                sg[0] = s0; sg[1] = s1; sg[2] = s2; sg[3] = s3; sg[4] = s4; sg[5] = s5;
                return;
            }
        }
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
        return;
    }
    R d1p = damage_bilinear(r0, P.XT, P.E1, P.GXT, P.fXT, P.fGT, lc);
    R d1m = damage_bilinear(r1, P.XC, P.E1, P.GXC, P.fXC, P.fGC, lc);
    R d2p = damage_exp(r2, YT, P.E2, P.GYT, lc);
    R d2m = damage_exp(r3, YC, P.E2, P.GYC, lc);
    R d6 = damage_exp(r2, SL, P.G12v, P.GSL, lc);
    R d1 = s0 >= R(0) ? d1p : d1m;
    R d2 = s1 >= R(0) ? d2p : d2m;
    // nominal stress: inverse of the damaged compliance (normal block by cofactors)
    R h00 = P.iE1 / (R(1) - d1), h11 = P.iE2 / (R(1) - d2), h22 = P.iE3;
    R h01 = P.mn12, h02 = P.mn13, h12 = P.mn23;
    R c00 = h11 * h22 - h12 * h12, c01 = h02 * h12 - h01 * h22, c02 = h01 * h12 - h02 * h11;
    R c11 = h00 * h22 - h02 * h02, c12 = h01 * h02 - h00 * h12, c22 = h00 * h11 - h01 * h01;
    R inv = R(1) / (h00 * c00 + h01 * c01 + h02 * c02);
    sg[0] = (c00 * e[0] + c01 * e[1] + c02 * e[2]) * inv;
    sg[1] = (c01 * e[0] + c11 * e[1] + c12 * e[2]) * inv;
    sg[2] = (c02 * e[0] + c12 * e[1] + c22 * e[2]) * inv;
    sg[3] = (R(1) - d2) * P.G23 * e[3];
    sg[4] = (R(1) - d6) * P.G13 * e[4];
    sg[5] = (R(1) - d6) * P.G12 * e[5];
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

// Returns the force coefficients on the corner basis (forces = inv8 of each).
template <typename R>
__device__ void hex_box_force(const R ux[8], const R uy[8], const R uz[8], R hx, R hy, R hz,
                              R ihx, R ihy, R ihz, const PlyC<R> &P, R kappa, R r[4], bool &changed,
                              Modes<R> &cx, Modes<R> &cy, Modes<R> &cz, R &uel)
{
    Modes<R> sx = fwd8(ux), sy = fwd8(uy), sz = fwd8(uz);
    const R gx = R(0.25) * ihx, gy = R(0.25) * ihy, gz = R(0.25) * ihz;
    // displacement gradient G = F - I
    R G00 = sx.xi * gx, G01 = sx.eta * gy, G02 = sx.zeta * gz;
    R G10 = sy.xi * gx, G11 = sy.eta * gy, G12 = sy.zeta * gz;
    R G20 = sz.xi * gx, G21 = sz.eta * gy, G22 = sz.zeta * gz;
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
    const R vol = hx * hy * hz;
    cdm_update(P, vol, e, r, sg, changed);
    // back to the global frame
    R S00 = cc * sg[0] - R(2) * cs * sg[5] + ss * sg[1];
    R S11 = ss * sg[0] + R(2) * cs * sg[5] + cc * sg[1];
    R S22 = sg[2];
    R S01 = cs * sg[0] + (cc - ss) * sg[5] - cs * sg[1];
    R S02 = c * sg[4] - s * sg[3];
    R S12 = s * sg[4] + c * sg[3];
    // nominal stress P = F S (index form (F S)_{iJ})
    R F00 = R(1) + G00, F11 = R(1) + G11, F22 = R(1) + G22;
    R P00 = F00 * S00 + G01 * S01 + G02 * S02;
    R P01 = F00 * S01 + G01 * S11 + G02 * S12;
    R P02 = F00 * S02 + G01 * S12 + G02 * S22;
    R P10 = G10 * S00 + F11 * S01 + G12 * S02;
    R P11 = G10 * S01 + F11 * S11 + G12 * S12;
    R P12 = G10 * S02 + F11 * S12 + G12 * S22;
    R P20 = G20 * S00 + G21 * S01 + F22 * S02;
    R P21 = G20 * S01 + G21 * S11 + F22 * S12;
    R P22 = G20 * S02 + G21 * S12 + F22 * S22;
    const R ax = R(0.25) * hy * hz, ay = R(0.25) * hx * hz, az = R(0.25) * hx * hy;
    // hourglass: k = kappa Cmax V sum b^2 / 3, q = s/8, force coefficient k s / 64
    const R khg = kappa * P.cmax * vol * (ihx * ihx + ihy * ihy + ihz * ihz) * R(1.0 / 6.0);
    const R kh = khg * R(1.0 / 64.0);
    cx.xi = P00 * ax; cx.eta = P01 * ay; cx.zeta = P02 * az;
    cy.xi = P10 * ax; cy.eta = P11 * ay; cy.zeta = P12 * az;
    cz.xi = P20 * ax; cz.eta = P21 * ay; cz.zeta = P22 * az;
    cx.ez = kh * sx.ez; cx.xz = kh * sx.xz; cx.xe = kh * sx.xe; cx.xez = kh * sx.xez;
    cy.ez = kh * sy.ez; cy.xz = kh * sy.xz; cy.xe = kh * sy.xe; cy.xez = kh * sy.xez;
    cz.ez = kh * sz.ez; cz.xz = kh * sz.xz; cz.xe = kh * sz.xe; cz.xez = kh * sz.xez;
    R w = sg[0] * e[0] + sg[1] * e[1] + sg[2] * e[2] + sg[3] * e[3] + sg[4] * e[4] + sg[5] * e[5];
    R q2 = sx.ez * sx.ez + sx.xz * sx.xz + sx.xe * sx.xe + sx.xez * sx.xez
         + sy.ez * sy.ez + sy.xz * sy.xz + sy.xe * sy.xe + sy.xez * sy.xez
         + sz.ez * sz.ez + sz.xz * sz.xz + sz.xe * sz.xe + sz.xez * sz.xez;
    uel = R(0.5) * vol * w + R(0.5) * khg * q2 * R(1.0 / 64.0);
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

template <int NT>
__device__ void block_reduce_store(double acc[PDN_NTERMS], double *out, double *sh)
{
    // deterministic: fixed shuffle tree inside each wave, waves summed in order
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    constexpr int NW = NT / 64;
#pragma unroll
    for (int k = 0; k < PDN_NTERMS; ++k) {
        double v = acc[k];
        for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
        if (lane == 0) sh[k * NW + wave] = v;
    }
    __syncthreads();
    if (threadIdx.x < PDN_NTERMS) {
        double v = 0;
        for (int w = 0; w < NW; ++w) v += sh[threadIdx.x * NW + w];
        out[threadIdx.x] = v;
    }
}

// one workgroup's tile of one plate; block partials go to A.partials[tile]
template <typename R, int TX, int TY>
__device__ __forceinline__ void elem_node_tile(const ElemArgs<R> &A, const int tile)
{
    constexpr int NE = TX * TY, NCX = TX + 1, NCY = TY + 1, NC = NCX * NCY;
    constexpr int NT = PDN_TILE_THREADS(TX, TY);
    constexpr bool F32 = sizeof(R) == 4;
    __shared__ R Ubuf[F32 ? 2 : 1][3][F32 ? NC : 1];   // node planes k-1, k in FP32
    __shared__ R Fs[2][4][3][NE];           // element corner forces: [bottom/top][corner][xyz]
    __shared__ double D64[2][3][NC];        // FP64 displacement of planes k-1, k
    __shared__ double V64[2][3][NC];        // FP64 velocity of planes k-1, k (own slot)
    __shared__ double red[PDN_NTERMS * (NT / 64)];
    // element-type plane copy: the FP64 staging itself when R is double
    R (*U)[3][NC] = F32 ? reinterpret_cast<R (*)[3][NC]>(&Ubuf[0][0][0])
                        : reinterpret_cast<R (*)[3][NC]>(&D64[0][0][0]);

    const int t = threadIdx.x;
    const int tx = tile % A.tiles_x, ty = tile / A.tiles_x;
    const int e0x = tx * (TX - 1), e0y = ty * (TY - 1);
    const bool lastx = tx == A.tiles_x - 1, lasty = ty == A.tiles_y - 1;
    const int nx = A.nx, ny = A.ny;
    const int64_t plane = (int64_t)(nx + 1) * (ny + 1);

    // element role: one element column per thread
    const bool erole = t < NE;
    const int ea = t % TX, eb = t / TX;
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

    double carry[3] = {0, 0, 0}, fin[3];
    double acc[PDN_NTERMS];
#pragma unroll
    for (int k = 0; k < PDN_NTERMS; ++k) acc[k] = 0.0;

    // node plane k is fetched from HBM one iteration ahead (kept in registers
    // while the previous layer is computed), then staged in LDS
    double pd[3] = {0, 0, 0}, pv[3] = {0, 0, 0};
    auto fetch_plane = [&](int k) {
        if (nvalid) {
            const int64_t nk = col + plane * k;
#pragma unroll
            for (int c = 0; c < 3; ++c) pd[c] = A.d_in[3 * nk + c];
            if (nown) {
#pragma unroll
                for (int c = 0; c < 3; ++c) pv[c] = A.v_in[3 * nk + c];
            }
        }
    };
    auto stage_plane = [&](int k) {
        const int p = k & 1;
        if (nvalid) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                D64[p][c][t] = pd[c];
                if (F32) U[p][c][t] = (R)pd[c];
            }
            if (nown) {
#pragma unroll
                for (int c = 0; c < 3; ++c) V64[p][c][t] = pv[c];
            }
        } else if (nrole) {
            U[p][0][t] = U[p][1][t] = U[p][2][t] = R(0);
        }
    };
    // damage thresholds of the element in layer l, fetched one layer ahead
    R rn[4] = {R(1), R(1), R(1), R(1)};
    auto fetch_r = [&](int l) {
        if (l < A.NL && evalid) {
            const LayerInfo L = A.layers[l];
            if (L.type == 0 && A.ply[L.ply].law != 0)
                load_state(A.r, ie + (int64_t)nx * (je + (int64_t)ny * L.index), rn);
        }
    };

    // lumped-mass integration of plane kp with total internal force f; next predictor
    auto update_node = [&](int kp, const double f[3]) {
        const int p = kp & 1;
        const int64_t n = col + plane * kp;
        const int fix_lat = (A.clamp_lateral && (gi == 0 || gi == nx || gj == 0 || gj == ny)) ? 7 : 0;
        const int bits = fix_lat | (kp == 0 ? (int)A.bc_bottom[col] : 0);
        const double m = A.mx[gi] * A.my[gj] * A.mz[kp];
        const double im = A.imx[gi] * A.imy[gj] * A.imz[kp];
        const double dt = A.dt, g = A.grav;
        acc[T_MZ] += m * D64[p][2][t];         // gravity work = -g (sum m d_z - its initial value)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const double d = D64[p][c][t], v = V64[p][c][t];
            const bool fx = (bits >> c) & 1;
            const double fe = c == 2 ? -m * g : 0.0;
            const double a = fx ? 0.0 : (fe - f[c]) * im;
            const double vn = fx ? 0.0 : v + dt * a;
            const double dn = fx ? d : d + dt * v + A.phi * dt * dt * a;
            acc[T_KE] += 0.5 * m * v * vn;
            acc[T_WA] += 0.5 * dt * v * f[c];
            acc[T_WB] += 0.5 * dt * vn * f[c];
            A.d_out[3 * n + c] = dn;
            A.v_out[3 * n + c] = vn;
        }
        if (kp == A.K - 1 && gi >= A.ci0 && gi < A.ci1 && gj >= A.cj0 && gj < A.cj1) {
            const int64_t ci = (gi - A.ci0) + (int64_t)(A.ci1 - A.ci0) * (gj - A.cj0);
            A.fside[3 * ci + 0] = f[0];
            A.fside[3 * ci + 1] = f[1];
            A.fside[3 * ci + 2] = f[2];
        }
    };

    fetch_plane(0);
    stage_plane(0);
    fetch_plane(1);
    fetch_r(0);
    for (int k = 1; k < A.K; ++k) {
        const LayerInfo L = A.layers[k - 1];
        stage_plane(k);
        R r[4] = {rn[0], rn[1], rn[2], rn[3]};
        if (k + 1 < A.K) fetch_plane(k + 1);
        fetch_r(k);
        if (L.type == 0) {
            __syncthreads();
            if (erole) {
                R* F0 = &Fs[0][0][0][t];
                if (evalid) {
                    const int kb = (k - 1) & 1, kt = k & 1;
                    const int sl[4] = {s0, s0 + 1, s0 + 1 + NCX, s0 + NCX};
                    R ux[8], uy[8], uz[8];
#pragma unroll
                    for (int q = 0; q < 4; ++q) {
                        ux[q] = U[kb][0][sl[q]]; uy[q] = U[kb][1][sl[q]]; uz[q] = U[kb][2][sl[q]];
                        ux[q + 4] = U[kt][0][sl[q]]; uy[q + 4] = U[kt][1][sl[q]]; uz[q + 4] = U[kt][2][sl[q]];
                    }
                    const PlyC<R> &P = A.ply[L.ply];
                    const int64_t e = ie + (int64_t)nx * (je + (int64_t)ny * L.index);
                    bool changed = false;
                    R uel;
                    Modes<R> cm[3];
                    hex_box_force(ux, uy, uz, A.hx[ie], A.hy[je], (R)L.hz, A.ihx[ie], A.ihy[je], (R)L.ihz, P,
                                  A.kappa, r, changed, cm[0], cm[1], cm[2], uel);
                    if (eown) {
                        if (changed) store_state(A.r, e, r);
                        acc[T_UEL] += (double)uel;
                    }
#pragma unroll
                    for (int c = 0; c < 3; ++c) {
                        R f[8];
                        inv8(cm[c], f);
#pragma unroll
                        for (int q = 0; q < 4; ++q) {
                            F0[(q * 3 + c) * NE] = f[q];                    // bottom corners
                            F0[((4 + q) * 3 + c) * NE] = f[q + 4];          // top corners
                        }
                    }
                } else {
#pragma unroll
                    for (int q = 0; q < 24; ++q) F0[q * NE] = R(0);
                }
            }
            __syncthreads();
            if (nown) {
                // node (np, nq) is corner 0 of element (np, nq), 1 of (np-1, nq),
                // 2 of (np-1, nq-1) and 3 of (np, nq-1); the four corner forces of
                // one layer are summed in the element type, in this order
                R fb[3] = {R(0), R(0), R(0)}, ft[3] = {R(0), R(0), R(0)};
                if (np < TX && nq < TY) {
                    const int e = np + TX * nq;
#pragma unroll
                    for (int c = 0; c < 3; ++c) { fb[c] += Fs[0][0][c][e]; ft[c] += Fs[1][0][c][e]; }
                }
                if (np >= 1 && nq < TY) {
                    const int e = np - 1 + TX * nq;
#pragma unroll
                    for (int c = 0; c < 3; ++c) { fb[c] += Fs[0][1][c][e]; ft[c] += Fs[1][1][c][e]; }
                }
                if (np >= 1 && nq >= 1) {
                    const int e = np - 1 + TX * (nq - 1);
#pragma unroll
                    for (int c = 0; c < 3; ++c) { fb[c] += Fs[0][2][c][e]; ft[c] += Fs[1][2][c][e]; }
                }
                if (np < TX && nq >= 1) {
                    const int e = np + TX * (nq - 1);
#pragma unroll
                    for (int c = 0; c < 3; ++c) { fb[c] += Fs[0][3][c][e]; ft[c] += Fs[1][3][c][e]; }
                }
#pragma unroll
                for (int c = 0; c < 3; ++c) { fin[c] = carry[c] + (double)fb[c]; carry[c] = (double)ft[c]; }
            }
        } else if (nown) {
            // zero-thickness interface, nodal (Newton-Cotes) points: the points of
            // the four elements sharing a node pair coincide, so the pair carries
            // one state and the summed tributary area
            const PlyC<R> &P = A.ply[L.ply];
            const int64_t pi = col + plane * L.index;
            const int pb = (k - 1) & 1, pt = k & 1;
            R rd = A.rd[pi];
            R tau[3];
            bool changed;
            const R d1 = (R)(D64[pt][0][t] - D64[pb][0][t]);
            const R d2 = (R)(D64[pt][1][t] - D64[pb][1][t]);
            const R d3 = (R)(D64[pt][2][t] - D64[pb][2][t]);
            czm_update(P, d1, d2, d3, rd, tau, changed);
            if (changed) A.rd[pi] = rd;
            const double ap = A.mx[gi] * A.my[gj];   // (sum of adjacent widths / 2)(... / 2)
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const double ftc = ap * (double)tau[c];
                fin[c] = carry[c] - ftc;
                carry[c] = ftc;
            }
            acc[T_UEL] += 0.5 * ap * (double)(tau[0] * d1 + tau[1] * d2 + tau[2] * d3);
        }
        if (nown) update_node(k - 1, fin);
    }
    if (nown) update_node(A.K - 1, carry);
    block_reduce_store<NT>(acc, A.partials + (int64_t)tile * PDN_NTERMS, red);
}

template <typename R, int TX, int TY>
__global__ __launch_bounds__(PDN_TILE_THREADS(TX, TY))
void k_elem_node(ElemArgs<R> A)
{
    elem_node_tile<R, TX, TY>(A, xcd_tile(blockIdx.x, gridDim.x));
}

// case of global block b in a batch: the last c with start[c] <= b
__device__ __forceinline__ int batch_case(const int *start, int ncase, int b)
{
    int lo = 0, hi = ncase - 1;
    while (lo < hi) {
        const int mid = (lo + hi + 1) >> 1;
        if (start[mid] <= b) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

// many plates in one launch: tiles of case c are blocks start[c] .. start[c+1)-1
// (after the XCD remap, so that one case's neighbouring tiles share an L2)
template <typename R, int TX, int TY>
__global__ __launch_bounds__(PDN_TILE_THREADS(TX, TY))
void k_elem_node_batch(const ElemArgs<R> *__restrict__ args, const int *__restrict__ start, int ncase)
{
    const int b = xcd_tile(blockIdx.x, gridDim.x);
    const int c = batch_case(start, ncase, b);
    const ElemArgs<R> A = args[c];
    elem_node_tile<R, TX, TY>(A, b - start[c]);
}

// ---------------------------------------------------------------------------
// contact kernel: one thread per candidate node, many workgroups; the last
// workgroup to finish reduces the per-workgroup results in a fixed order
// ---------------------------------------------------------------------------

template <int NT>
__device__ double blk_sum(double v, double *sh)
{
    // deterministic sum over the workgroup; result valid in thread 0
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    __syncthreads();
    if (lane == 0) sh[wave] = v;
    __syncthreads();
    double s = 0;
    if (threadIdx.x == 0)
        for (int w = 0; w < NT / 64; ++w) s += sh[w];
    return s;
}

// workgroup blk of the nblk workgroups that serve one plate
__device__ __forceinline__ void contact_block(const ContactArgs &C, const int blk, const int nblk)
{
    constexpr int NT = PDN_K1_THREADS;
    __shared__ double sh[NT / 64];
    __shared__ double row[PDN_CQ];
    __shared__ int am_last;
    DevGlobals *G = C.gl;
    const int t = threadIdx.x;
    const double dt = G->dt, phi = G->phi, R = G->R, g = G->g, ms = G->ms;

    // rigid body first (Gauss-Seidel): every workgroup advances the striker with
    // the force frozen from the plate's last step (identical arithmetic); only
    // the last workgroup stores it
    const double Fz = G->Fprev[2];
    const double az = -g - Fz / ms;                   // lateral striker motion constrained
    const double cz_old = G->c[2], Vz_old = G->V[2];
    const double cx = G->c[0], cy = G->c[1];
    const double cz = cz_old + dt * Vz_old + 0.5 * dt * dt * az;

    const int cw = C.ci1 - C.ci0, ch = C.cj1 - C.cj0, nc = cw * ch;
    const int64_t plane = (int64_t)(C.nx + 1) * (C.ny + 1);
    const int j = blk * NT + t;
    double q[PDN_CQ];
    for (int k = 0; k < PDN_CQ; ++k) q[k] = 0.0;
    // slots 0..7: element-kernel partials of the previous level (strided rows)
    for (int b = j; b < C.nblocks; b += nblk * NT)
        for (int k = 0; k < PDN_NTERMS; ++k) q[k] += C.partials[(int64_t)b * PDN_NTERMS + k];
    if (j < nc) {
        const int i = C.ci0 + j % cw, jj = C.cj0 + j / cw;
        const int64_t n = i + (int64_t)(C.nx + 1) * jj + plane * (C.K - 1);
        const bool lat = C.clamp_lateral && (i == 0 || i == C.nx || jj == 0 || jj == C.ny);
        const double m = C.mx[i] * C.my[jj] * C.mztop;
        double dd[3] = {C.d[3 * n], C.d[3 * n + 1], C.d[3 * n + 2]};
        const double rx = C.xs[i] + dd[0] - cx, ry = C.ys[jj] + dd[1] - cy, rz = C.ztop + dd[2] - cz;
        const double dist = sqrt(rx * rx + ry * ry + rz * rz);
        const double gap = dist - R;
        double nv[3] = {0.0, 0.0, -1.0};
        if (dist > 0.0) { nv[0] = rx / dist; nv[1] = ry / dist; nv[2] = rz / dist; }
        // detection on the predictor; Dirichlet projection; release of adhesion
        // nodes (Eq. 2) with step repetition.  The reaction of a node depends on
        // that node only, so the repeated pass re-evaluates it locally.
        bool act = C.active[j] != 0 || (gap < 0.0 && rz <= 0.0);
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
        C.active[j] = act ? 1 : 0;
        double dv[3] = {0, 0, 0};
        if (act) {
            for (int c = 0; c < 3; ++c) {
                const double da = fc[c] / m;
                dv[c] = dt * da;
                C.d[3 * n + c] = dd[c] + phi * dt * dt * da;
                C.v[3 * n + c] += dv[c];
            }
            q[15] += 1.0;                                         // active
            const bool ring = (i == C.ci0 && i > 0) || (i == C.ci1 - 1 && i < C.nx) ||
                              (jj == C.cj0 && jj > 0) || (jj == C.cj1 - 1 && jj < C.ny);
            if (ring) q[16] += 1.0;                               // left the search window
        }
        q[17] += (double)released;
        for (int c = 0; c < 3; ++c) {
            const double vpv = C.vprev[3 * j + c];
            q[8 + c] += fc[c];                                    // reaction sum
            q[11] += 0.5 * m * vpv * dv[c];                       // kinetic-energy correction
            q[12] += 0.5 * dt * dv[c] * C.fside[3 * j + c];       // internal-work correction
            q[14] += 0.5 * dt * vpv * (C.fcprev[3 * j + c] + fc[c]);   // contact work on the plate
            C.vprev[3 * j + c] = C.v[3 * n + c];
            C.fcprev[3 * j + c] = fc[c];
        }
    }
    for (int k = 0; k < PDN_CQ; ++k) {
        const double s = blk_sum<NT>(q[k], sh);
        if (t == 0) row[k] = s;
    }
    __syncthreads();
    if (t < PDN_CQ) C.blk[(int64_t)blk * PDN_CQ + t] = row[t];
    __threadfence();
    __syncthreads();
    if (t == 0) {
        const unsigned tk = atomicAdd(&G->ticket, 1u);
        am_last = tk == (unsigned)nblk - 1;
    }
    __syncthreads();
    if (!am_last) return;
    __threadfence();
    if (t < PDN_CQ) {
        double s = 0;
        for (int b = 0; b < nblk; ++b) s += __builtin_nontemporal_load(&C.blk[(int64_t)b * PDN_CQ + t]);
        row[t] = s;
    }
    __syncthreads();
    if (t == 0) {
        const double *P = row;                                    // 0..7 partials, 8.. contact
        const double kes_level = 0.5 * ms * (G->V[0] * G->V[0] + G->V[1] * G->V[1] + G->V[2] * G->V[2]);
        // books of level s (= completed steps), final now
        if (!G->first) {
            G->e_wint += G->half_int + P[T_WA];
            G->e_wc += P[14];
        } else {
            G->mz0 = P[T_MZ];
        }
        // gravity is constant: its work is -g (sum m d_z - initial), the
        // trapezoidal sum telescoped (phi = 1)
        G->e_wgp = -g * (P[T_MZ] - G->mz0);
        G->half_int = P[T_WB] + P[12];
        G->e_kep = P[T_KE] + P[11];
        G->e_uel = P[T_UEL];
        G->e_kes = kes_level;
        G->e_ws = G->ws_acc;
        G->e_wgs = G->wgs_acc;
        G->e_level = (double)G->step;
        G->fallback_gp += P[T_AUX];
        // a non-finite displacement or velocity propagates into these sums
        if (!(isfinite(P[T_KE]) && isfinite(P[T_WA]) && isfinite(P[T_WB]) && isfinite(P[T_MZ])))
            G->flag_unstable = 1;
        if (P[16] > 0.0) G->flag_overflow = 1;
        // striker update and its works (force frozen over the step)
        const double dz = cz - cz_old;
        G->ws_acc += Fz * dz;
        G->wgs_acc += ms * g * (-dz);
        G->c[2] = cz;
        G->V[2] = Vz_old + dt * az;
        G->Fprev[0] = P[8]; G->Fprev[1] = P[9]; G->Fprev[2] = P[10];
        const int passes = P[17] > 0.0 ? 2 : 1;
        G->reset_passes += passes;
        G->released += (int64_t)P[17];
        if (passes > G->max_passes) G->max_passes = passes;
        G->active = (int64_t)P[15];
        if (G->step < G->hist_cap) {
            C.hist[3 * G->step + 0] = (double)(G->step + 1) * dt;
            C.hist[3 * G->step + 1] = -P[10];
            C.hist[3 * G->step + 2] = -(cz - G->c0[2]);
        }
        G->step += 1;
        G->first = 0;
        G->ticket = 0;
    }
}

__global__ __launch_bounds__(PDN_K1_THREADS) void k_contact(ContactArgs C)
{
    contact_block(C, blockIdx.x, gridDim.x);
}

__global__ __launch_bounds__(PDN_K1_THREADS)
void k_contact_batch(const ContactArgs *__restrict__ args, const int *__restrict__ start, int ncase)
{
    const int c = batch_case(start, ncase, blockIdx.x);
    const ContactArgs C = args[c];
    contact_block(C, blockIdx.x - start[c], start[c + 1] - start[c]);
}

// candidate bookkeeping at (re)initialisation
__global__ void k_contact_init(ContactArgs C, int reset_active)
{
    const int cw = C.ci1 - C.ci0, nc = cw * (C.cj1 - C.cj0);
    const int64_t plane = (int64_t)(C.nx + 1) * (C.ny + 1);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nc; j += gridDim.x * blockDim.x) {
        const int i = C.ci0 + j % cw, jj = C.cj0 + j / cw;
        const int64_t n = i + (int64_t)(C.nx + 1) * jj + plane * (C.K - 1);
        for (int c = 0; c < 3; ++c) {
            C.vprev[3 * j + c] = C.v[3 * n + c];
            C.fcprev[3 * j + c] = 0.0;
        }
        if (reset_active) C.active[j] = 0;
    }
}

// ---------------------------------------------------------------------------
// damage fields
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_damage_bulk(const R *r, const LayerInfo *layers, const int *bulk_layer, const PlyC<R> *ply,
                              const R *hx, const R *hy, int nx, int ny, int64_t ne, int kind, double *out)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
        const int ie = (int)(e % nx), je = (int)((e / nx) % ny), lb = (int)(e / ((int64_t)nx * ny));
        const LayerInfo L = layers[bulk_layer[lb]];
        const PlyC<R> &P = ply[L.ply];
        double val = 0;
        if (P.law != 0) {
            const R lc = cbrt(hx[ie] * hy[je] * (R)L.hz);
            const R *q = r + 4 * e;
            if (kind == 0) {
                R a = damage_bilinear(q[0], P.XT, P.E1, P.GXT, P.fXT, P.fGT, lc);
                R b = damage_bilinear(q[1], P.XC, P.E1, P.GXC, P.fXC, P.fGC, lc);
                val = (double)rmax(a, b);
            } else if (kind == 1) {
                R a = damage_exp(q[2], cap_strength(P.YT, P.E2, P.GYT, lc), P.E2, P.GYT, lc);
                R b = damage_exp(q[3], cap_strength(P.YC, P.E2, P.GYC, lc), P.E2, P.GYC, lc);
                val = (double)rmax(a, b);
            } else {
                val = (double)damage_exp(q[2], cap_strength(P.SL, P.G12v, P.GSL, lc), P.G12v, P.GSL, lc);
            }
        }
        out[e] = val;
    }
}

// cohesive D per interface element: max over its 4 node pairs, at the current jump
template <typename R>
__global__ void k_damage_coh(const R *rd, const double *d, const LayerInfo *layers, const int *coh_layer,
                             const PlyC<R> *ply, int nx, int ny, int64_t nce, double *out)
{
    const int64_t plane = (int64_t)(nx + 1) * (ny + 1);
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < nce; e += (int64_t)gridDim.x * blockDim.x) {
        const int ie = (int)(e % nx), je = (int)((e / nx) % ny), ic = (int)(e / ((int64_t)nx * ny));
        const int l = coh_layer[ic];
        const PlyC<R> &P = ply[layers[l].ply];
        double mx = 0;
        for (int q = 0; q < 4; ++q) {
            const int i = ie + (q == 1 || q == 2), j = je + (q >= 2);
            const int64_t col = i + (int64_t)(nx + 1) * j;
            const int64_t nb = col + plane * l, nt = col + plane * (l + 1);
            R rr = rd[col + plane * ic], tau[3];
            bool ch;
            R D = czm_update(P, (R)(d[3 * nt] - d[3 * nb]), (R)(d[3 * nt + 1] - d[3 * nb + 1]),
                             (R)(d[3 * nt + 2] - d[3 * nb + 2]), rr, tau, ch);
            if ((double)D > mx) mx = (double)D;
        }
        out[e] = mx;
    }
}

__global__ void k_project_max(const double *in, int64_t ncol, int nlayers, double *out)
{
    for (int64_t c = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; c < ncol; c += (int64_t)gridDim.x * blockDim.x) {
        double m = 0;
        for (int l = 0; l < nlayers; ++l) m = fmax(m, in[c + ncol * l]);
        out[c] = m;
    }
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------

template <typename R, int TX, int TY>
static hipError_t launch_en(const ElemArgs<R> &a, hipStream_t s)
{
    const int nb = a.tiles_x * a.tiles_y;
    hipLaunchKernelGGL((k_elem_node<R, TX, TY>), dim3(nb), dim3(PDN_TILE_THREADS(TX, TY)), 0, s, a);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_elem_node(const ElemArgs<R> &a, int tile, hipStream_t s)
{
    switch (tile) {
    case PDN_TILE_16x16: return launch_en<R, 16, 16>(a, s);
    case PDN_TILE_32x8: return launch_en<R, 32, 8>(a, s);
    case PDN_TILE_8x8: return launch_en<R, 8, 8>(a, s);
    case PDN_TILE_15x15: return launch_en<R, 15, 15>(a, s);
    default: return hipErrorInvalidValue;
    }
}
template <typename R, int TX, int TY>
static int lds_of()
{
    hipFuncAttributes at;
    if (hipFuncGetAttributes(&at, reinterpret_cast<const void *>(&k_elem_node<R, TX, TY>)) != hipSuccess) return -1;
    return (int)at.sharedSizeBytes;
}

template <typename R>
static int lds_r(int tile)
{
    switch (tile) {
    case PDN_TILE_16x16: return lds_of<R, 16, 16>();
    case PDN_TILE_32x8: return lds_of<R, 32, 8>();
    case PDN_TILE_8x8: return lds_of<R, 8, 8>();
    case PDN_TILE_15x15: return lds_of<R, 15, 15>();
    default: return -1;
    }
}

int elem_node_lds_bytes(int mixed, int tile) { return mixed ? lds_r<float>(tile) : lds_r<double>(tile); }

template hipError_t launch_elem_node<float>(const ElemArgs<float> &, int, hipStream_t);
template hipError_t launch_elem_node<double>(const ElemArgs<double> &, int, hipStream_t);

template <typename R, int TX, int TY>
static hipError_t launch_enb(const ElemArgs<R> *args, const int *start, int ncase, int nblocks, hipStream_t s)
{
    hipLaunchKernelGGL((k_elem_node_batch<R, TX, TY>), dim3(nblocks), dim3(PDN_TILE_THREADS(TX, TY)), 0, s, args,
                       start, ncase);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_elem_node_batch(const ElemArgs<R> *args, const int *start, int ncase, int nblocks, int tile,
                                  hipStream_t s)
{
    if (ncase < 1 || nblocks < 1) return hipErrorInvalidValue;
    switch (tile) {
    case PDN_TILE_16x16: return launch_enb<R, 16, 16>(args, start, ncase, nblocks, s);
    case PDN_TILE_32x8: return launch_enb<R, 32, 8>(args, start, ncase, nblocks, s);
    case PDN_TILE_8x8: return launch_enb<R, 8, 8>(args, start, ncase, nblocks, s);
    case PDN_TILE_15x15: return launch_enb<R, 15, 15>(args, start, ncase, nblocks, s);
    default: return hipErrorInvalidValue;
    }
}
template hipError_t launch_elem_node_batch<float>(const ElemArgs<float> *, const int *, int, int, int, hipStream_t);
template hipError_t launch_elem_node_batch<double>(const ElemArgs<double> *, const int *, int, int, int,
                                                   hipStream_t);

hipError_t launch_contact_batch(const ContactArgs *args, const int *start, int ncase, int nblocks, hipStream_t s)
{
    if (ncase < 1 || nblocks < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_contact_batch, dim3(nblocks), dim3(PDN_K1_THREADS), 0, s, args, start, ncase);
    return hipGetLastError();
}

int contact_blocks(const ContactArgs &c)
{
    const int nc = (c.ci1 - c.ci0) * (c.cj1 - c.cj0);
    const int nb = (nc + PDN_K1_THREADS - 1) / PDN_K1_THREADS;
    return nb < 1 ? 1 : nb;
}

hipError_t launch_contact(const ContactArgs &c, hipStream_t s)
{
    hipLaunchKernelGGL(k_contact, dim3(contact_blocks(c)), dim3(PDN_K1_THREADS), 0, s, c);
    return hipGetLastError();
}

hipError_t launch_contact_init(const ContactArgs &c, int reset_active, hipStream_t s)
{
    const int nc = (c.ci1 - c.ci0) * (c.cj1 - c.cj0);
    const int nb = (nc + 255) / 256 > 0 ? (nc + 255) / 256 : 1;
    hipLaunchKernelGGL(k_contact_init, dim3(nb), dim3(256), 0, s, c, reset_active);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_damage_bulk(const R *r, const LayerInfo *layers, const int *bulk_layer, const PlyC<R> *ply,
                              const R *hx, const R *hy, int nx, int ny, int64_t ne, int kind, double *out,
                              hipStream_t s)
{
    int64_t nb = (ne + 255) / 256;
    if (nb > 65536) nb = 65536;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_damage_bulk<R>, dim3((unsigned)nb), dim3(256), 0, s, r, layers, bulk_layer, ply, hx, hy,
                       nx, ny, ne, kind, out);
    return hipGetLastError();
}
template hipError_t launch_damage_bulk<float>(const float *, const LayerInfo *, const int *, const PlyC<float> *,
                                              const float *, const float *, int, int, int64_t, int, double *,
                                              hipStream_t);
template hipError_t launch_damage_bulk<double>(const double *, const LayerInfo *, const int *, const PlyC<double> *,
                                               const double *, const double *, int, int, int64_t, int, double *,
                                               hipStream_t);

template <typename R>
hipError_t launch_damage_coh(const R *rd, const double *d, const LayerInfo *layers, const int *coh_layer,
                             const PlyC<R> *ply, int nx, int ny, int64_t nce, double *out, hipStream_t s)
{
    int64_t nb = (nce + 255) / 256;
    if (nb > 65536) nb = 65536;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_damage_coh<R>, dim3((unsigned)nb), dim3(256), 0, s, rd, d, layers, coh_layer, ply, nx, ny,
                       nce, out);
    return hipGetLastError();
}
template hipError_t launch_damage_coh<float>(const float *, const double *, const LayerInfo *, const int *,
                                             const PlyC<float> *, int, int, int64_t, double *, hipStream_t);
template hipError_t launch_damage_coh<double>(const double *, const double *, const LayerInfo *, const int *,
                                              const PlyC<double> *, int, int, int64_t, double *, hipStream_t);

hipError_t launch_project_max(const double *in, int64_t ncol, int nlayers, double *out, hipStream_t s)
{
    int64_t nb = (ncol + 255) / 256;
    if (nb > 65536) nb = 65536;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_project_max, dim3((unsigned)nb), dim3(256), 0, s, in, ncol, nlayers, out);
    return hipGetLastError();
}

}  // namespace pdn
