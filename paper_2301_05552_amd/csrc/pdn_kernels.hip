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
#include "pdn_elem.h"

namespace pdn {

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
        G->sur_gp += P[T_SURN];
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

template <typename R>
hipError_t launch_elem_node(const ElemArgs<R> &a, int tile, bool sur, hipStream_t s)
{
    return sur ? launch_elem_node_sur<R>(a, tile, s) : launch_elem_node_v<R, false>(a, tile, s);
}
template hipError_t launch_elem_node<float>(const ElemArgs<float> &, int, bool, hipStream_t);
template hipError_t launch_elem_node<double>(const ElemArgs<double> &, int, bool, hipStream_t);

int elem_node_lds_bytes(int mixed, int tile, bool sur)
{
    if (sur) return elem_node_lds_bytes_sur(mixed, tile);
    return mixed ? lds_v<float, false>(tile) : lds_v<double, false>(tile);
}

template <typename R>
hipError_t launch_elem_node_batch(const ElemArgs<R> *args, const int *start, int ncase, int nblocks, int tile,
                                  bool sur, hipStream_t s)
{
    return sur ? launch_elem_node_batch_sur<R>(args, start, ncase, nblocks, tile, s)
               : launch_elem_node_batch_v<R, false>(args, start, ncase, nblocks, tile, s);
}
template hipError_t launch_elem_node_batch<float>(const ElemArgs<float> *, const int *, int, int, int, bool,
                                                  hipStream_t);
template hipError_t launch_elem_node_batch<double>(const ElemArgs<double> *, const int *, int, int, int, bool,
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
