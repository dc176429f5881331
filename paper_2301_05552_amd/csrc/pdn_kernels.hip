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
//                The contact step (Algorithms 1-2: detection, projection,
//                reaction, release with the repeat flag) is done in the same
//                pass on the top plane.
//  k_books     : one workgroup after a contact pass: fixed-order sums of the
//                reaction and the energy books, striker update, history row.
//  k_contact_init, k_cand_scatter : candidate bookkeeping.
//  k_damage_*  : damage-field outputs.
#include "pdn_internal.h"
#include "pdn_launch.h"
#include "pdn_elem.h"

namespace pdn {

// candidate bookkeeping at (re)initialisation: velocity and reaction of the
// last step from the state, corrected copies equal to the state, and (on a
// restart of the contact) both active sets cleared
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
            C.cand[6 * j + c] = C.d[3 * n + c];
            C.cand[6 * j + 3 + c] = C.v[3 * n + c];
        }
        if (reset_active) C.active[j] = C.active[j + nc] = 0;
    }
}

// the contact pass leaves corrected top-surface candidates in C.cand: put them
// into the state buffers (before the state is read or restarted from)
__global__ void k_cand_scatter(ContactArgs C)
{
    const int cw = C.ci1 - C.ci0, nc = cw * (C.cj1 - C.cj0);
    const int64_t plane = (int64_t)(C.nx + 1) * (C.ny + 1);
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nc; j += gridDim.x * blockDim.x) {
        const int i = C.ci0 + j % cw, jj = C.cj0 + j / cw;
        const int64_t n = i + (int64_t)(C.nx + 1) * jj + plane * (C.K - 1);
        for (int c = 0; c < 3; ++c) {
            C.d[3 * n + c] = C.cand[6 * j + c];
            C.v[3 * n + c] = C.cand[6 * j + 3 + c];
        }
    }
}

// ---------------------------------------------------------------------------
// damage fields
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_damage_bulk(const R *r, int ngp, const LayerInfo *layers, const int *bulk_layer,
                              const PlyC<R> *ply, const R *hx, const R *hy, int nx, int ny, int64_t ne, int kind,
                              double *out)
{
    for (int64_t e = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; e < ne; e += (int64_t)gridDim.x * blockDim.x) {
        const int ie = (int)(e % nx), je = (int)((e / nx) % ny), lb = (int)(e / ((int64_t)nx * ny));
        const LayerInfo L = layers[bulk_layer[lb]];
        const PlyC<R> &P = ply[L.ply];
        double val = 0;
        // the largest over the element's Gauss points
        for (int g = 0; g < ngp && P.law != 0; ++g) {
            const R lc = cbrt(hx[ie] * hy[je] * (R)L.hz);
            // one point: record e; eight: a layer's records point by point
            const int64_t rec = ngp == 1 ? e : 8 * (int64_t)nx * ny * lb + (int64_t)g * nx * ny + ie + (int64_t)nx * je;
            const R *q = r + 4 * rec;
            double vg;
            if (kind == 0) {
                R a = damage_bilinear(q[0], P.XT, P.E1, P.GXT, P.fXT, P.fGT, lc);
                R b = damage_bilinear(q[1], P.XC, P.E1, P.GXC, P.fXC, P.fGC, lc);
                vg = (double)rmax(a, b);
            } else if (kind == 1) {
                R a = damage_exp(q[2], cap_strength(P.YT, P.E2, P.GYT, lc), P.E2, P.GYT, lc);
                R b = damage_exp(q[3], cap_strength(P.YC, P.E2, P.GYC, lc), P.E2, P.GYC, lc);
                vg = (double)rmax(a, b);
            } else {
                vg = (double)damage_exp(q[2], cap_strength(P.SL, P.G12v, P.GSL, lc), P.G12v, P.GSL, lc);
            }
            val = fmax(val, vg);
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
hipError_t launch_elem_node(const ElemArgs<R> &a, int tile, int sur, int ngp, hipStream_t s)
{
    if (ngp == 8)
        return sur ? hipErrorInvalidValue
                   : a.ep ? launch_elem_node_full_plas<R>(a, tile, s) : launch_elem_node_full<R>(a, tile, s);
    if (a.ep) return sur ? hipErrorInvalidValue : launch_elem_node_plas<R>(a, tile, s);
    if (sur == 2 && tile == PDN_TILE_15x15) return launch_elem_node_sur_wide<R>(a, tile, s);
    return sur ? launch_elem_node_sur<R>(a, tile, s) : launch_elem_node_v<R, false>(a, tile, s);
}
template hipError_t launch_elem_node<float>(const ElemArgs<float> &, int, int, int, hipStream_t);
template hipError_t launch_elem_node<double>(const ElemArgs<double> &, int, int, int, hipStream_t);

template <typename R>
hipError_t launch_books(const ElemArgs<R> &a, hipStream_t s)
{
    hipLaunchKernelGGL(k_books<R>, dim3(1), dim3(PDN_BOOKS_THREADS), 0, s, a);
    return hipGetLastError();
}
template hipError_t launch_books<float>(const ElemArgs<float> &, hipStream_t);
template hipError_t launch_books<double>(const ElemArgs<double> &, hipStream_t);

int elem_node_lds_bytes(int mixed, int tile, bool sur)
{
    if (sur) return elem_node_lds_bytes_sur(mixed, tile);
    return mixed ? lds_v<float, false>(tile) : lds_v<double, false>(tile);
}

template <typename R>
hipError_t launch_elem_node_batch(const ElemArgs<R> *args, const int *start, int ncase, int nblocks, int tile,
                                  bool sur, int ngp, bool contact, hipStream_t s)
{
    hipError_t e = ngp == 8 ? (sur ? hipErrorInvalidValue
                                   : launch_elem_node_batch_full<R>(args, start, ncase, nblocks, tile, s))
                 : sur      ? launch_elem_node_batch_sur<R>(args, start, ncase, nblocks, tile, s)
                            : launch_elem_node_batch_v<R, false>(args, start, ncase, nblocks, tile, s);
    if (e == hipSuccess && contact) {
        hipLaunchKernelGGL(k_books_batch<R>, dim3(ncase), dim3(PDN_BOOKS_THREADS), 0, s, args);
        e = hipGetLastError();
    }
    return e;
}
template hipError_t launch_elem_node_batch<float>(const ElemArgs<float> *, const int *, int, int, int, bool, int,
                                                  bool, hipStream_t);
template hipError_t launch_elem_node_batch<double>(const ElemArgs<double> *, const int *, int, int, int, bool, int,
                                                   bool, hipStream_t);

hipError_t launch_contact_init(const ContactArgs &c, int reset_active, hipStream_t s)
{
    const int nc = (c.ci1 - c.ci0) * (c.cj1 - c.cj0);
    const int nb = (nc + 255) / 256 > 0 ? (nc + 255) / 256 : 1;
    hipLaunchKernelGGL(k_contact_init, dim3(nb), dim3(256), 0, s, c, reset_active);
    return hipGetLastError();
}

hipError_t launch_cand_scatter(const ContactArgs &c, hipStream_t s)
{
    const int nc = (c.ci1 - c.ci0) * (c.cj1 - c.cj0);
    const int nb = (nc + 255) / 256 > 0 ? (nc + 255) / 256 : 1;
    hipLaunchKernelGGL(k_cand_scatter, dim3(nb), dim3(256), 0, s, c);
    return hipGetLastError();
}

template <typename R>
hipError_t launch_damage_bulk(const R *r, int ngp, const LayerInfo *layers, const int *bulk_layer,
                              const PlyC<R> *ply, const R *hx, const R *hy, int nx, int ny, int64_t ne, int kind,
                              double *out, hipStream_t s)
{
    int64_t nb = (ne + 255) / 256;
    if (nb > 65536) nb = 65536;
    if (nb < 1) nb = 1;
    hipLaunchKernelGGL(k_damage_bulk<R>, dim3((unsigned)nb), dim3(256), 0, s, r, ngp, layers, bulk_layer, ply, hx,
                       hy, nx, ny, ne, kind, out);
    return hipGetLastError();
}
template hipError_t launch_damage_bulk<float>(const float *, int, const LayerInfo *, const int *,
                                              const PlyC<float> *, const float *, const float *, int, int, int64_t,
                                              int, double *, hipStream_t);
template hipError_t launch_damage_bulk<double>(const double *, int, const LayerInfo *, const int *,
                                               const PlyC<double> *, const double *, const double *, int, int,
                                               int64_t, int, double *, hipStream_t);

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
