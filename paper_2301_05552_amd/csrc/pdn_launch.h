// pdn_launch.h -- host-side launchers of the libpdn kernels (internal).
#pragma once
#include "pdn.h"
#include "pdn_internal.h"
#include "pdn_mlp.h"

#define PDN_MAX2(a, b) ((a) > (b) ? (a) : (b))
// threads of an element-tile workgroup: one per element column and one per node column
#define PDN_TILE_THREADS(TX, TY) ((PDN_MAX2((TX) * (TY), ((TX) + 1) * ((TY) + 1)) + 63) / 64 * 64)

// scratch of pdn_surrogate_grad_noalloc (per device): packed network, then the
// records of up to PDN_SUR_GRAD_NOALLOC_MAX points, then one partial gradient
// per 128-point training workgroup
#define PDN_SUR_NOALLOC_OFF_REC SUR_PACK_BYTES
#define PDN_SUR_NOALLOC_OFF_PART (PDN_SUR_NOALLOC_OFF_REC + PDN_SUR_GRAD_NOALLOC_MAX * 20 * 4)
#define PDN_SUR_NOALLOC_PARTS (PDN_SUR_GRAD_NOALLOC_MAX / 128)
#define PDN_SUR_NOALLOC_SCRATCH_BYTES (PDN_SUR_NOALLOC_OFF_PART + PDN_SUR_NOALLOC_PARTS * (PDN_SUR_NPARAM + 1) * 4)
#define PDN_SUR_NOALLOC_MAX_DEVICES 64

enum { PDN_TILE_16x16 = 0, PDN_TILE_32x8 = 1, PDN_TILE_8x8 = 2, PDN_TILE_15x15 = 3, PDN_TILE_31x15 = 4,
       PDN_TILE_COUNT = 5 };
static const int pdn_tile_dims[PDN_TILE_COUNT][2] = {{16, 16}, {32, 8}, {8, 8}, {15, 15}, {31, 15}};

namespace pdn {
// sur: 0 the plain build; 1 the build that evaluates the surrogate network on
// plies of law 2 (held to 2 waves per SIMD); 2 the same at 1 wave per SIMD
// (15x15 tile; other tiles take 1).  ngp: Gauss points of a bulk
// element (1 with hourglass control, or 8)
template <typename R>
hipError_t launch_elem_node(const ElemArgs<R> &a, int tile, int sur, int ngp, hipStream_t s);
// shear plasticity (one point, a.ep non-null): built for the 15x15, 16x16 and 8x8 tiles
template <typename R>
hipError_t launch_elem_node_plas(const ElemArgs<R> &a, int tile, hipStream_t s);
// full integration (ngp 8): built for the 15x15 and 16x16 tiles
template <typename R>
hipError_t launch_elem_node_full(const ElemArgs<R> &a, int tile, hipStream_t s);
// full integration with shear plasticity (ngp 8, a.ep non-null: 4 per Gauss
// point): the same tiles
template <typename R>
hipError_t launch_elem_node_full_plas(const ElemArgs<R> &a, int tile, hipStream_t s);
template <typename R>
hipError_t launch_elem_node_batch_full(const ElemArgs<R> *args, const int *start, int ncase, int nblocks, int tile,
                                       hipStream_t s);
inline bool tile_has_full(int tile) { return tile == PDN_TILE_15x15 || tile == PDN_TILE_16x16; }
// one-point elements with shear plasticity: those and 8x8 (more workgroups on small plates;
// the autotuner chooses)
inline bool tile_has_plas(int tile) { return tile_has_full(tile) || tile == PDN_TILE_8x8; }
// closes a contact pass (a.contact): books, striker update, history row
template <typename R>
hipError_t launch_books(const ElemArgs<R> &a, hipStream_t s);
template <typename R>
hipError_t launch_elem_node_sur(const ElemArgs<R> &a, int tile, hipStream_t s);
// the same at 1 wave per SIMD (15x15 tile)
template <typename R>
hipError_t launch_elem_node_sur_wide(const ElemArgs<R> &a, int tile, hipStream_t s);
// batched launches: case c owns blocks start[c] .. start[c+1]-1 (args and start in device memory)
// contact: the arguments are contact passes; a books kernel closes each case's step
template <typename R>
hipError_t launch_elem_node_batch(const ElemArgs<R> *args, const int *start, int ncase, int nblocks, int tile,
                                  bool sur, int ngp, bool contact, hipStream_t s);
template <typename R>
hipError_t launch_elem_node_batch_sur(const ElemArgs<R> *args, const int *start, int ncase, int nblocks, int tile,
                                      hipStream_t s);

// mesh multiplication (pdn_mmu.hip): one division level on the device
struct MmuLevel {
    int64_t nn, nh, nc;              // the divided mesh
    int64_t n_edges, n_faces;        // divided edges and faces of the base mesh
    int64_t nb0, nb_int0;            // boundary faces of the base mesh (of them, interface lateral faces)
};
hipError_t mmu_divide(const double *X, int64_t nn, const int32_t *H, int64_t nh, const int32_t *C, int64_t nc,
                      const int32_t *htag, const int32_t *ctag, double **Xo, int32_t **Ho, int32_t **Co,
                      int32_t **hto, int32_t **cto, MmuLevel *info, hipStream_t s);

int elem_node_lds_bytes(int mixed, int tile, bool sur);   // static LDS of one workgroup (-1 on error)
int elem_node_lds_bytes_sur(int mixed, int tile);
hipError_t launch_contact_init(const ContactArgs &c, int reset_active, hipStream_t s);
hipError_t launch_cand_scatter(const ContactArgs &c, hipStream_t s);
// per element: the largest over its ngp Gauss points
template <typename R>
hipError_t launch_damage_bulk(const R *r, int ngp, const LayerInfo *layers, const int *bulk_layer,
                              const PlyC<R> *ply, const R *hx, const R *hy, int nx, int ny, int64_t ne, int kind,
                              double *out, hipStream_t s);
template <typename R>
hipError_t launch_damage_coh(const R *rd, const double *d, const LayerInfo *layers, const int *coh_layer,
                             const PlyC<R> *ply, int nx, int ny, int64_t nce, double *out, hipStream_t s);
hipError_t launch_project_max(const double *in, int64_t ncol, int nlayers, double *out, hipStream_t s);

// constitutive surrogate (pdn_sur.hip); pk is a packed network (SUR_PACK_BYTES)
hipError_t launch_sur_pack(const float *w, void *pk, hipStream_t s);
hipError_t launch_sur_data(const PlyC<double> &P, double vol, uint64_t seed, int64_t p0, int64_t np, int n_inc,
                           float *out, hipStream_t s);
int sur_grad_blocks(int64_t batch, int nblk);
hipError_t launch_sur_grad(const void *pk, const float *data, int64_t n_data, int64_t base, int64_t batch, int nblk,
                           int randomize, uint64_t seed, float scale, float *partials, hipStream_t s);
hipError_t launch_sur_adam(const float *partials, int nparts, float *w, float *m, float *v, float lr, float b1,
                           float b2, float eps, float bc1, float bc2, float *loss_out, hipStream_t s);
hipError_t launch_sur_eval(const void *pk, const float *x, int64_t n, float *y, hipStream_t s);
int sur_loss_blocks(int64_t n);
// FP32 gradient: one partial (SUR_NPARAM + 1 floats, loss last) per 16 points
int sur_grad32_blocks(int64_t n);
hipError_t launch_sur_grad32(const float *w, const float *data, int64_t n, float scale, float *partials,
                             hipStream_t s);
hipError_t launch_sur_interleave(const float *x, const float *t, int64_t n, float *rec, hipStream_t s);
hipError_t launch_sur_grad_reduce(const float *part, int nparts, double count, float *grad, double *loss,
                                  hipStream_t s);
// device address of the fixed scratch array on `device` (must be the current device)
hipError_t sur_noalloc_scratch(int device, void **out);
hipError_t launch_sur_loss(const void *pk, const float *data, int64_t i0, int64_t n, double *partials, hipStream_t s);
}  // namespace pdn
