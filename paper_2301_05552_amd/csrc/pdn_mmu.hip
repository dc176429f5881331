// pdn_mmu.hip -- mesh multiplication of hexahedral meshes with interface
// elements on the device (Section 2.4, Eq. mmu, Algorithm 3).
//
// One division level: every divided edge gets its midpoint, every divided
// face its centre and every bulk element its centre; a bulk hexahedron
// becomes eight, an 8-node interface element (zero thickness; bottom face
// 0-3, top face 4-7) becomes four, divided only by planes parallel to its
// normal (its edges across the thickness and its lateral faces are not
// divided, and it has no centre node).
//
//  k_mmu_edge_keys / k_mmu_face_keys : one 64-bit key per element edge / face
//      slot: (smaller node, larger node) for an edge, (smallest node, node
//      diagonally opposite it) for a quadrilateral face;
//  radix sort of the keys with their slots (hipCUB), head flags, exclusive
//      scan: the unique edges and faces numbered in ascending key order, and
//      every slot's number;
//  k_mmu_coords : positions of the new mesh (old nodes, edge midpoints, face
//      centres, element centres; sums in a fixed order);
//  k_mmu_children : connectivity of the children from each element's
//      3 x 3 x 3 (bulk) or 3 x 3 x 2 (interface) lattice of nodes.
// Boundary faces (used by one element; interface lateral faces counted apart)
// are counted from a sort of every face key.
#include "pdn_launch.h"

#include <hipcub/hipcub.hpp>

#include <vector>

namespace pdn {

namespace {

__constant__ int kEdge[12][2] = {{0, 1}, {1, 2}, {2, 3}, {3, 0}, {4, 5}, {5, 6}, {6, 7}, {7, 4},
                                 {0, 4}, {1, 5}, {2, 6}, {3, 7}};
__constant__ int kFace[6][4] = {{0, 1, 2, 3}, {4, 5, 6, 7}, {0, 1, 5, 4}, {1, 2, 6, 5}, {2, 3, 7, 6}, {3, 0, 4, 7}};
// lattice positions (a, b, c) of the corners, edge midpoints and face centres
__constant__ int kCornerAt[8][3] = {{0, 0, 0}, {2, 0, 0}, {2, 2, 0}, {0, 2, 0},
                                    {0, 0, 2}, {2, 0, 2}, {2, 2, 2}, {0, 2, 2}};
__constant__ int kEdgeAt[12][3] = {{1, 0, 0}, {2, 1, 0}, {1, 2, 0}, {0, 1, 0}, {1, 0, 2}, {2, 1, 2},
                                   {1, 2, 2}, {0, 1, 2}, {0, 0, 1}, {2, 0, 1}, {2, 2, 1}, {0, 2, 1}};
__constant__ int kFaceAt[6][3] = {{1, 1, 0}, {1, 1, 2}, {1, 0, 1}, {2, 1, 1}, {1, 2, 1}, {0, 1, 1}};
__constant__ int kChild[8][3] = {{0, 0, 0}, {1, 0, 0}, {1, 1, 0}, {0, 1, 0},
                                 {0, 0, 1}, {1, 0, 1}, {1, 1, 1}, {0, 1, 1}};

__device__ __forceinline__ uint64_t edge_key(int a, int b)
{
    const uint32_t lo = (uint32_t)(a < b ? a : b), hi = (uint32_t)(a < b ? b : a);
    return ((uint64_t)lo << 32) | hi;
}

__device__ __forceinline__ uint64_t face_key(const int q[4])
{
    int m = 0;
    for (int k = 1; k < 4; ++k)
        if (q[k] < q[m]) m = k;
    return ((uint64_t)(uint32_t)q[m] << 32) | (uint32_t)q[(m + 2) & 3];
}

// divided edge slots: 12 per bulk element (slot 12 e + l), then 8 per interface
// (slot 12 nh + 8 c + l, the edges of its bottom and top faces)
__global__ void k_mmu_edge_keys(const int32_t *__restrict__ H, int64_t nh, const int32_t *__restrict__ C, int64_t nc,
                                uint64_t *__restrict__ keys, int32_t *__restrict__ slots)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nb = 12 * nh, n = nb + 8 * nc;
    if (s >= n) return;
    const int32_t *E;
    int l;
    if (s < nb) { E = H + 8 * (s / 12); l = (int)(s % 12); }
    else { E = C + 8 * ((s - nb) / 8); l = (int)((s - nb) % 8); }
    keys[s] = edge_key(E[kEdge[l][0]], E[kEdge[l][1]]);
    slots[s] = (int32_t)s;
}

// face slots: 6 per bulk element, then per interface its bottom and top faces
// (divided) and, with `lateral`, its 4 lateral faces (slot 6 nh + 6 c + l)
__global__ void k_mmu_face_keys(const int32_t *__restrict__ H, int64_t nh, const int32_t *__restrict__ C, int64_t nc,
                                int per_interface, uint64_t *__restrict__ keys, int32_t *__restrict__ slots)
{
    const int64_t s = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t nb = 6 * nh, n = nb + per_interface * nc;
    if (s >= n) return;
    const int32_t *E;
    int l;
    if (s < nb) { E = H + 8 * (s / 6); l = (int)(s % 6); }
    else { E = C + 8 * ((s - nb) / per_interface); l = (int)((s - nb) % per_interface); }
    const int q[4] = {E[kFace[l][0]], E[kFace[l][1]], E[kFace[l][2]], E[kFace[l][3]]};
    keys[s] = face_key(q);
    slots[s] = (int32_t)s;
}

__global__ void k_mmu_heads(const uint64_t *__restrict__ k, int64_t n, int32_t *__restrict__ head)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) head[i] = (i == 0 || k[i] != k[i - 1]) ? 1 : 0;
}

// number of each slot (ascending key order) and the first slot of each number
__global__ void k_mmu_number(const int32_t *__restrict__ slot_sorted, const int32_t *__restrict__ head,
                             const int32_t *__restrict__ pos, int64_t n, int32_t *__restrict__ id_of_slot,
                             int32_t *__restrict__ first_slot)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const int32_t id = pos[i] + head[i] - 1;
    id_of_slot[slot_sorted[i]] = id;
    if (head[i]) first_slot[id] = slot_sorted[i];
}

// boundary faces: keys used once; counts[0] all, counts[1] interface lateral faces
__global__ void k_mmu_boundary(const uint64_t *__restrict__ k, const int32_t *__restrict__ slot_sorted, int64_t n,
                               int64_t first_lateral, unsigned long long *__restrict__ counts)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    const bool single = (i == 0 || k[i] != k[i - 1]) && (i == n - 1 || k[i] != k[i + 1]);
    if (!single) return;
    atomicAdd(&counts[0], 1ull);
    const int64_t s = slot_sorted[i];
    if (s >= first_lateral && ((s - first_lateral) % 6) >= 2) atomicAdd(&counts[1], 1ull);
}

__device__ __forceinline__ const int32_t *face_slot_nodes(const int32_t *H, int64_t nh, const int32_t *C, int64_t s,
                                                          int &l)
{
    if (s < 6 * nh) { l = (int)(s % 6); return H + 8 * (s / 6); }
    l = (int)((s - 6 * nh) % 2);
    return C + 8 * ((s - 6 * nh) / 2);
}

// positions of the divided mesh
__global__ void k_mmu_coords(const double *__restrict__ X, int64_t nn, const int32_t *__restrict__ H, int64_t nh,
                             const int32_t *__restrict__ C, const int32_t *__restrict__ H8,
                             const uint64_t *__restrict__ ekeys_sorted, const int32_t *__restrict__ e_first,
                             int64_t ne, const int32_t *__restrict__ f_first, int64_t nf, double *__restrict__ Xo)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t n = nn + ne + nf + nh;
    if (i >= n) return;
    double p[3];
    if (i < nn) {
        for (int c = 0; c < 3; ++c) p[c] = X[3 * i + c];
    } else if (i < nn + ne) {
        // the edge of a first slot: its end nodes, smaller first
        const int64_t s = e_first[i - nn];
        const int32_t *E;
        int l;
        if (s < 12 * nh) { E = H + 8 * (s / 12); l = (int)(s % 12); }
        else { E = C + 8 * ((s - 12 * nh) / 8); l = (int)((s - 12 * nh) % 8); }
        int a = E[kEdge[l][0]], b = E[kEdge[l][1]];
        if (b < a) { const int t = a; a = b; b = t; }
        for (int c = 0; c < 3; ++c) p[c] = 0.5 * (X[3 * a + c] + X[3 * b + c]);
    } else if (i < nn + ne + nf) {
        int l;
        const int32_t *E = face_slot_nodes(H, nh, C, f_first[i - nn - ne], l);
        int q[4] = {E[kFace[l][0]], E[kFace[l][1]], E[kFace[l][2]], E[kFace[l][3]]};
        for (int u = 1; u < 4; ++u)                         // ascending node numbers
            for (int v = u; v > 0 && q[v] < q[v - 1]; --v) { const int t = q[v]; q[v] = q[v - 1]; q[v - 1] = t; }
        for (int c = 0; c < 3; ++c)
            p[c] = 0.25 * (((X[3 * q[0] + c] + X[3 * q[1] + c]) + X[3 * q[2] + c]) + X[3 * q[3] + c]);
    } else {
        const int32_t *E = H8 + 8 * (i - nn - ne - nf);
        for (int c = 0; c < 3; ++c) {
            double t = X[3 * E[0] + c];
            for (int a = 1; a < 8; ++a) t = t + X[3 * E[a] + c];
            p[c] = 0.125 * t;
        }
    }
    for (int c = 0; c < 3; ++c) Xo[3 * i + c] = p[c];
}

// children: bulk element e -> 8e .. 8e+7 (octant i + 2j + 4k), interface c ->
// 4c .. 4c+3 (quadrant i + 2j); tags inherited
__global__ void k_mmu_children(const int32_t *__restrict__ H, int64_t nh, const int32_t *__restrict__ C, int64_t nc,
                               const int32_t *__restrict__ e_id, const int32_t *__restrict__ f_id, int64_t nn,
                               int64_t ne, int64_t nf, const int32_t *__restrict__ htag,
                               const int32_t *__restrict__ ctag, int32_t *__restrict__ Ho, int32_t *__restrict__ Co,
                               int32_t *__restrict__ hto, int32_t *__restrict__ cto)
{
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= nh + nc) return;
    int L[3][3][3];
    if (t < nh) {
        const int64_t e = t;
        for (int a = 0; a < 8; ++a) L[kCornerAt[a][0]][kCornerAt[a][1]][kCornerAt[a][2]] = H[8 * e + a];
        for (int l = 0; l < 12; ++l) L[kEdgeAt[l][0]][kEdgeAt[l][1]][kEdgeAt[l][2]] = (int)(nn + e_id[12 * e + l]);
        for (int l = 0; l < 6; ++l)
            L[kFaceAt[l][0]][kFaceAt[l][1]][kFaceAt[l][2]] = (int)(nn + ne + f_id[6 * e + l]);
        L[1][1][1] = (int)(nn + ne + nf + e);
        for (int ch = 0; ch < 8; ++ch)
            for (int v = 0; v < 8; ++v)
                Ho[64 * e + 8 * ch + v] =
                    L[kChild[ch][0] + kChild[v][0]][kChild[ch][1] + kChild[v][1]][kChild[ch][2] + kChild[v][2]];
        if (htag)
            for (int ch = 0; ch < 8; ++ch) hto[8 * e + ch] = htag[e];
    } else {
        const int64_t c = t - nh;
        const int64_t es = 12 * nh + 8 * c, fs = 6 * nh + 2 * c;
        for (int a = 0; a < 8; ++a) L[kCornerAt[a][0]][kCornerAt[a][1]][kCornerAt[a][2]] = C[8 * c + a];
        for (int l = 0; l < 8; ++l) L[kEdgeAt[l][0]][kEdgeAt[l][1]][kEdgeAt[l][2]] = (int)(nn + e_id[es + l]);
        L[1][1][0] = (int)(nn + ne + f_id[fs]);
        L[1][1][2] = (int)(nn + ne + f_id[fs + 1]);
        for (int ch = 0; ch < 4; ++ch)
            for (int v = 0; v < 4; ++v) {
                const int a = kChild[ch][0] + kChild[v][0], b = kChild[ch][1] + kChild[v][1];
                Co[32 * c + 8 * ch + v] = L[a][b][0];
                Co[32 * c + 8 * ch + v + 4] = L[a][b][2];
            }
        if (ctag)
            for (int ch = 0; ch < 4; ++ch) cto[4 * c + ch] = ctag[c];
    }
}

// device buffers freed on scope exit
struct Bufs {
    std::vector<void *> ps;
    ~Bufs()
    {
        for (void *p : ps) (void)hipFree(p);
    }
    template <typename T>
    hipError_t get(T **p, size_t n)
    {
        *p = nullptr;
        hipError_t e = hipMalloc((void **)p, (n ? n : 1) * sizeof(T));
        if (e == hipSuccess) ps.push_back((void *)*p);
        return e;
    }
};

#define MMU_CHK(call)                                  \
    do {                                               \
        const hipError_t e_ = (call);                  \
        if (e_ != hipSuccess) return e_;               \
    } while (0)

inline unsigned blocks_of(int64_t n) { return (unsigned)((n + 255) / 256 > 0 ? (n + 255) / 256 : 1); }

// sort keys with their slots; number the unique keys in ascending order
hipError_t number_keys(uint64_t *keys, int32_t *slots, int64_t n, Bufs &B, int32_t *id_of_slot, int32_t *first_slot,
                       int64_t *n_unique, uint64_t **keys_sorted_out, int32_t **slots_sorted_out, hipStream_t s)
{
    *n_unique = 0;
    if (n == 0) return hipSuccess;
    uint64_t *ks;
    int32_t *ss, *head, *pos;
    MMU_CHK(B.get(&ks, n));
    MMU_CHK(B.get(&ss, n));
    MMU_CHK(B.get(&head, n));
    MMU_CHK(B.get(&pos, n));
    size_t tb = 0;
    MMU_CHK(hipcub::DeviceRadixSort::SortPairs(nullptr, tb, keys, ks, slots, ss, (int)n, 0, 64, s));
    void *tmp;
    MMU_CHK(B.get((char **)&tmp, tb));
    MMU_CHK(hipcub::DeviceRadixSort::SortPairs(tmp, tb, keys, ks, slots, ss, (int)n, 0, 64, s));
    hipLaunchKernelGGL(k_mmu_heads, dim3(blocks_of(n)), dim3(256), 0, s, ks, n, head);
    MMU_CHK(hipGetLastError());
    size_t tb2 = 0;
    MMU_CHK(hipcub::DeviceScan::ExclusiveSum(nullptr, tb2, head, pos, (int)n, s));
    void *tmp2;
    MMU_CHK(B.get((char **)&tmp2, tb2));
    MMU_CHK(hipcub::DeviceScan::ExclusiveSum(tmp2, tb2, head, pos, (int)n, s));
    int32_t last[2];
    MMU_CHK(hipMemcpyAsync(&last[0], pos + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MMU_CHK(hipMemcpyAsync(&last[1], head + n - 1, sizeof(int32_t), hipMemcpyDeviceToHost, s));
    MMU_CHK(hipStreamSynchronize(s));
    *n_unique = (int64_t)last[0] + last[1];
    if (id_of_slot) {
        hipLaunchKernelGGL(k_mmu_number, dim3(blocks_of(n)), dim3(256), 0, s, ss, head, pos, n, id_of_slot,
                           first_slot);
        MMU_CHK(hipGetLastError());
    }
    if (keys_sorted_out) *keys_sorted_out = ks;
    if (slots_sorted_out) *slots_sorted_out = ss;
    return hipSuccess;
}

}  // namespace

// One division level on the device.  In: X (3 nn), H (8 nh), C (8 nc), tags
// (may be null).  Out: buffers allocated here (hipMalloc; the caller frees
// them with hipFree) and the level's counts.
hipError_t mmu_divide(const double *X, int64_t nn, const int32_t *H, int64_t nh, const int32_t *C, int64_t nc,
                      const int32_t *htag, const int32_t *ctag, double **Xo, int32_t **Ho, int32_t **Co,
                      int32_t **hto, int32_t **cto, MmuLevel *info, hipStream_t s)
{
    *Xo = nullptr; *Ho = *Co = *hto = *cto = nullptr;
    Bufs B;
    // divided edges
    const int64_t se = 12 * nh + 8 * nc;
    uint64_t *ek;
    int32_t *es, *e_id, *e_first;
    MMU_CHK(B.get(&ek, se));
    MMU_CHK(B.get(&es, se));
    MMU_CHK(B.get(&e_id, se));
    MMU_CHK(B.get(&e_first, se));
    if (se) {
        hipLaunchKernelGGL(k_mmu_edge_keys, dim3(blocks_of(se)), dim3(256), 0, s, H, nh, C, nc, ek, es);
        MMU_CHK(hipGetLastError());
    }
    int64_t ne = 0;
    uint64_t *eks = nullptr;
    MMU_CHK(number_keys(ek, es, se, B, e_id, e_first, &ne, &eks, nullptr, s));
    // divided faces
    const int64_t sf = 6 * nh + 2 * nc;
    uint64_t *fk;
    int32_t *fs, *f_id, *f_first;
    MMU_CHK(B.get(&fk, sf));
    MMU_CHK(B.get(&fs, sf));
    MMU_CHK(B.get(&f_id, sf));
    MMU_CHK(B.get(&f_first, sf));
    if (sf) {
        hipLaunchKernelGGL(k_mmu_face_keys, dim3(blocks_of(sf)), dim3(256), 0, s, H, nh, C, nc, 2, fk, fs);
        MMU_CHK(hipGetLastError());
    }
    int64_t nf = 0;
    MMU_CHK(number_keys(fk, fs, sf, B, f_id, f_first, &nf, nullptr, nullptr, s));
    // boundary faces of the base mesh (all faces, interface lateral ones included)
    const int64_t sa = 6 * nh + 6 * nc;
    uint64_t *ak, *aks = nullptr;
    int32_t *as, *ass = nullptr;
    unsigned long long *bc;
    MMU_CHK(B.get(&ak, sa));
    MMU_CHK(B.get(&as, sa));
    MMU_CHK(B.get(&bc, 2));
    MMU_CHK(hipMemsetAsync(bc, 0, 2 * sizeof(unsigned long long), s));
    unsigned long long bh[2] = {0, 0};
    if (sa) {
        hipLaunchKernelGGL(k_mmu_face_keys, dim3(blocks_of(sa)), dim3(256), 0, s, H, nh, C, nc, 6, ak, as);
        MMU_CHK(hipGetLastError());
        int64_t na = 0;
        MMU_CHK(number_keys(ak, as, sa, B, nullptr, nullptr, &na, &aks, &ass, s));
        hipLaunchKernelGGL(k_mmu_boundary, dim3(blocks_of(sa)), dim3(256), 0, s, aks, ass, sa, 6 * nh, bc);
        MMU_CHK(hipGetLastError());
        MMU_CHK(hipMemcpyAsync(bh, bc, sizeof bh, hipMemcpyDeviceToHost, s));
        MMU_CHK(hipStreamSynchronize(s));
    }
    // the divided mesh
    const int64_t nn1 = nn + ne + nf + nh;
    if (nn1 > INT32_MAX || 8 * nh > INT32_MAX || 4 * nc > INT32_MAX) return hipErrorInvalidValue;
    MMU_CHK(hipMalloc((void **)Xo, (size_t)(3 * nn1 > 0 ? 3 * nn1 : 1) * sizeof(double)));
    MMU_CHK(hipMalloc((void **)Ho, (size_t)(64 * nh > 0 ? 64 * nh : 1) * sizeof(int32_t)));
    MMU_CHK(hipMalloc((void **)Co, (size_t)(32 * nc > 0 ? 32 * nc : 1) * sizeof(int32_t)));
    if (htag) MMU_CHK(hipMalloc((void **)hto, (size_t)(8 * nh > 0 ? 8 * nh : 1) * sizeof(int32_t)));
    if (ctag) MMU_CHK(hipMalloc((void **)cto, (size_t)(4 * nc > 0 ? 4 * nc : 1) * sizeof(int32_t)));
    hipLaunchKernelGGL(k_mmu_coords, dim3(blocks_of(nn1)), dim3(256), 0, s, X, nn, H, nh, C, H, eks, e_first, ne,
                       f_first, nf, *Xo);
    MMU_CHK(hipGetLastError());
    if (nh + nc) {
        hipLaunchKernelGGL(k_mmu_children, dim3(blocks_of(nh + nc)), dim3(256), 0, s, H, nh, C, nc, e_id, f_id, nn,
                           ne, nf, htag, ctag, *Ho, *Co, *hto, *cto);
        MMU_CHK(hipGetLastError());
    }
    MMU_CHK(hipStreamSynchronize(s));
    info->nn = nn1;
    info->nh = 8 * nh;
    info->nc = 4 * nc;
    info->n_edges = ne;
    info->n_faces = nf;
    info->nb0 = (int64_t)bh[0];
    info->nb_int0 = (int64_t)bh[1];
    return hipSuccess;
}

}  // namespace pdn
