// pdn_sur.hip -- training set, training and evaluation of the constitutive
// surrogate network (gfx950).
//
//  k_sur_pack  : plain fp32 parameters -> bf16 matrix-core fragments + biases
//  k_sur_data  : strain paths through the exact intralaminar law (FP64), one
//                thread per path, (input, output) records in fp32
//  k_sur_grad  : forward and back-propagation of 32-point blocks on the
//                matrix cores; weight gradients contract over the points
//                (operands staged in LDS); one partial per workgroup
//  k_sur_adam  : fixed-order sum of the partials, Adam update
//  k_sur_eval / k_sur_loss : forward pass (the element kernel's routine)
#include "pdn_internal.h"
#include "pdn_launch.h"
#include "pdn_law.h"
#include "pdn_mlp.h"

#include <mutex>

namespace pdn {

#define SUR_REC 20                          // record: 10 inputs, 10 targets
#define SUR_TW 4                            // waves per training workgroup

// ---------------------------------------------------------------------------
// packing
// ---------------------------------------------------------------------------
__global__ void k_sur_pack(const float *__restrict__ w, uint4 *__restrict__ pk)
{
    const int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t < SF_COUNT * 64) {
        const int f = t >> 6, lane = t & 63, h = lane >> 5, m = lane & 31;
        bf16x8 v;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            float x = 0.f;
            if (f < SF_A2) {                                  // W1^T, bias as input 10
                const int k = 8 * h + i, o = 32 * (f - SF_A1) + m;
                x = k < SUR_NIN ? w[SUR_W1 + k * SUR_NH + o] : (k == SUR_NIN ? w[SUR_B1 + o] : 0.f);
            } else if (f < SF_A3) {                           // W2^T
                const int q = f - SF_A2;
                x = w[SUR_W2 + sur_unit(q & 3, h, i) * SUR_NH + 32 * (q >> 2) + m];
            } else if (f < SF_A4) {                           // W3^T
                const int q = f - SF_A3;
                x = w[SUR_W3 + sur_unit(q & 3, h, i) * SUR_NH + 32 * (q >> 2) + m];
            } else if (f < SF_A4B) {                          // W4^T (rows >= 10 zero)
                x = m < SUR_NOUT ? w[SUR_W4 + sur_unit(f - SF_A4, h, i) * SUR_NOUT + m] : 0.f;
            } else if (f < SF_A3B) {                          // W4 (k = output rows)
                const int row = sur_row(i, h);
                x = row < SUR_NOUT ? w[SUR_W4 + (32 * (f - SF_A4B) + m) * SUR_NOUT + row] : 0.f;
            } else if (f < SF_A2B) {                          // W3
                const int q = f - SF_A3B;
                x = w[SUR_W3 + (32 * (q >> 2) + m) * SUR_NH + sur_unit(q & 3, h, i)];
            } else {                                          // W2
                const int q = f - SF_A2B;
                x = w[SUR_W2 + (32 * (q >> 2) + m) * SUR_NH + sur_unit(q & 3, h, i)];
            }
            v[i] = (__bf16)x;
        }
        pk[t] = __builtin_bit_cast(uint4, v);
        return;
    }
    const int b = t - SF_COUNT * 64;
    if (b < 5 * 64 * 16) {
        const int blk = b >> 10, lane = (b >> 4) & 63, r = b & 15;
        const int row = sur_row(r, lane >> 5);
        float x;
        if (blk < 2) x = w[SUR_B2 + 32 * blk + row];
        else if (blk < 4) x = w[SUR_B3 + 32 * (blk - 2) + row];
        else x = row < SUR_NOUT ? w[SUR_B4 + row] : 0.f;
        reinterpret_cast<float *>(reinterpret_cast<char *>(pk) + SUR_FRAG_BYTES)[b] = x;
    }
}

// ---------------------------------------------------------------------------
// training set: strain paths (onset-scaled) through the exact law
// ---------------------------------------------------------------------------
struct SplitMix {
    uint64_t s;
    __device__ uint64_t next()
    {
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    __device__ double uniform() { return (double)(next() >> 11) * (1.0 / 9007199254740992.0); }
};

// Path p of the recipe (seeded SplitMix64 draws, every step one correctly
// rounded double operation, no fused multiply-adds): amplitude along a unit
// direction u per increment, monotone for even p, 2-4 reversals for odd p.
__device__ void sur_path_amp(uint64_t seed, int64_t p, int n_inc, double u[6], double *amp)
{
    SplitMix g{seed + (uint64_t)p};
    for (int k = 0; k < 6; ++k) u[k] = __dsub_rn(__dmul_rn(2.0, g.uniform()), 1.0);
    double nrm = __dmul_rn(u[0], u[0]);
    for (int k = 1; k < 6; ++k) nrm = __dadd_rn(nrm, __dmul_rn(u[k], u[k]));
    nrm = __dsqrt_rn(nrm);
    if (nrm == 0.0) {
        u[0] = 1.0;
        for (int k = 1; k < 6; ++k) u[k] = 0.0;
    } else {
        for (int k = 0; k < 6; ++k) u[k] = __ddiv_rn(u[k], nrm);
    }
    if ((p & 1) == 0) {
        const double A = __dmul_rn(3.0, g.uniform());
        for (int i = 1; i <= n_inc; ++i) amp[i - 1] = __dmul_rn(A, __ddiv_rn((double)i, (double)n_inc));
    } else {
        const int nr = 2 + (int)__dmul_rn(3.0, g.uniform());
        const int legs = nr + 1;
        double a[6];
        a[0] = 0.0;
        for (int j = 1; j <= legs; ++j) a[j] = (j & 1 ? 1.0 : -1.0) * __dmul_rn(3.0, g.uniform());
        const int per = n_inc / legs;
        int o = 0;
        for (int j = 1; j <= legs; ++j) {
            const int nj = per + (j == legs ? n_inc - per * legs : 0);
            for (int i = 1; i <= nj; ++i)
                amp[o++] = __dadd_rn(a[j - 1], __dmul_rn(__dsub_rn(a[j], a[j - 1]), __ddiv_rn((double)i, (double)nj)));
        }
    }
}

// record of increment i: (x, s_in) -> (sigma / X, s_out), s = 1 - 1/r
__global__ void k_sur_data(PlyC<double> P, double vol, uint64_t seed, int64_t p0, int64_t np, int n_inc,
                           float *__restrict__ out)
{
    const int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= np || n_inc > 64) return;
    const int64_t p = p0 + q;
    double u[6], amp[64];
    sur_path_amp(seed, p, n_inc, u, amp);
    const double X[6] = {P.XT, P.YT, P.YT, P.SL, P.SL, P.SL};
    const double E[6] = {P.E1, P.E2, P.E2, P.G23, P.G12, P.G12};
    double sc[6];
    for (int k = 0; k < 6; ++k) sc[k] = __ddiv_rn(X[k], E[k]);
    double r[4] = {1.0, 1.0, 1.0, 1.0};
    for (int i = 0; i < n_inc; ++i) {
        double x[6], e[6], sg[6];
        for (int k = 0; k < 6; ++k) {
            x[k] = __dmul_rn(amp[i], u[k]);
            e[k] = __dmul_rn(x[k], sc[k]);
        }
        float *rec = out + (q * n_inc + i) * SUR_REC;
        for (int k = 0; k < 6; ++k) rec[k] = (float)x[k];
        for (int k = 0; k < 4; ++k) rec[6 + k] = (float)(1.0 - 1.0 / r[k]);
        bool ch;
        cdm_update(P, vol, e, r, sg, ch);
        for (int k = 0; k < 6; ++k) rec[10 + k] = (float)(sg[k] / X[k]);
        for (int k = 0; k < 4; ++k) rec[16 + k] = (float)(1.0 - 1.0 / r[k]);
    }
}

// ---------------------------------------------------------------------------
// training: forward + back-propagation on the matrix cores
// ---------------------------------------------------------------------------
struct SurStage {                            // one wave's operands of a 32-point block, [unit][point]
    __bf16 x[32][32];                        // inputs (rows 0..9, 10 = constant 1, rest 0)
    __bf16 h[3][64][32];                     // hidden activations of layers 1..3
    __bf16 d[3][64][32];                     // back-propagated errors of layers 1..3
    __bf16 d4[32][32];                       // output errors (rows 0..9)
};

__device__ __forceinline__ bf16x8 stage_frag(const __bf16 *row, int cs, int h)
{
    return *reinterpret_cast<const bf16x8 *>(row + 16 * cs + 8 * h);
}

__device__ __forceinline__ uint64_t mix64(uint64_t z)
{
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

// Output blocks of the gradient (32 x 32, accumulated over the points):
//   0-1 dW4 (input block), 2-3 dW1 (output block; column 10 is b1), 4-7 dW2,
//   8-11 dW3 (output block * 2 + input block), 12 db4, 13-14 db2, 15-16 db3.
// A bias block multiplies by a constant-1 operand: every column holds the sum.
#define SUR_GBLOCKS 17
enum { GS_X, GS_H0, GS_H1, GS_H2, GS_D0, GS_D1, GS_D2, GS_D4, GS_ONE };

__device__ __forceinline__ void grad_block_src(int b, int &sa, int &ra, int &sb, int &rb)
{
    if (b < 2) { sa = GS_D4; ra = 0; sb = GS_H2; rb = 32 * b; }
    else if (b < 4) { sa = GS_D0; ra = 32 * (b - 2); sb = GS_X; rb = 0; }
    else if (b < 8) { sa = GS_D1; ra = 32 * ((b - 4) >> 1); sb = GS_H0; rb = 32 * ((b - 4) & 1); }
    else if (b < 12) { sa = GS_D2; ra = 32 * ((b - 8) >> 1); sb = GS_H1; rb = 32 * ((b - 8) & 1); }
    else if (b == 12) { sa = GS_D4; ra = 0; sb = GS_ONE; rb = 0; }
    else if (b < 15) { sa = GS_D1; ra = 32 * (b - 13); sb = GS_ONE; rb = 0; }
    else { sa = GS_D2; ra = 32 * (b - 15); sb = GS_ONE; rb = 0; }
}

__device__ __forceinline__ const __bf16 *stage_rows(const SurStage &T, int src)
{
    switch (src) {
    case GS_X: return &T.x[0][0];
    case GS_H0: return &T.h[0][0][0];
    case GS_H1: return &T.h[1][0][0];
    case GS_H2: return &T.h[2][0][0];
    case GS_D0: return &T.d[0][0][0];
    case GS_D1: return &T.d[1][0][0];
    case GS_D2: return &T.d[2][0][0];
    default: return &T.d4[0][0];
    }
}

// plain-parameter index of register r of gradient block b in lane (h, n); -1 if none
__device__ __forceinline__ int grad_block_index(int b, int r, int h, int n)
{
    const int m = sur_row(r, h);
    if (b < 2) return m < SUR_NOUT ? SUR_W4 + (32 * b + n) * SUR_NOUT + m : -1;
    if (b < 4) {
        const int o = 32 * (b - 2) + m;
        return n < SUR_NIN ? SUR_W1 + n * SUR_NH + o : (n == SUR_NIN ? SUR_B1 + o : -1);
    }
    if (b < 8) return SUR_W2 + (32 * ((b - 4) & 1) + n) * SUR_NH + 32 * ((b - 4) >> 1) + m;
    if (b < 12) return SUR_W3 + (32 * ((b - 8) & 1) + n) * SUR_NH + 32 * ((b - 8) >> 1) + m;
    if (n != 0) return -1;
    if (b == 12) return m < SUR_NOUT ? SUR_B4 + m : -1;
    if (b < 15) return SUR_B2 + 32 * (b - 13) + m;
    return SUR_B3 + 32 * (b - 15) + m;
}

// Each wave processes `nblk` blocks of 32 records.  Record of minibatch slot q
// (global index base + q): a SplitMix64 hash of it modulo n_data when
// `randomize`, else the index itself (slots past n_data contribute nothing).
// The loss is sum (y - t)^2 * scale, its gradient 2 (y - t) scale.  One
// partial (gradient, then loss) per workgroup.
__global__ __launch_bounds__(64 * SUR_TW)
void k_sur_grad(const uint4 *__restrict__ pk0, const float *__restrict__ data, int64_t n_data, int64_t base,
                int nblk, int randomize, uint64_t seed, float scale, float *__restrict__ partials)
{
    __shared__ __attribute__((aligned(16))) SurStage stages[SUR_TW];
    __shared__ float lred[SUR_TW];
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, h = lane >> 5, n = lane & 31;
    SurStage &S = stages[wave];
    constexpr int NACC = (SUR_GBLOCKS + SUR_TW - 1) / SUR_TW;
    f32x16 acc[NACC];
#pragma unroll
    for (int k = 0; k < NACC; ++k) acc[k] = f32x16_zero();
    bf16x8 ones;
#pragma unroll
    for (int i = 0; i < 8; ++i) ones[i] = (__bf16)1.f;
    float lsum = 0.f;
    for (int j = 0; j < nblk; ++j) {
        // re-read the weight fragments in every block instead of keeping all of
        // them live across the loop (they would take ~240 registers)
        const uint4 *pk = pk0;
        asm volatile("" : "+s"(pk));
        const int64_t q = base + ((int64_t)(blockIdx.x * SUR_TW + wave) * nblk + j) * 32 + n;
        int64_t idx = randomize ? (int64_t)(mix64(seed ^ (uint64_t)q) % (uint64_t)n_data) : q;
        const bool valid = idx < n_data;
        if (!valid) idx = 0;
        const float *rec = data + idx * SUR_REC;
        // ---- forward ----
        bf16x8 xb;
#pragma unroll
        for (int i = 0; i < 8; ++i) {
            const int k = 8 * h + i;
            const float v = !valid ? 0.f : (k < SUR_NIN ? rec[k] : (k == SUR_NIN ? 1.f : 0.f));
            xb[i] = (__bf16)v;
            S.x[k][n] = xb[i];
            S.x[16 + k][n] = (__bf16)0.f;
        }
        f32x16 z[2];
        bf16x8 a[4], ds[3][4];               // activations; SiLU'(z) of layers 1..3
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) z[mb] = mfma_bf16(sur_frag(pk, SF_A1 + mb, lane), xb, f32x16_zero());
#pragma unroll
        for (int l = 0; l < 3; ++l) {
            if (l == 1) sur_hidden(pk, SF_A2, SUR_BP2, lane, a, z);
            if (l == 2) sur_hidden(pk, SF_A3, SUR_BP3, lane, a, z);
#pragma unroll
            for (int c = 0; c < 4; ++c)
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const float zz = z[c >> 1][8 * (c & 1) + i], sg = sur_sigmoid(zz);
                    a[c][i] = (__bf16)(zz * sg);
                    ds[l][c][i] = (__bf16)(sg + zz * sg * (1.f - sg));
                    S.h[l][sur_unit(c, h, i)][n] = a[c][i];
                }
        }
        f32x16 z4 = sur_bias(pk, SUR_BP4, 0, lane);
#pragma unroll
        for (int c = 0; c < 4; ++c) z4 = mfma_bf16(sur_frag(pk, SF_A4 + c, lane), a[c], z4);
        // ---- output error ----
        bf16x8 d4b;
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = sur_row(r, h);
            float d = 0.f;
            if (row < SUR_NOUT && valid) {
                const float yv = row < SUR_NLIN ? z4[r] : sur_sigmoid(z4[r]);
                const float e = yv - rec[SUR_NIN + row];
                lsum += e * e;
                d = 2.f * scale * e;
                if (row >= SUR_NLIN) d *= yv * (1.f - yv);
            }
            const __bf16 dd = (__bf16)d;
            S.d4[row][n] = dd;
            if (r < 8) d4b[r] = dd;
        }
        // ---- back-propagation through the hidden layers (times SiLU') ----
        f32x16 gz[2];
        bf16x8 db[4];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) gz[mb] = mfma_bf16(sur_frag(pk, SF_A4B + mb, lane), d4b, f32x16_zero());
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                db[c][i] = (__bf16)(gz[c >> 1][8 * (c & 1) + i] * (float)ds[2][c][i]);
                S.d[2][sur_unit(c, h, i)][n] = db[c][i];
            }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            gz[mb] = f32x16_zero();
#pragma unroll
            for (int c = 0; c < 4; ++c) gz[mb] = mfma_bf16(sur_frag(pk, SF_A3B + mb * 4 + c, lane), db[c], gz[mb]);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                db[c][i] = (__bf16)(gz[c >> 1][8 * (c & 1) + i] * (float)ds[1][c][i]);
                S.d[1][sur_unit(c, h, i)][n] = db[c][i];
            }
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) {
            gz[mb] = f32x16_zero();
#pragma unroll
            for (int c = 0; c < 4; ++c) gz[mb] = mfma_bf16(sur_frag(pk, SF_A2B + mb * 4 + c, lane), db[c], gz[mb]);
        }
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int i = 0; i < 8; ++i)
                S.d[0][sur_unit(c, h, i)][n] = (__bf16)(gz[c >> 1][8 * (c & 1) + i] * (float)ds[0][c][i]);
        __syncthreads();
        // ---- gradient blocks of this wave: contraction over the workgroup's points ----
#pragma unroll
        for (int k = 0; k < NACC; ++k) {
            const int b = wave + SUR_TW * k;
            if (b < SUR_GBLOCKS) {
                int sa, ra, sb, rb;
                grad_block_src(b, sa, ra, sb, rb);
                for (int wv = 0; wv < SUR_TW; ++wv) {
                    const __bf16 *pa = stage_rows(stages[wv], sa) + (ra + n) * 32;
                    const __bf16 *pb = stage_rows(stages[wv], sb) + (rb + n) * 32;
#pragma unroll
                    for (int cs = 0; cs < 2; ++cs)
                        acc[k] = mfma_bf16(stage_frag(pa, cs, h), sb == GS_ONE ? ones : stage_frag(pb, cs, h), acc[k]);
                }
            }
        }
        __syncthreads();
    }
    // ---- this workgroup's partial: every parameter written by exactly one lane ----
    float *out = partials + (int64_t)blockIdx.x * (SUR_NPARAM + 1);
#pragma unroll
    for (int k = 0; k < NACC; ++k) {
        const int b = wave + SUR_TW * k;
        if (b < SUR_GBLOCKS)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int idx = grad_block_index(b, r, h, n);
                if (idx >= 0) out[idx] = acc[k][r];
            }
    }
    float l = lsum;
    for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
    if (lane == 0) lred[wave] = l;
    __syncthreads();
    if (threadIdx.x == 0) {
        float t = 0.f;
        for (int w = 0; w < SUR_TW; ++w) t += lred[w];
        out[SUR_NPARAM] = t;
    }
}

// Adam on the fixed-order sum of the workgroup partials; slot SUR_NPARAM of a
// partial is its loss, summed into loss_out
__global__ void k_sur_adam(const float *__restrict__ partials, int nparts, float *__restrict__ w,
                           float *__restrict__ m, float *__restrict__ v, float lr, float b1, float b2, float eps,
                           float bc1, float bc2, float *__restrict__ loss_out)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > SUR_NPARAM) return;
    float g = 0.f;
    for (int b = 0; b < nparts; ++b) g += partials[(int64_t)b * (SUR_NPARAM + 1) + p];
    if (p == SUR_NPARAM) {
        if (loss_out) *loss_out = g;
        return;
    }
    const float mm = b1 * m[p] + (1.f - b1) * g;
    const float vv = b2 * v[p] + (1.f - b2) * g * g;
    m[p] = mm;
    v[p] = vv;
    w[p] -= lr * (mm / bc1) / (sqrtf(vv / bc2) + eps);
}

// ---------------------------------------------------------------------------
// evaluation (the forward routine of the element kernel)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void k_sur_eval(const uint4 *__restrict__ pk, const float *__restrict__ x,
                                                  int64_t n, float *__restrict__ y)
{
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    float xi[SUR_NIN], yi[SUR_NOUT];
#pragma unroll
    for (int k = 0; k < SUR_NIN; ++k) xi[k] = i < n ? x[i * SUR_NIN + k] : 0.f;
    sur_forward_wave(pk, xi, yi);
    if (i < n)
#pragma unroll
        for (int k = 0; k < SUR_NOUT; ++k) y[i * SUR_NOUT + k] = yi[k];
}

// sum (y - t)^2 over records i0 .. i0+n-1, one partial per workgroup
__global__ __launch_bounds__(256) void k_sur_loss(const uint4 *__restrict__ pk, const float *__restrict__ data,
                                                  int64_t i0, int64_t n, double *__restrict__ partials)
{
    __shared__ double sh[4];
    const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    const float *rec = data + (i0 + (i < n ? i : 0)) * SUR_REC;
    float xi[SUR_NIN], yi[SUR_NOUT];
#pragma unroll
    for (int k = 0; k < SUR_NIN; ++k) xi[k] = i < n ? rec[k] : 0.f;
    sur_forward_wave(pk, xi, yi);
    double l = 0.0;
    if (i < n)
#pragma unroll
        for (int k = 0; k < SUR_NOUT; ++k) {
            const double e = (double)yi[k] - (double)rec[SUR_NIN + k];
            l += e * e;
        }
    for (int o = 32; o > 0; o >>= 1) l += __shfl_xor(l, o, 64);
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = l;
    __syncthreads();
    if (threadIdx.x == 0) partials[blockIdx.x] = sh[0] + sh[1] + sh[2] + sh[3];
}

// ---------------------------------------------------------------------------
// launchers
// ---------------------------------------------------------------------------
hipError_t launch_sur_pack(const float *w, void *pk, hipStream_t s)
{
    const int n = SF_COUNT * 64 + 5 * 64 * 16;
    hipLaunchKernelGGL(k_sur_pack, dim3((n + 255) / 256), dim3(256), 0, s, w, reinterpret_cast<uint4 *>(pk));
    return hipGetLastError();
}

hipError_t launch_sur_data(const PlyC<double> &P, double vol, uint64_t seed, int64_t p0, int64_t np, int n_inc,
                           float *out, hipStream_t s)
{
    if (np < 1 || n_inc < 1 || n_inc > 64) return hipErrorInvalidValue;
    const int64_t nb = (np + 127) / 128;
    hipLaunchKernelGGL(k_sur_data, dim3((unsigned)nb), dim3(128), 0, s, P, vol, seed, p0, np, n_inc, out);
    return hipGetLastError();
}

int sur_grad_blocks(int64_t batch, int nblk) { return (int)((batch + 32LL * SUR_TW * nblk - 1) / (32LL * SUR_TW * nblk)); }

hipError_t launch_sur_grad(const void *pk, const float *data, int64_t n_data, int64_t base, int64_t batch, int nblk,
                           int randomize, uint64_t seed, float scale, float *partials, hipStream_t s)
{
    const int nb = sur_grad_blocks(batch, nblk);
    hipLaunchKernelGGL(k_sur_grad, dim3(nb), dim3(64 * SUR_TW), 0, s, reinterpret_cast<const uint4 *>(pk), data,
                       n_data, base, nblk, randomize, seed, scale, partials);
    return hipGetLastError();
}

hipError_t launch_sur_adam(const float *partials, int nparts, float *w, float *m, float *v, float lr, float b1,
                           float b2, float eps, float bc1, float bc2, float *loss_out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sur_adam, dim3((SUR_NPARAM + 1 + 255) / 256), dim3(256), 0, s, partials, nparts, w, m, v,
                       lr, b1, b2, eps, bc1, bc2, loss_out);
    return hipGetLastError();
}

hipError_t launch_sur_eval(const void *pk, const float *x, int64_t n, float *y, hipStream_t s)
{
    const int64_t nb = (n + 255) / 256;
    hipLaunchKernelGGL(k_sur_eval, dim3((unsigned)(nb > 0 ? nb : 1)), dim3(256), 0, s,
                       reinterpret_cast<const uint4 *>(pk), x, n, y);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// FP32 gradient (vector units): the same loss and gradient as k_sur_grad with
// FP32 operands throughout, for a check against the FP64 reference at FP32
// accuracy and for training in single precision.  A workgroup of 256 lanes
// takes 16 points; lane t holds point t % 16 and units 4 (t / 16) .. +3 of
// each hidden layer; pre-activations, activations and back-propagated
// errors are staged in LDS as [unit][point]; the workgroup's partial gradient
// (summed over its points) and loss go to partials[block].
// ---------------------------------------------------------------------------
#define SG32_PTS 16

__device__ __forceinline__ float sg32_sigmoid(float z) { return 1.0f / (1.0f + expf(-z)); }

__global__ __launch_bounds__(256) void k_sur_grad32(const float *__restrict__ w, const float *__restrict__ data,
                                                    int64_t n, float scale, float *__restrict__ partials)
{
    __shared__ float X[SUR_NIN][SG32_PTS], T[SUR_NOUT][SG32_PTS];
    __shared__ float Z[3][SUR_NH][SG32_PTS], Hh[3][SUR_NH][SG32_PTS], D[3][SUR_NH][SG32_PTS];
    __shared__ float D4[SUR_NOUT][SG32_PTS], Lp[SUR_NOUT][SG32_PTS];
    const int t = threadIdx.x, p = t % SG32_PTS, g = t / SG32_PTS;
    const int64_t i0 = (int64_t)blockIdx.x * SG32_PTS;
    for (int q = t; q < SG32_PTS * SUR_REC; q += 256) {
        const int pp = q / SUR_REC, k = q % SUR_REC;
        const float v = i0 + pp < n ? data[(i0 + pp) * SUR_REC + k] : 0.f;
        if (k < SUR_NIN) X[k][pp] = v;
        else T[k - SUR_NIN][pp] = v;
    }
    __syncthreads();
    // forward: hidden layers
    const int wof[3] = {SUR_W1, SUR_W2, SUR_W3}, bof[3] = {SUR_B1, SUR_B2, SUR_B3};
    for (int l = 0; l < 3; ++l) {
        const int K = l == 0 ? SUR_NIN : SUR_NH;
        for (int j = 0; j < 4; ++j) {
            const int u = 4 * g + j;
            float z = w[bof[l] + u];
            for (int k = 0; k < K; ++k) z += w[wof[l] + k * SUR_NH + u] * (l == 0 ? X[k][p] : Hh[l - 1][k][p]);
            Z[l][u][p] = z;
            Hh[l][u][p] = z * sg32_sigmoid(z);
        }
        __syncthreads();
    }
    // output layer, loss and output errors (points past n contribute nothing)
    if (t < SUR_NOUT * SG32_PTS) {
        const int o = t / SG32_PTS, pp = t % SG32_PTS;
        float z = w[SUR_B4 + o];
        for (int k = 0; k < SUR_NH; ++k) z += w[SUR_W4 + k * SUR_NOUT + o] * Hh[2][k][pp];
        const float y = o < SUR_NLIN ? z : sg32_sigmoid(z);
        const float e = i0 + pp < n ? y - T[o][pp] : 0.f;
        Lp[o][pp] = e * e * scale;
        // sigmoid'(z) = s(z) s(-z): 1 - s(z) is formed as s(-z), without cancellation
        D4[o][pp] = 2.0f * e * scale * (o < SUR_NLIN ? 1.0f : y * sg32_sigmoid(-z));
    }
    __syncthreads();
    // back-propagation through layers 3, 2, 1
    for (int l = 2; l >= 0; --l) {
        for (int j = 0; j < 4; ++j) {
            const int k = 4 * g + j;
            float a = 0.f;
            if (l == 2) {
                for (int o = 0; o < SUR_NOUT; ++o) a += w[SUR_W4 + k * SUR_NOUT + o] * D4[o][p];
            } else {
                const int wn = l == 1 ? SUR_W3 : SUR_W2;
                for (int u = 0; u < SUR_NH; ++u) a += w[wn + k * SUR_NH + u] * D[l + 1][u][p];
            }
            const float z = Z[l][k][p], sg = sg32_sigmoid(z);
            D[l][k][p] = a * (sg + z * sg * sg32_sigmoid(-z));     // SiLU'(z), 1 - s(z) as s(-z)
        }
        __syncthreads();
    }
    // partial gradient of this workgroup's points, and its loss
    float *out = partials + (size_t)blockIdx.x * (SUR_NPARAM + 1);
    for (int q = t; q <= SUR_NPARAM; q += 256) {
        float v = 0.f;
        if (q < SUR_B1) {
            const int k = q / SUR_NH, u = q % SUR_NH;
            for (int pp = 0; pp < SG32_PTS; ++pp) v += X[k][pp] * D[0][u][pp];
        } else if (q < SUR_W2) {
            for (int pp = 0; pp < SG32_PTS; ++pp) v += D[0][q - SUR_B1][pp];
        } else if (q < SUR_B2) {
            const int i = (q - SUR_W2) / SUR_NH, u = (q - SUR_W2) % SUR_NH;
            for (int pp = 0; pp < SG32_PTS; ++pp) v += Hh[0][i][pp] * D[1][u][pp];
        } else if (q < SUR_W3) {
            for (int pp = 0; pp < SG32_PTS; ++pp) v += D[1][q - SUR_B2][pp];
        } else if (q < SUR_B3) {
            const int i = (q - SUR_W3) / SUR_NH, u = (q - SUR_W3) % SUR_NH;
            for (int pp = 0; pp < SG32_PTS; ++pp) v += Hh[1][i][pp] * D[2][u][pp];
        } else if (q < SUR_W4) {
            for (int pp = 0; pp < SG32_PTS; ++pp) v += D[2][q - SUR_B3][pp];
        } else if (q < SUR_B4) {
            const int k = (q - SUR_W4) / SUR_NOUT, o = (q - SUR_W4) % SUR_NOUT;
            for (int pp = 0; pp < SG32_PTS; ++pp) v += Hh[2][k][pp] * D4[o][pp];
        } else if (q < SUR_NPARAM) {
            for (int pp = 0; pp < SG32_PTS; ++pp) v += D4[q - SUR_B4][pp];
        } else {
            for (int o = 0; o < SUR_NOUT; ++o)
                for (int pp = 0; pp < SG32_PTS; ++pp) v += Lp[o][pp];
        }
        out[q] = v;
    }
}

int sur_grad32_blocks(int64_t n) { return (int)((n + SG32_PTS - 1) / SG32_PTS); }

hipError_t launch_sur_grad32(const float *w, const float *data, int64_t n, float scale, float *partials,
                             hipStream_t s)
{
    if (n < 1) return hipErrorInvalidValue;
    hipLaunchKernelGGL(k_sur_grad32, dim3((unsigned)sur_grad32_blocks(n)), dim3(256), 0, s, w, data, n, scale,
                       partials);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// gradient without allocation: a fixed device array holds the packed network,
// the interleaved records and the workgroup partials
// ---------------------------------------------------------------------------
__global__ void k_sur_interleave(const float *__restrict__ x, const float *__restrict__ t, int64_t n,
                                 float *__restrict__ rec)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n * SUR_REC) return;
    const int64_t p = i / SUR_REC;
    const int k = (int)(i - p * SUR_REC);
    rec[i] = k < SUR_NIN ? x[p * SUR_NIN + k] : t[p * SUR_NOUT + (k - SUR_NIN)];
}

// parameter p: the partials of the nparts workgroups summed in workgroup order
// in FP64 (the order and precision of the host reduction of pdn_surrogate_grad)
__global__ void k_sur_grad_reduce(const float *__restrict__ part, int nparts, double count,
                                  float *__restrict__ grad, double *__restrict__ loss)
{
    const int p = blockIdx.x * blockDim.x + threadIdx.x;
    if (p > SUR_NPARAM) return;
    double g = 0.0;
    for (int b = 0; b < nparts; ++b) g += (double)part[(size_t)b * (SUR_NPARAM + 1) + p];
    if (p < SUR_NPARAM) grad[p] = (float)g;
    else if (loss) *loss = g / count;
}

hipError_t launch_sur_interleave(const float *x, const float *t, int64_t n, float *rec, hipStream_t s)
{
    const int64_t nb = (n * SUR_REC + 255) / 256;
    hipLaunchKernelGGL(k_sur_interleave, dim3((unsigned)nb), dim3(256), 0, s, x, t, n, rec);
    return hipGetLastError();
}

hipError_t launch_sur_grad_reduce(const float *part, int nparts, double count, float *grad, double *loss,
                                  hipStream_t s)
{
    hipLaunchKernelGGL(k_sur_grad_reduce, dim3((SUR_NPARAM + 1 + 255) / 256), dim3(256), 0, s, part, nparts, count,
                       grad, loss);
    return hipGetLastError();
}

int sur_loss_blocks(int64_t n) { return (int)((n + 255) / 256); }

hipError_t launch_sur_loss(const void *pk, const float *data, int64_t i0, int64_t n, double *partials, hipStream_t s)
{
    hipLaunchKernelGGL(k_sur_loss, dim3((unsigned)sur_loss_blocks(n)), dim3(256), 0, s,
                       reinterpret_cast<const uint4 *>(pk), data, i0, n, partials);
    return hipGetLastError();
}

}  // namespace pdn

// Scratch of pdn_surrogate_grad_noalloc: one copy per device, held until the
// process ends.  Host code never passes this name to a kernel (on the host it
// is only a stand-in for the symbol); it uses the device address that
// hipGetSymbolAddress returns for the current device.
static __device__ __align__(256) unsigned char scratch[PDN_SUR_NOALLOC_SCRATCH_BYTES];

namespace pdn {
namespace {
std::mutex g_scratch_mu;
void *g_scratch_ptr[PDN_SUR_NOALLOC_MAX_DEVICES];
}  // namespace

hipError_t sur_noalloc_scratch(int device, void **out)
{
    *out = nullptr;
    if (device < 0 || device >= PDN_SUR_NOALLOC_MAX_DEVICES) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));   // device must be current
        if (e != hipSuccess) return e;
        if (!p) return hipErrorInvalidSymbol;
        g_scratch_ptr[device] = p;
    }
    *out = g_scratch_ptr[device];
    return hipSuccess;
}
}  // namespace pdn
