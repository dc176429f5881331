// pdn_mlp.h -- constitutive surrogate network on the gfx950 matrix cores
// (device code, internal).
//
// The network 10 -> 64 -> 64 -> 64 -> 10 (SiLU hidden layers) stands in for
// the intralaminar update of Section 2.3.1.  Inputs: the six material-frame
// strains scaled by their onset strains X_k / E_k and the four damage
// thresholds as s = 1 - 1/r; outputs: the six stresses over X_k and the four
// new s through a logistic sigmoid.
//
// Arithmetic: v_mfma_f32_32x32x16_bf16 (bf16 operands, fp32 accumulation).
// Layers are evaluated transposed, Z^T = W^T X^T, with the 32 Gauss points of
// one block as the 32 columns.  For this instruction lane l holds
//   A[m = l%32][k = 8(l/32) + i], B[k = 8(l/32) + i][n = l%32], i = 0..7,
//   D[m = 8(r/4) + 4(l/32) + r%4][n = l%32], r = 0..15,
// so registers 8c'..8c'+7 of one 32-row output block are exactly the B
// operand of the next layer's k-chunk c' of that block, up to a fixed
// permutation of k that the packed weights absorb.  Activations never leave
// the registers.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pdn {

typedef __attribute__((ext_vector_type(8))) __bf16 bf16x8;
typedef __attribute__((ext_vector_type(16))) float f32x16;

// plain parameter vector (fp32, W stored [in][out])
#define SUR_NIN 10
#define SUR_NH 64
#define SUR_NOUT 10
#define SUR_NLIN 6                      // stress outputs; the last four pass a sigmoid
#define SUR_W1 0                        // [10][64]
#define SUR_B1 640
#define SUR_W2 704                      // [64][64]
#define SUR_B2 4800
#define SUR_W3 4864                     // [64][64]
#define SUR_B3 8960
#define SUR_W4 9024                     // [64][10]
#define SUR_B4 9664
#define SUR_NPARAM 9674

// packed network: 16-byte A-operand fragments, 64 lanes each, then the biases
// of layers 2-4 in accumulator order.  Forward: A1 (2: output block; k = 10 is
// the bias of layer 1, fed by a constant input 1), A2, A3 (8: block * 4 +
// k-chunk), A4 (4: k-chunk).  Backward (transposed weights): A4B (2), A3B, A2B (8).
enum { SF_A1 = 0, SF_A2 = 2, SF_A3 = 10, SF_A4 = 18, SF_A4B = 22, SF_A3B = 24, SF_A2B = 32, SF_COUNT = 40 };
#define SUR_FRAG_BYTES (40 * 64 * 16)          // SF_COUNT fragments
// bias packs (floats, [block][lane][16]): BP2 (2 blocks), BP3 (2), BP4 (1)
#define SUR_BP2 0
#define SUR_BP3 (2 * 64 * 16)
#define SUR_BP4 (4 * 64 * 16)
#define SUR_PACK_BYTES (SUR_FRAG_BYTES + 5 * 64 * 16 * 4)
static_assert(SUR_FRAG_BYTES == SF_COUNT * 64 * 16, "fragment count");

// hidden unit fed to element i of lane half h in k-chunk c (the permutation above)
__host__ __device__ __forceinline__ int sur_unit(int c, int h, int i)
{
    return 32 * (c >> 1) + 8 * (2 * (c & 1) + (i >> 2)) + 4 * h + (i & 3);
}
// output row of accumulator register r in lane half h
__host__ __device__ __forceinline__ int sur_row(int r, int h) { return 8 * (r >> 2) + 4 * h + (r & 3); }

__device__ __forceinline__ f32x16 mfma_bf16(const bf16x8 &a, const bf16x8 &b, const f32x16 &c)
{
    return __builtin_amdgcn_mfma_f32_32x32x16_bf16(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ bf16x8 sur_frag(const uint4 *__restrict__ pk, int f, int lane)
{
    return __builtin_bit_cast(bf16x8, pk[f * 64 + lane]);
}

__device__ __forceinline__ f32x16 sur_bias(const uint4 *__restrict__ pk, int off, int blk, int lane)
{
    const float4 *b = reinterpret_cast<const float4 *>(reinterpret_cast<const char *>(pk) + SUR_FRAG_BYTES) +
                      (off + (blk * 64 + lane) * 16) / 4;
    f32x16 c;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
        const float4 v = b[q];
        c[4 * q] = v.x; c[4 * q + 1] = v.y; c[4 * q + 2] = v.z; c[4 * q + 3] = v.w;
    }
    return c;
}

__device__ __forceinline__ f32x16 f32x16_zero()
{
    f32x16 c;
#pragma unroll
    for (int r = 0; r < 16; ++r) c[r] = 0.f;
    return c;
}

__device__ __forceinline__ float sur_sigmoid(float z) { return __builtin_amdgcn_rcpf(1.f + __expf(-z)); }
__device__ __forceinline__ float sur_silu(float z) { return z * sur_sigmoid(z); }

// next layer's k-chunk (0/1 within an output block) from SiLU of accumulator registers 8c'..8c'+7
__device__ __forceinline__ bf16x8 sur_act_chunk(const f32x16 &z, int cc)
{
    bf16x8 b;
#pragma unroll
    for (int i = 0; i < 8; ++i) b[i] = (__bf16)sur_silu(z[8 * cc + i]);
    return b;
}

// one hidden layer (64 -> 64) on a block of 32 points: a[c] are its input chunks
__device__ __forceinline__ void sur_hidden(const uint4 *__restrict__ pk, int frag, int bias_off, int lane,
                                           const bf16x8 a[4], f32x16 z[2])
{
#pragma unroll
    for (int mb = 0; mb < 2; ++mb) {
        z[mb] = sur_bias(pk, bias_off, mb, lane);
#pragma unroll
        for (int c = 0; c < 4; ++c) z[mb] = mfma_bf16(sur_frag(pk, frag + mb * 4 + c, lane), a[c], z[mb]);
    }
}

// Forward pass of the wave's 64 points, one per lane: x are this lane's ten
// inputs, y receives its ten outputs.  All 64 lanes of the wave must execute
// it together (operands are exchanged across lanes).
__device__ __forceinline__ void sur_forward_wave(const uint4 *__restrict__ pk, const float x[SUR_NIN],
                                                 float y[SUR_NOUT])
{
    const int lane = threadIdx.x & 63, h = lane >> 5;
    bf16x8 lo, hi;
#pragma unroll
    for (int i = 0; i < 8; ++i) lo[i] = (__bf16)x[i];
    hi[0] = (__bf16)x[8];
    hi[1] = (__bf16)x[9];
    hi[2] = (__bf16)1.f;                 // constant input: bias of the first layer
#pragma unroll
    for (int i = 3; i < 8; ++i) hi[i] = (__bf16)0.f;
    // block 0 holds points 0..31 (lanes 0..31), block 1 points 32..63: the
    // upper lane half supplies k = 8..15, so each lane swaps one half with
    // its partner lane ^ 32
    const uint4 snd = __builtin_bit_cast(uint4, h ? lo : hi);
    uint4 rcv;
    rcv.x = __shfl_xor(snd.x, 32, 64);
    rcv.y = __shfl_xor(snd.y, 32, 64);
    rcv.z = __shfl_xor(snd.z, 32, 64);
    rcv.w = __shfl_xor(snd.w, 32, 64);
    const bf16x8 other = __builtin_bit_cast(bf16x8, rcv);
    f32x16 out[2];
#pragma unroll
    for (int nb = 0; nb < 2; ++nb) {
        const bf16x8 xb = nb == 0 ? (h ? other : lo) : (h ? hi : other);
        f32x16 z[2];
        bf16x8 a[4];
#pragma unroll
        for (int mb = 0; mb < 2; ++mb) z[mb] = mfma_bf16(sur_frag(pk, SF_A1 + mb, lane), xb, f32x16_zero());
#pragma unroll
        for (int c = 0; c < 4; ++c) a[c] = sur_act_chunk(z[c >> 1], c & 1);
        sur_hidden(pk, SF_A2, SUR_BP2, lane, a, z);
#pragma unroll
        for (int c = 0; c < 4; ++c) a[c] = sur_act_chunk(z[c >> 1], c & 1);
        sur_hidden(pk, SF_A3, SUR_BP3, lane, a, z);
#pragma unroll
        for (int c = 0; c < 4; ++c) a[c] = sur_act_chunk(z[c >> 1], c & 1);
        f32x16 o = sur_bias(pk, SUR_BP4, 0, lane);
#pragma unroll
        for (int c = 0; c < 4; ++c) o = mfma_bf16(sur_frag(pk, SF_A4 + c, lane), a[c], o);
        out[nb] = o;
    }
    // lane half 0 holds rows 0-3, 8, 9 and half 1 rows 4-7 of each column;
    // point l (< 32) is column l of block 0, point l (>= 32) column l-32 of block 1
    float s[6], r[6];
#pragma unroll
    for (int q = 0; q < 6; ++q) s[q] = h ? (q < 4 ? out[0][q] : 0.f) : out[1][q];
#pragma unroll
    for (int q = 0; q < 6; ++q) r[q] = __shfl_xor(s[q], 32, 64);
    if (h == 0) {
        y[0] = out[0][0]; y[1] = out[0][1]; y[2] = out[0][2]; y[3] = out[0][3];
        y[4] = r[0]; y[5] = r[1]; y[6] = r[2]; y[7] = r[3];
        y[8] = out[0][4]; y[9] = out[0][5];
    } else {
        y[0] = r[0]; y[1] = r[1]; y[2] = r[2]; y[3] = r[3];
        y[4] = out[1][0]; y[5] = out[1][1]; y[6] = out[1][2]; y[7] = out[1][3];
        y[8] = r[4]; y[9] = r[5];
    }
#pragma unroll
    for (int q = SUR_NLIN; q < SUR_NOUT; ++q) y[q] = sur_sigmoid(y[q]);
}

}  // namespace pdn
