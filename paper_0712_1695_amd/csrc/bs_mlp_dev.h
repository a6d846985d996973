// bs_mlp_dev.h -- device code shared by the training kernels and the fused
// inference of the ray-tracing kernel: pair features, the BF16 MFMA tile and
// the network's forward pass (internal).
#pragma once

#include <hip/hip_runtime.h>

namespace bsk {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(16 * sizeof(float)))) float f32x16;

// --------------------------------------------------------------- features

__device__ __forceinline__ void sort4_desc(float &a, float &b, float &c, float &d)
{
#define BS_SWP(x, y)                                                                                               \
    {                                                                                                              \
        const float hi = fmaxf(x, y), lo = fminf(x, y);                                                            \
        x = hi;                                                                                                    \
        y = lo;                                                                                                    \
    }
    BS_SWP(a, b) BS_SWP(c, d) BS_SWP(a, c) BS_SWP(b, d) BS_SWP(b, c)
#undef BS_SWP
}

// a[4][3]: vertex positions relative to x; inc: incident flag.  Quotients
// are products with hardware reciprocals and reciprocal square roots (one
// unit in the last place).
__device__ inline void pair_features(const float (&a)[4][3], float hbar, bool inc, float *f)
{
    float c[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) c[k] = 0.25f * ((a[0][k] + a[1][k]) + (a[2][k] + a[3][k]));
    const float d2 = c[0] * c[0] + c[1] * c[1] + c[2] * c[2];
    const float id = __builtin_amdgcn_rsqf(d2), d = d2 * id;
    float hmax2 = 0.f, hmin2 = 3e38f;
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = i + 1; j < 4; ++j) {
            const float ex = a[j][0] - a[i][0], ey = a[j][1] - a[i][1], ez = a[j][2] - a[i][2];
            const float l2 = ex * ex + ey * ey + ez * ez;
            hmax2 = fmaxf(hmax2, l2);
            hmin2 = fminf(hmin2, l2);
        }
    const float ihT = __builtin_amdgcn_rsqf(hmax2), hT = hmax2 * ihT;
    const float ihmin = __builtin_amdgcn_rsqf(hmin2);
    // face volumes [a_p, a_q, a_r] (face f opposite vertex f, ascending p < q < r)
    float vol[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const int p = f == 0 ? 1 : 0, q = f <= 1 ? 2 : 1, r = f <= 2 ? 3 : 2;
        const float nx = a[q][1] * a[r][2] - a[q][2] * a[r][1];
        const float ny = a[q][2] * a[r][0] - a[q][0] * a[r][2];
        const float nz = a[q][0] * a[r][1] - a[q][1] * a[r][0];
        vol[f] = a[p][0] * nx + a[p][1] * ny + a[p][2] * nz;
    }
    const float D = (vol[0] - vol[1]) + (vol[2] - vol[3]); // signed 6V
    const float iD = __builtin_amdgcn_rcpf(D);
    const float s = hT * id;
    float l0 = vol[0] * iD * s, l1 = -vol[1] * iD * s, l2 = vol[2] * iD * s, l3 = -vol[3] * iD * s;
    sort4_desc(l0, l1, l2, l3);
    // outward unit normals, cosines with -c/d, distances to the face planes
    float cs[4], dmin = 3e38f;
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const int p = f == 0 ? 1 : 0, q = f <= 1 ? 2 : 1, r = f <= 2 ? 3 : 2;
        const float e1x = a[q][0] - a[p][0], e1y = a[q][1] - a[p][1], e1z = a[q][2] - a[p][2];
        const float e2x = a[r][0] - a[p][0], e2y = a[r][1] - a[p][1], e2z = a[r][2] - a[p][2];
        float nx = e1y * e2z - e1z * e2y, ny = e1z * e2x - e1x * e2z, nz = e1x * e2y - e1y * e2x;
        // orient away from the opposite vertex f
        const float o = nx * (a[f][0] - a[p][0]) + ny * (a[f][1] - a[p][1]) + nz * (a[f][2] - a[p][2]);
        const float inv = (o > 0.f ? -1.f : 1.f) * __builtin_amdgcn_rsqf(nx * nx + ny * ny + nz * nz);
        nx *= inv;
        ny *= inv;
        nz *= inv;
        cs[f] = -(nx * c[0] + ny * c[1] + nz * c[2]) * id;
        // plane through a_p; x is the origin
        dmin = fminf(dmin, fabsf(nx * a[p][0] + ny * a[p][1] + nz * a[p][2]));
    }
    sort4_desc(cs[0], cs[1], cs[2], cs[3]);
    f[0] = d * ihT;
    f[1] = d * __builtin_amdgcn_rcpf(hbar);
    f[2] = hT * ihmin;
    f[3] = hbar * id;
    f[4] = l0;
    f[5] = l1;
    f[6] = l2;
    f[7] = l3;
    f[8] = cs[0];
    f[9] = cs[1];
    f[10] = cs[2];
    f[11] = cs[3];
    f[12] = inc ? 1.f : 0.f;
    f[13] = fabsf(D) * (ihT * ihT * ihT);
    f[14] = dmin * ihT;
    f[15] = 1.f;
}

// --------------------------------------------------------------- MFMA tiles
//
// v_mfma_f32_32x32x16_bf16 operand layout (lane l, 8 values s = 0..7):
//   A (32 x 16): A[l % 32][8 (l / 32) + s]      B (16 x 32): B[8 (l / 32) + s][l % 32]
//   C (32 x 32), 16 values r: C[8 (r / 4) + 4 (l / 32) + r % 4][l % 32]
// Strided element access lets one helper serve plain and transposed operands.

__device__ __forceinline__ __bf16 to_bf16(float x) { return (__bf16)x; }

template <typename TA, typename TB>
__device__ __forceinline__ void mfma_tile(f32x16 &acc, const TA *A, int sar, int sak, const TB *B, int sbk, int sbc,
                                          int lane)
{
    bf16x8 av, bv;
    const int r = lane & 31, kb = 8 * (lane >> 5);
#pragma unroll
    for (int s = 0; s < 8; ++s) {
        av[s] = (__bf16)A[r * sar + (kb + s) * sak];
        bv[s] = (__bf16)B[(kb + s) * sbk + r * sbc];
    }
    acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
}

__device__ __forceinline__ int tile_row(int lane, int r) { return 8 * (r >> 2) + 4 * (lane >> 5) + (r & 3); }

struct MlpLds {
    __bf16 x[64][16];   // standardised features
    __bf16 a1[64][64];  // relu(z1)
    __bf16 a2[64][64];  // relu(z2)
    __bf16 g[64][64];   // backprop buffer (dz2 / dz1)
    __bf16 d3[64][32];  // dz3 (4 columns used), zero padded to a full B tile
    float z3[64][4];
    unsigned long long m1[64], m2[64]; // relu masks of z1, z2 (bit j: unit j > 0)
    float red[64];
};

__device__ __forceinline__ float wave_sum_f(float v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// Forward of 64 rows into L (x already staged): L needs x, a1, a2, z3.
template <typename LDS>
__device__ void mlp_forward_tile(LDS &L, const __bf16 *W1, const __bf16 *b1, const __bf16 *W2, const __bf16 *b2,
                                 const __bf16 *W3, const __bf16 *b3, int lane)
{
    // layer 1: [64 x 16] x [16 x 64]
    for (int rt = 0; rt < 2; ++rt)
        for (int ct = 0; ct < 2; ++ct) {
            f32x16 acc = {};
            mfma_tile(acc, &L.x[32 * rt][0], 16, 1, W1 + 32 * ct, 64, 1, lane);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 32 * rt + tile_row(lane, r), col = 32 * ct + (lane & 31);
                const float z = acc[r] + (float)b1[col];
                L.a1[row][col] = to_bf16(fmaxf(z, 0.f));
            }
        }
    __syncthreads();
    // layer 2: [64 x 64] x [64 x 64]
    for (int rt = 0; rt < 2; ++rt)
        for (int ct = 0; ct < 2; ++ct) {
            f32x16 acc = {};
#pragma unroll
            for (int kt = 0; kt < 4; ++kt)
                mfma_tile(acc, &L.a1[32 * rt][16 * kt], 64, 1, W2 + (16 * kt) * 64 + 32 * ct, 64, 1, lane);
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 32 * rt + tile_row(lane, r), col = 32 * ct + (lane & 31);
                const float z = acc[r] + (float)b2[col];
                L.a2[row][col] = to_bf16(fmaxf(z, 0.f));
            }
        }
    __syncthreads();
    // layer 3: [64 x 64] x [64 x 4] (columns 4..31 of the tile unused)
    for (int rt = 0; rt < 2; ++rt) {
        f32x16 acc = {};
        const int col = lane & 31;
        // B columns beyond 3 read column 0 and are discarded
        const int cc = col < 4 ? col : 0;
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
            bf16x8 av, bv;
            const int r = lane & 31, kb = 8 * (lane >> 5);
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                av[s] = L.a2[32 * rt + r][16 * kt + kb + s];
                bv[s] = W3[(16 * kt + kb + s) * 4 + cc];
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
        }
        if (col < 4) {
#pragma unroll
            for (int r = 0; r < 16; ++r) L.z3[32 * rt + tile_row(lane, r)][col] = acc[r] + (float)b3[col];
        }
    }
    __syncthreads();
}


// ------------------------------------------------- fused inference network
//
// The ray-tracing kernels run the network on the pairs of one node, 64 at a
// time, with every layer transposed (rows = units, columns = pairs):
//   Z1^T = W1^T X^T,  Z2^T = W2^T relu(Z1)^T,  Z3^T = W3^T relu(Z2)^T.
// A 32 x 32 output tile leaves lane l holding units 8j + 4(l/32) + i
// (j, i < 4) of pair l % 32; that is the B operand of the next layer once
// the K index k = 8h + s of k-tile kt (lane half h = l/32) is mapped to the
// unit
//   U(kt, h, s) = 32 (kt/2) + 8 (2 (kt%2) + s/4) + 4 h + s%4,
// so activations never leave registers.  The weights are repacked on the
// host into these A-operand vectors (one 16-byte load per lane and MFMA).
struct PackedNet {
    bf16x8 w1[2][64];    // layer 1, [row tile][lane]: W1[8(l/32) + s][32 rt + l%32]
    bf16x8 w2[2][4][64]; // layer 2, [row tile][k tile][lane]: W2[U(kt, l/32, s)][32 rt + l%32]
    bf16x8 w3[4][64];    // layer 3, [k tile][lane]: W3[U(kt, l/32, s)][l%32] for l%32 < 4, else 0
    float b1[2][2][16];  // bias of output register r: [row tile][l/32][r] = b1[32 rt + 8(r/4) + 4(l/32) + r%4]
    float b2[2][2][16];
    float b3[4];
    float mu[16], isg[16];
};

__device__ __forceinline__ int packed_unit(int kt, int h, int s) { return 32 * (kt >> 1) + 8 * (2 * (kt & 1) + (s >> 2)) + 4 * h + (s & 3); }

// Logits of 64 pairs: xb[p] = standardised features of pair p (BF16); the
// logits of pair p land in zs[p].  Every lane of the wave takes part.
__device__ __forceinline__ void mlp_forward_packed(const PackedNet *__restrict__ W, const __bf16 (*xb)[16],
                                                   float (*zs)[4], int lane)
{
    // both column tiles (pairs 0..31, 32..63) per weight vector, so that each
    // weight vector is used as soon as it is loaded
    const int h = lane >> 5, col = lane & 31;
    bf16x8 xv[2];
#pragma unroll
    for (int ct = 0; ct < 2; ++ct) xv[ct] = *(const bf16x8 *)&xb[32 * ct + col][8 * h];
    bf16x8 a1[2][4];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        const bf16x8 w = W->w1[rt][lane];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) {
            f32x16 c = {};
            c = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, xv[ct], c, 0, 0, 0);
#pragma unroll
            for (int r = 0; r < 16; ++r)
                a1[ct][2 * rt + (r >> 3)][r & 7] = (__bf16)fmaxf(c[r] + W->b1[rt][h][r], 0.f);
        }
    }
    bf16x8 a2[2][4];
#pragma unroll
    for (int rt = 0; rt < 2; ++rt) {
        f32x16 c[2] = {{}, {}};
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
            const bf16x8 w = W->w2[rt][kt][lane];
#pragma unroll
            for (int ct = 0; ct < 2; ++ct) c[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, a1[ct][kt], c[ct], 0, 0, 0);
        }
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int r = 0; r < 16; ++r)
                a2[ct][2 * rt + (r >> 3)][r & 7] = (__bf16)fmaxf(c[ct][r] + W->b2[rt][h][r], 0.f);
    }
    f32x16 c[2] = {{}, {}};
#pragma unroll
    for (int kt = 0; kt < 4; ++kt) {
        const bf16x8 w = W->w3[kt][lane];
#pragma unroll
        for (int ct = 0; ct < 2; ++ct) c[ct] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(w, a2[ct][kt], c[ct], 0, 0, 0);
    }
    if (h == 0) {
#pragma unroll
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int r = 0; r < 4; ++r) zs[32 * ct + col][r] = c[ct][r] + W->b3[r];
    }
}

// LDS of the fused inference: staged features and logits of one batch.
struct InferLds {
    __bf16 x[64][16];
    float z3[64][4];
};

} // namespace bsk
