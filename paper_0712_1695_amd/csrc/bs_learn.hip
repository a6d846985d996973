// bs_learn.hip -- learned rule selector: pair features, labels from the
// method itself, and the 16-64-64-4 network's BF16-MFMA training and
// inference kernels (gfx950).
//
// Features of a pair (node x, tetrahedron T with vertices v_j, a_j = v_j - x),
// all scale-free; c = centroid - x, d = |c|, h_T / h_min the longest /
// shortest edge, 6V the absolute triple product of the edges, lambda_j the
// barycentric coordinates of x, n_f the outward unit normal of face f:
//   f0 = d / h_T          f1 = d / hbar        f2 = h_T / h_min
//   f3 = hbar / d         f4..f7 = lambda_j h_T / d, sorted descending
//   f8..f11 = n_f . (-c / d), sorted descending
//   f12 = incident flag   f13 = 6V / h_T^3     f14 = min_f dist(x, plane f) / h_T
//   f15 = 1
// Labels (Introduction: Gauss rules serve distant elements; Section 2.1: ray
// tracing for the rest): the cheapest Gauss rule (1, 4, 11 points) whose
// relative error against a high-accuracy value of the pair's integral is
// within tau, else ray tracing.  The high-accuracy value is the exact radial
// integral over the signed cones from x to the four faces (linear vorticity
// integrates exactly along each radius), with a collapsed Gauss rule on each
// face, in FP64.
//
// Network (BF16 weights and activations, FP32 accumulation on the matrix
// cores): z1 = xs W1 + b1, a1 = relu(z1), z2 = a1 W2 + b2, a2 = relu(z2),
// z3 = a2 W3 + b3; xs = (x - mu) * inv_sigma.  Training minimises the
// class-weighted softmax cross-entropy with Adam on FP32 master weights.
#include "bs_internal.h"
#include "bs_learn.h"
#include "bs_mlp_dev.h"

#include <hip/hip_runtime.h>

namespace bsk {

// --------------------------------------------------------------- labels

// exact velocity of one tet at the origin (vertices a[j] relative to x,
// vorticity w[j]) by the signed-cone decomposition; tri: collapsed Gauss rule
// on the reference triangle (u, v, weight), nq points.
__device__ void cone_reference(const double (&a)[4][3], const double (&w)[4][3], const double *tri, int nq,
                               double *out)
{
    // vorticity extended to x: barycentric weights of the origin
    double vol[4];
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const int p = f == 0 ? 1 : 0, q = f <= 1 ? 2 : 1, r = f <= 2 ? 3 : 2;
        const double nx = a[q][1] * a[r][2] - a[q][2] * a[r][1];
        const double ny = a[q][2] * a[r][0] - a[q][0] * a[r][2];
        const double nz = a[q][0] * a[r][1] - a[q][1] * a[r][0];
        vol[f] = a[p][0] * nx + a[p][1] * ny + a[p][2] * nz;
    }
    const double D = (vol[0] - vol[1]) + (vol[2] - vol[3]);
    const double lam[4] = {vol[0] / D, -vol[1] / D, vol[2] / D, -vol[3] / D};
    double wx[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) wx[k] = lam[0] * w[0][k] + lam[1] * w[1][k] + lam[2] * w[2][k] + lam[3] * w[3][k];
    double acc[3] = {0.0, 0.0, 0.0};
    for (int f = 0; f < 4; ++f) {
        const int p = f == 0 ? 1 : 0, q = f <= 1 ? 2 : 1, r = f <= 2 ? 3 : 2;
        double e1[3], e2[3], n[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) {
            e1[k] = a[q][k] - a[p][k];
            e2[k] = a[r][k] - a[p][k];
        }
        n[0] = e1[1] * e2[2] - e1[2] * e2[1];
        n[1] = e1[2] * e2[0] - e1[0] * e2[2];
        n[2] = e1[0] * e2[1] - e1[1] * e2[0];
        const double area2 = sqrt(n[0] * n[0] + n[1] * n[1] + n[2] * n[2]);
        // signed distance of x (origin) from the plane, and of the opposite vertex
        const double dx = -(n[0] * a[p][0] + n[1] * a[p][1] + n[2] * a[p][2]) / area2;
        const double dv = (n[0] * (a[f][0] - a[p][0]) + n[1] * (a[f][1] - a[p][1]) + n[2] * (a[f][2] - a[p][2])) /
                          area2;
        if (dx == 0.0) continue;
        const double sg = ((dx > 0) == (dv > 0)) ? 1.0 : -1.0;
        const double hF = fabs(dx);
        double fa[3] = {0.0, 0.0, 0.0};
        for (int qd = 0; qd < nq; ++qd) {
            const double u = tri[3 * qd], v = tri[3 * qd + 1], wt = tri[3 * qd + 2];
            const double l0 = 1.0 - u - v;
            double P[3], W[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                P[k] = a[p][k] + u * e1[k] + v * e2[k];
                W[k] = 0.5 * (wx[k] + (l0 * w[p][k] + u * w[q][k] + v * w[r][k]));
            }
            const double R2 = P[0] * P[0] + P[1] * P[1] + P[2] * P[2];
            const double s = wt * hF / (R2 * sqrt(R2));
            fa[0] += s * (P[1] * W[2] - P[2] * W[1]);
            fa[1] += s * (P[2] * W[0] - P[0] * W[2]);
            fa[2] += s * (P[0] * W[1] - P[1] * W[0]);
        }
#pragma unroll
        for (int k = 0; k < 3; ++k) acc[k] += sg * area2 * fa[k];
    }
    const double c = 1.0 / (4.0 * M_PI);
#pragma unroll
    for (int k = 0; k < 3; ++k) out[k] = acc[k] * c;
}

// Gauss rule value in FP64: v = sum_q w_q |T| / 4pi (p_q x omega_q) / |p_q|^3
// for x at the origin (r = x - p = -p: (W x r) = -(W x p) = p x W).
__device__ void gauss_value(const double (&a)[4][3], const double (&w)[4][3], const float *lam, const float *wq,
                            int npts, double vol, double *out)
{
    out[0] = out[1] = out[2] = 0.0;
    for (int q = 0; q < npts; ++q) {
        double p[3] = {0, 0, 0}, o[3] = {0, 0, 0};
#pragma unroll
        for (int j = 0; j < 4; ++j)
#pragma unroll
            for (int k = 0; k < 3; ++k) {
                p[k] += (double)lam[4 * q + j] * a[j][k];
                o[k] += (double)lam[4 * q + j] * w[j][k];
            }
        const double R2 = p[0] * p[0] + p[1] * p[1] + p[2] * p[2];
        const double f = (double)wq[q] * vol / (4.0 * M_PI * R2 * sqrt(R2));
        out[0] += f * (p[1] * o[2] - p[2] * o[1]);
        out[1] += f * (p[2] * o[0] - p[0] * o[2]);
        out[2] += f * (p[0] * o[1] - p[1] * o[0]);
    }
}

__global__ void __launch_bounds__(64) k_label(DevMesh m, const int2 *__restrict__ pairs, int n, float hbar,
                                              const double *__restrict__ tri, int nq, const float *__restrict__ rules,
                                              double tau, float *__restrict__ feats, int8_t *__restrict__ labels,
                                              float *__restrict__ errs)
{
    const int k = blockIdx.x * 64 + threadIdx.x;
    if (k >= n) return;
    const int2 pr = pairs[k];
    const int self = pr.x, t = pr.y;
    const int4 id4 = m.tid[t];
    const int id[4] = {id4.x, id4.y, id4.z, id4.w};
    float af[4][3];
    double ad[4][3], wd[4][3];
    bool inc = false;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        inc |= id[j] == self;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float vh = m.xh[c * m.npad + id[j]], vl = m.xl[c * m.npad + id[j]];
            const float xh = m.xh[c * m.npad + self], xl = m.xl[c * m.npad + self];
            af[j][c] = (vh - xh) + (vl - xl);
            ad[j][c] = ((double)vh + (double)vl) - ((double)xh + (double)xl);
            wd[j][c] = (double)m.om[c * m.npad + id[j]];
        }
    }
    float f[16];
    pair_features(af, hbar, inc, f);
#pragma unroll
    for (int q = 0; q < 16; ++q) feats[(size_t)k * 16 + q] = f[q];
    double ref[3];
    cone_reference(ad, wd, tri, nq, ref);
    // |T| from the relative positions
    double e[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) e[j][c] = ad[j + 1][c] - ad[0][c];
    const double vol = fabs(e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                            e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                            e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0])) / 6.0;
    const double rn = sqrt(ref[0] * ref[0] + ref[1] * ref[1] + ref[2] * ref[2]);
    // rule table: barycentric points of the 1-, 4- and 11-point rules (16 x 4),
    // then their 16 weights
    const int npts[3] = {1, 4, 11};
    const int off[3] = {0, 1, 5};
    int label = 3; // ray tracing unless a Gauss rule meets the budget
    for (int r = 2; r >= 0; --r) {
        double g[3];
        gauss_value(ad, wd, rules + 4 * off[r], rules + 64 + off[r], npts[r], vol, g);
        const double dx = g[0] - ref[0], dy = g[1] - ref[1], dz = g[2] - ref[2];
        const double er = sqrt(dx * dx + dy * dy + dz * dz) / fmax(rn, 1e-300);
        errs[(size_t)k * 3 + r] = (float)er;
        if (er <= tau) label = r; // scanning down: the cheapest qualifying rule wins
    }
    labels[k] = (int8_t)label;
}

hipError_t launch_label(const DevMesh &m, const int2 *pairs, int n, float hbar, const double *tri, int nq,
                        const float *rules, double tau, float *feats, int8_t *labels, float *errs, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_label, dim3((n + 63) / 64), dim3(64), 0, s, m, pairs, n, hbar, tri, nq, rules, tau, feats,
                       labels, errs);
    return hipGetLastError();
}

// --------------------------------------------------------------- training
//
// One block = one wave = 64 rows of the mini-batch.  Parameters are read as
// BF16 (the forward copy); gradients accumulate in FP32 and are written per
// block (unnormalised: sum of c_y dCE/dtheta), with the block's weight sum.

// Gradient of one 64-row tile.  rows >= nvalid are ignored (zero weight).
// grads: [5508] FP32 block partial in blob order without mu / inv_sigma
// (W1, b1, W2, b2, W3, b3); wsum: block weight sum.
__global__ void __launch_bounds__(64) k_mlp_grad(const float *__restrict__ feats, const int8_t *__restrict__ labels,
                                                 const int *__restrict__ index, int n, const __bf16 *__restrict__ wb,
                                                 const float *__restrict__ class_w, float *__restrict__ gpart,
                                                 float *__restrict__ wpart, float *__restrict__ lpart)
{
    __shared__ MlpLds L;
    const int lane = threadIdx.x;
    const int row0 = blockIdx.x * 64;
    const __bf16 *mu = wb, *isg = wb + 16, *W1 = wb + 32, *b1 = W1 + 1024, *W2 = b1 + 64, *b2 = W2 + 4096,
                 *W3 = b2 + 64, *b3 = W3 + 256;
    const int rowi = row0 + lane;
    const bool valid = rowi < n;
    const int src = valid ? (index ? index[rowi] : rowi) : 0;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const float v = valid ? feats[(size_t)src * 16 + q] : 0.f;
        L.x[lane][q] = to_bf16((v - (float)mu[q]) * (float)isg[q]);
    }
    __syncthreads();
    mlp_forward_tile(L, W1, b1, W2, b2, W3, b3, lane);
    // softmax cross-entropy, weighted; d3 = c_y (p - onehot)
    const int y = valid ? labels[src] : 0;
    const float cy = valid ? class_w[y] : 0.f;
    float z[4], zm = -3e38f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        z[c] = L.z3[lane][c];
        zm = fmaxf(zm, z[c]);
    }
    float e[4], se = 0.f;
#pragma unroll
    for (int c = 0; c < 4; ++c) {
        e[c] = __expf(z[c] - zm);
        se += e[c];
    }
    const float lse = zm + __logf(se);
#pragma unroll
    for (int c = 0; c < 32; ++c) {
        const float p = c < 4 ? e[c] / se : 0.f;
        const float d = c < 4 ? cy * (p - (c == y ? 1.f : 0.f)) : 0.f;
        L.d3[lane][c] = to_bf16(d);
    }
    const float lossw = cy * (lse - z[y]);
    // masks of z1 > 0, z2 > 0 from the stored activations (relu output > 0)
    unsigned long long mk1 = 0, mk2 = 0;
    for (int j = 0; j < 64; ++j) {
        mk1 |= (unsigned long long)((float)L.a1[lane][j] > 0.f) << j;
        mk2 |= (unsigned long long)((float)L.a2[lane][j] > 0.f) << j;
    }
    L.m1[lane] = mk1;
    L.m2[lane] = mk2;
    __syncthreads();
    float *G = gpart + (size_t)blockIdx.x * kMlpGradLen;
    float *gW1 = G, *gb1 = G + 1024, *gW2 = gb1 + 64, *gb2 = gW2 + 4096, *gW3 = gb2 + 64, *gb3 = gW3 + 256;
    // dW3 = a2^T d3: [64 hidden x 64 rows] x [64 rows x 4]
    for (int rt = 0; rt < 2; ++rt) {
        f32x16 acc = {};
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) mfma_tile(acc, &L.a2[16 * kt][32 * rt], 1, 64, &L.d3[16 * kt][0], 32, 1, lane);
        const int col = lane & 31;
        if (col < 4) {
#pragma unroll
            for (int r = 0; r < 16; ++r) gW3[(32 * rt + tile_row(lane, r)) * 4 + col] = acc[r];
        }
    }
    // db3
    for (int c = 0; c < 4; ++c) {
        const float v = wave_sum_f((float)L.d3[lane][c]);
        if (lane == 0) gb3[c] = v;
    }
    // dz2 = (d3 W3^T) * [z2 > 0]: [64 x 16(4 used)] x [16 x 64]
    for (int rt = 0; rt < 2; ++rt)
        for (int ct = 0; ct < 2; ++ct) {
            f32x16 acc = {};
            {
                bf16x8 av, bv;
                const int r = lane & 31, kb = 8 * (lane >> 5);
#pragma unroll
                for (int s = 0; s < 8; ++s) {
                    const int k = kb + s;
                    av[s] = L.d3[32 * rt + r][k];
                    bv[s] = k < 4 ? W3[(32 * ct + r) * 4 + k] : (__bf16)0.f;
                }
                acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 32 * rt + tile_row(lane, r), col = 32 * ct + (lane & 31);
                const bool on = (L.m2[row] >> col) & 1ull;
                L.g[row][col] = to_bf16(on ? acc[r] : 0.f);
            }
        }
    __syncthreads();
    // dW2 = a1^T dz2, db2
    for (int rt = 0; rt < 2; ++rt)
        for (int ct = 0; ct < 2; ++ct) {
            f32x16 acc = {};
#pragma unroll
            for (int kt = 0; kt < 4; ++kt)
                mfma_tile(acc, &L.a1[16 * kt][32 * rt], 1, 64, &L.g[16 * kt][32 * ct], 64, 1, lane);
#pragma unroll
            for (int r = 0; r < 16; ++r) gW2[(32 * rt + tile_row(lane, r)) * 64 + 32 * ct + (lane & 31)] = acc[r];
        }
    {
        float v = 0.f;
        for (int r = 0; r < 64; ++r) v += (float)L.g[r][lane];
        gb2[lane] = v;
    }
    // dz1 = (dz2 W2^T) * [z1 > 0]: computed into registers, then stored over g
    f32x16 t1[2][2];
    for (int rt = 0; rt < 2; ++rt)
        for (int ct = 0; ct < 2; ++ct) {
            f32x16 acc = {};
#pragma unroll
            for (int kt = 0; kt < 4; ++kt)
                mfma_tile(acc, &L.g[32 * rt][16 * kt], 64, 1, W2 + (32 * ct) * 64 + 16 * kt, 1, 64, lane);
            t1[rt][ct] = acc;
        }
    __syncthreads();
    for (int rt = 0; rt < 2; ++rt)
        for (int ct = 0; ct < 2; ++ct)
#pragma unroll
            for (int r = 0; r < 16; ++r) {
                const int row = 32 * rt + tile_row(lane, r), col = 32 * ct + (lane & 31);
                const bool on = (L.m1[row] >> col) & 1ull;
                L.g[row][col] = to_bf16(on ? t1[rt][ct][r] : 0.f);
            }
    __syncthreads();
    // dW1 = xs^T dz1: [16 x 64 rows] x [64 rows x 64]; the tile has 32 rows, 16 used
    for (int ct = 0; ct < 2; ++ct) {
        f32x16 acc = {};
#pragma unroll
        for (int kt = 0; kt < 4; ++kt) {
            bf16x8 av, bv;
            const int r = lane & 31, kb = 8 * (lane >> 5);
#pragma unroll
            for (int s = 0; s < 8; ++s) {
                av[s] = r < 16 ? L.x[16 * kt + kb + s][r] : (__bf16)0.f;
                bv[s] = L.g[16 * kt + kb + s][32 * ct + r];
            }
            acc = __builtin_amdgcn_mfma_f32_32x32x16_bf16(av, bv, acc, 0, 0, 0);
        }
#pragma unroll
        for (int r = 0; r < 16; ++r) {
            const int row = tile_row(lane, r);
            if (row < 16) gW1[row * 64 + 32 * ct + (lane & 31)] = acc[r];
        }
    }
    {
        float v = 0.f;
        for (int r = 0; r < 64; ++r) v += (float)L.g[r][lane];
        gb1[lane] = v;
    }
    const float ws = wave_sum_f(cy), ls = wave_sum_f(lossw);
    if (lane == 0) {
        wpart[blockIdx.x] = ws;
        lpart[blockIdx.x] = ls;
    }
}

// Deterministic reduction of the block partials and one Adam step.
// master: FP32 weights in blob order without mu / inv_sigma; m, v: moments;
// wb: BF16 forward copy (full blob, mu / inv_sigma untouched).
__global__ void __launch_bounds__(256) k_mlp_adam(const float *__restrict__ gpart, const float *__restrict__ wpart,
                                                  int nblocks, float *__restrict__ master, float *__restrict__ mom1,
                                                  float *__restrict__ mom2, __bf16 *__restrict__ wb, float lr,
                                                  float beta1, float beta2, float eps, float bc1, float bc2,
                                                  float *__restrict__ grad_out)
{
    const int j = blockIdx.x * 256 + threadIdx.x;
    if (j >= kMlpGradLen) return;
    double W = 0.0, g = 0.0;
    for (int b = 0; b < nblocks; ++b) {
        W += (double)wpart[b];
        g += (double)gpart[(size_t)b * kMlpGradLen + j];
    }
    const float gr = W > 0.0 ? (float)(g / W) : 0.f;
    if (grad_out) grad_out[j] = gr;
    if (lr == 0.f) return; // gradient only
    const float m1 = beta1 * mom1[j] + (1.f - beta1) * gr;
    const float m2 = beta2 * mom2[j] + (1.f - beta2) * gr * gr;
    mom1[j] = m1;
    mom2[j] = m2;
    const float w = master[j] - lr * (m1 / bc1) / (sqrtf(m2 / bc2) + eps);
    master[j] = w;
    wb[32 + j] = (__bf16)w;
}

__global__ void k_sum_f(const float *__restrict__ a, int n, double *__restrict__ out)
{
    if (threadIdx.x == 0 && blockIdx.x == 0) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += a[i];
        out[0] = s;
    }
}

hipError_t launch_mlp_grad_step(const float *feats, const int8_t *labels, const int *index, int n, __bf16 *wb,
                                const float *class_w, float *gpart, float *wpart, float *lpart, float *master,
                                float *mom1, float *mom2, float lr, float beta1, float beta2, float eps, int step,
                                float *grad_out, hipStream_t s)
{
    const int nb = (n + 63) / 64;
    hipLaunchKernelGGL(k_mlp_grad, dim3(nb), dim3(64), 0, s, feats, labels, index, n, wb, class_w, gpart, wpart,
                       lpart);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const float bc1 = 1.f - powf(beta1, (float)step), bc2 = 1.f - powf(beta2, (float)step);
    hipLaunchKernelGGL(k_mlp_adam, dim3((kMlpGradLen + 255) / 256), dim3(256), 0, s, gpart, wpart, nb, master, mom1,
                       mom2, wb, lr, beta1, beta2, eps, bc1 > 0.f ? bc1 : 1.f, bc2 > 0.f ? bc2 : 1.f, grad_out);
    return hipGetLastError();
}

hipError_t launch_sum_f(const float *a, int n, double *out, hipStream_t s)
{
    hipLaunchKernelGGL(k_sum_f, dim3(1), dim3(64), 0, s, a, n, out);
    return hipGetLastError();
}

// Logits of n rows (inference check): one wave per 64 rows.
__global__ void __launch_bounds__(64) k_mlp_logits(const float *__restrict__ feats, int n,
                                                   const __bf16 *__restrict__ wb, float *__restrict__ logits)
{
    __shared__ MlpLds L;
    const int lane = threadIdx.x;
    const int rowi = blockIdx.x * 64 + lane;
    const bool valid = rowi < n;
    const __bf16 *mu = wb, *isg = wb + 16, *W1 = wb + 32, *b1 = W1 + 1024, *W2 = b1 + 64, *b2 = W2 + 4096,
                 *W3 = b2 + 64, *b3 = W3 + 256;
#pragma unroll
    for (int q = 0; q < 16; ++q) {
        const float v = valid ? feats[(size_t)rowi * 16 + q] : 0.f;
        L.x[lane][q] = to_bf16((v - (float)mu[q]) * (float)isg[q]);
    }
    __syncthreads();
    mlp_forward_tile(L, W1, b1, W2, b2, W3, b3, lane);
    if (valid)
#pragma unroll
        for (int c = 0; c < 4; ++c) logits[(size_t)rowi * 4 + c] = L.z3[lane][c];
}

hipError_t launch_mlp_logits(const float *feats, int n, const __bf16 *wb, float *logits, hipStream_t s)
{
    if (n <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_mlp_logits, dim3((n + 63) / 64), dim3(64), 0, s, feats, n, wb, logits);
    return hipGetLastError();
}

} // namespace bsk
