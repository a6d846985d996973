// bs_kernels.hip -- gfx950 kernels of the Biot-Savart node-velocity library.
//
// Velocity at node x from tetrahedron T (eq. 1 of Carley, "Evaluation of
// Biot-Savart integrals on tetrahedral meshes"):
//   v(x) = -(1/4pi) int_T (x - y) x omega(y) / |x - y|^3 dV
// Far pairs: a symmetric Gauss rule, v += sum_q (W_q x r_q) / |r_q|^3 with
// r_q = x - p_q and W_q = w_q |T| omega(p_q) / 4pi (the standard approach the
// Introduction names for distant elements).
// Near pairs: ray tracing (Section 2.1).  Every line of the N x M angular
// rule is split at x into two rays d = +-s; a ray that crosses T between
// distances rho_near < rho_far contributes
//   kappa * (rho_far - rho_near)/2 * d x (omega_near + omega_far),
// which is eq. 5 with the sign of R restored (the integrand of eq. 2 on the
// full line is sgn(R) s x omega).  The face crossings are the
// Moller-Trumbore intersections; they are computed from signed volumes of
// the ray with the tet edges, one value per edge shared by the two faces
// (and the neighbouring tets) that contain the edge, so a ray is never
// counted as entering without leaving.
//
// Fixed rule per pair, decided in binary32 exactly as the CPU reference
// decides it: d^2 = ((dx*dx + dy*dy) + dz*dz) from the binary32 node and
// centroid coordinates against the squared cut distances; a tetrahedron
// having the node as a vertex is always ray traced.
//
// Kernels:
//   k_gauss_all  every pair by one Gauss rule (G1 for the fixed policy:
//                the far field of all pairs), tet records wave-uniform;
//   k_far_mfma   the G1 pairs of the fixed rule on the matrix cores (FP32
//                MFMA; pairs with another rule masked out);
//   k_band_piece per 64-node block: pairs whose fixed rule is G4 / G11,
//                after k_far_mfma (row pieces staged in LDS);
//   k_band       the same after k_gauss_all, also removing their G1 term;
//   k_rt         one wave per node: ray tracing of its near tetrahedra;
//   k_combine    FP64 sum of the partials, back to input node order.
#include "bs_internal.h"
#include "bs_mlp_dev.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

namespace bsk {

static_assert(sizeof(PackedNet) == kPackedNetBytes, "packed network layout");

#define RULE_G1 0
#define RULE_G4 1
#define RULE_G11 2
#define RULE_RT 3

// Fold a into the compensated pair (s, c) (Knuth's TwoSum).
__device__ __forceinline__ void two_sum(float &s, float &c, float a)
{
    const float t = s + a;
    const float bp = t - s;
    const float err = (s - (t - bp)) + (a - bp);
    s = t;
    c += err;
}

// Rule of the pair (node `self` at (x, y, z), tetrahedron with centroid c
// and vertex ids id) under the fixed distance policy.  Every operation is
// rounded separately (the file is built without FP contraction).
// The copy of the counters a node or block adds to.
__device__ __forceinline__ unsigned long long *cnt_copy(unsigned long long *cnt, int key)
{
    return cnt + kCntStride * (key & (kCntStripes - 1));
}

__device__ __forceinline__ int fixed_rule(float x, float y, float z, float cx, float cy, float cz, int4 id,
                                          int self, const Thresholds &th)
{
    const bool inc = (id.x == self) | (id.y == self) | (id.z == self) | (id.w == self);
    const float dx = x - cx, dy = y - cy, dz = z - cz;
    const float sx = dx * dx, sy = dy * dy, sz = dz * dz;
    const float d2 = (sx + sy) + sz;
    int rule = d2 < th.g4_2 ? RULE_G4 : RULE_G1;
    rule = d2 < th.g11_2 ? RULE_G11 : rule;
    return (inc || d2 < th.rt2) ? RULE_RT : rule;
}

// One Gauss point: acc += (W x r) / |r|^3, r = x - p.
__device__ __forceinline__ void gauss_point(float x, float y, float z, const float *g, float &ax, float &ay,
                                            float &az)
{
    const float rx = x - g[0], ry = y - g[1], rz = z - g[2];
    const float r2 = fmaf(rx, rx, fmaf(ry, ry, rz * rz));
    const float inv = __builtin_amdgcn_rsqf(r2);
    const float inv3 = inv * inv * inv;
    const float ux = rx * inv3, uy = ry * inv3, uz = rz * inv3;
    ax = fmaf(g[4], uz, fmaf(-g[5], uy, ax));
    ay = fmaf(g[5], ux, fmaf(-g[3], uz, ay));
    az = fmaf(g[3], uy, fmaf(-g[4], ux, az));
}

// NPL nodes against one Gauss point, written in phases (differences, squared
// distances, reciprocal square roots, then the products) so that the NPL
// independent chains interleave.
template <int NPL>
__device__ __forceinline__ void gauss_point_n(const float *x, const float *y, const float *z, const float *g,
                                              float *ax, float *ay, float *az)
{
    const float px = g[0], py = g[1], pz = g[2], wx = g[3], wy = g[4], wz = g[5];
    float rx[NPL], ry[NPL], rz[NPL], iv[NPL];
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
        rx[k] = x[k] - px;
        ry[k] = y[k] - py;
        rz[k] = z[k] - pz;
        iv[k] = fmaf(rx[k], rx[k], fmaf(ry[k], ry[k], rz[k] * rz[k]));
    }
#pragma unroll
    for (int k = 0; k < NPL; ++k) iv[k] = __builtin_amdgcn_rsqf(iv[k]);
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
        const float inv3 = iv[k] * iv[k] * iv[k];
        const float ux = rx[k] * inv3, uy = ry[k] * inv3, uz = rz[k] * inv3;
        ax[k] = fmaf(wy, uz, fmaf(-wz, uy, ax[k]));
        ay[k] = fmaf(wz, ux, fmaf(-wx, uz, ay[k]));
        az[k] = fmaf(wx, uy, fmaf(-wy, ux, az[k]));
    }
}

// ---------------------------------------------------------------------------
// Every pair by the NPTS-point rule.  Block = 256 lanes x NPL nodes;
// blockIdx.y = split of the tet range.  The tet loop index is uniform across
// the wave, so the point records are fetched by scalar loads and used as
// scalar operands.  PREC: 0 naive FP32, 1 TwoSum-compensated FP32 tiles,
// 2 FP64 accumulation.
template <int NPTS, int NPL, int PREC>
__global__ void __launch_bounds__(256) k_gauss_all(const float *__restrict__ xh, int npad, int node0,
                                                   const float *__restrict__ rec, int T, int per_split,
                                                   double *__restrict__ part)
{
    constexpr int kTile = 32;
    const int t0 = blockIdx.y * per_split;
    const int t1 = min(T, t0 + per_split);
    const int base = node0 + blockIdx.x * (256 * NPL) + threadIdx.x;
    float x[NPL], y[NPL], z[NPL];
    float ax[NPL], ay[NPL], az[NPL];
    float sx[NPL], sy[NPL], sz[NPL], cx[NPL], cy[NPL], cz[NPL];
    double dx[NPL], dy[NPL], dz[NPL];
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
        const int i = base + 256 * k;
        x[k] = xh[i];
        y[k] = xh[npad + i];
        z[k] = xh[2 * npad + i];
        ax[k] = ay[k] = az[k] = 0.f;
        sx[k] = sy[k] = sz[k] = cx[k] = cy[k] = cz[k] = 0.f;
        dx[k] = dy[k] = dz[k] = 0.0;
    }
    if (PREC == 0) {
#pragma unroll 2
        for (int t = t0; t < t1; ++t) {
            const float *g = rec + (size_t)t * (NPTS * kRecG);
#pragma unroll
            for (int q = 0; q < NPTS; ++q) gauss_point_n<NPL>(x, y, z, g + q * kRecG, ax, ay, az);
        }
#pragma unroll
        for (int k = 0; k < NPL; ++k) {
            sx[k] = ax[k];
            sy[k] = ay[k];
            sz[k] = az[k];
        }
    } else {
        for (int tb = t0; tb < t1; tb += kTile) {
            const int te = min(tb + kTile, t1);
#pragma unroll
            for (int k = 0; k < NPL; ++k) ax[k] = ay[k] = az[k] = 0.f;
#pragma unroll 2
            for (int t = tb; t < te; ++t) {
                const float *g = rec + (size_t)t * (NPTS * kRecG);
#pragma unroll
                for (int q = 0; q < NPTS; ++q) gauss_point_n<NPL>(x, y, z, g + q * kRecG, ax, ay, az);
            }
#pragma unroll
            for (int k = 0; k < NPL; ++k) {
                if (PREC == 1) {
                    two_sum(sx[k], cx[k], ax[k]);
                    two_sum(sy[k], cy[k], ay[k]);
                    two_sum(sz[k], cz[k], az[k]);
                } else {
                    dx[k] += (double)ax[k];
                    dy[k] += (double)ay[k];
                    dz[k] += (double)az[k];
                }
            }
        }
    }
    double *o = part + (size_t)blockIdx.y * 3 * npad;
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
        const int i = base + 256 * k;
        if (PREC == 2) {
            o[i] = dx[k];
            o[npad + i] = dy[k];
            o[2 * npad + i] = dz[k];
        } else {
            o[i] = (double)sx[k] + (double)cx[k];
            o[npad + i] = (double)sy[k] + (double)cy[k];
            o[2 * npad + i] = (double)sz[k] + (double)cz[k];
        }
    }
}

// The PREC == 2 variant above accumulates FP32 tile sums in FP64; the
// per-term FP64 variant (every pair term converted and added in FP64) is
// this one, used for BS_PREC_FP64.
template <int NPTS, int NPL>
__global__ void __launch_bounds__(256) k_gauss_all_f64(const float *__restrict__ xh, int npad, int node0,
                                                       const float *__restrict__ rec, int T, int per_split,
                                                       double *__restrict__ part)
{
    const int t0 = blockIdx.y * per_split;
    const int t1 = min(T, t0 + per_split);
    const int base = node0 + blockIdx.x * (256 * NPL) + threadIdx.x;
    float x[NPL], y[NPL], z[NPL];
    double dx[NPL], dy[NPL], dz[NPL];
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
        const int i = base + 256 * k;
        x[k] = xh[i];
        y[k] = xh[npad + i];
        z[k] = xh[2 * npad + i];
        dx[k] = dy[k] = dz[k] = 0.0;
    }
    for (int t = t0; t < t1; ++t) {
        const float *g = rec + (size_t)t * (NPTS * kRecG);
#pragma unroll
        for (int q = 0; q < NPTS; ++q)
#pragma unroll
            for (int k = 0; k < NPL; ++k) {
                float a = 0.f, b = 0.f, c = 0.f;
                gauss_point(x[k], y[k], z[k], g + q * kRecG, a, b, c);
                dx[k] += (double)a;
                dy[k] += (double)b;
                dz[k] += (double)c;
            }
    }
    double *o = part + (size_t)blockIdx.y * 3 * npad;
#pragma unroll
    for (int k = 0; k < NPL; ++k) {
        const int i = base + 256 * k;
        o[i] = dx[k];
        o[npad + i] = dy[k];
        o[2 * npad + i] = dz[k];
    }
}

constexpr int kNpl = 4;

template <int NPTS>
static hipError_t launch_gauss_pts(const DevMesh &m, int precision, int splits, double *part, hipStream_t s)
{
    const int per = (m.T + splits - 1) / splits;
    const int node0 = m.blk0 * kBlockNodes; // a multiple of 1024 (see build_device_mesh)
    dim3 grid((m.nv - node0 + 256 * kNpl - 1) / (256 * kNpl), splits);
    if (precision == 0)
        hipLaunchKernelGGL((k_gauss_all<NPTS, kNpl, 0>), grid, dim3(256), 0, s, m.xh, m.npad, node0, NPTS == 1 ? m.g1
                           : NPTS == 4 ? m.g4 : m.g11, m.T, per, part);
    else if (precision == 1)
        hipLaunchKernelGGL((k_gauss_all<NPTS, kNpl, 1>), grid, dim3(256), 0, s, m.xh, m.npad, node0, NPTS == 1 ? m.g1
                           : NPTS == 4 ? m.g4 : m.g11, m.T, per, part);
    else
        hipLaunchKernelGGL((k_gauss_all_f64<NPTS, kNpl>), grid, dim3(256), 0, s, m.xh, m.npad, node0, NPTS == 1 ? m.g1
                           : NPTS == 4 ? m.g4 : m.g11, m.T, per, part);
    return hipGetLastError();
}

hipError_t launch_gauss_all(const DevMesh &m, int rule_pts, int precision, int splits, double *part,
                            hipStream_t s)
{
    if (m.npad % (256 * kNpl)) return hipErrorInvalidValue;
    if (rule_pts == 1) return launch_gauss_pts<1>(m, precision, splits, part, s);
    if (rule_pts == 4) return launch_gauss_pts<4>(m, precision, splits, part, s);
    if (rule_pts == 11) return launch_gauss_pts<11>(m, precision, splits, part, s);
    return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// Far field of the fixed-rule policies on the matrix cores.
//
// With positions relative to the centre c of a 64-node block (x' = x - c,
// p' = p - c) the 1-point term of a pair is s W x (x' - p') with
// s = |x' - p'|^-3, so the block's far field is
//   v(x) = (sum_t s W_t) x x' - sum_t s (W_t x p'_t).
// Both sums over the tets are contractions:
//   |x' - p'|^2 = |x'|^2 + [x', 1] . [-2 p', |p'|^2]        (K = 4)
// on v_mfma_f32_16x16x4f32 (rows = 16 tets, columns = 16 nodes), then
//   sum_t s [W, W x p']
// on the 16 independent 4x4 blocks of v_mfma_f32_4x4x1f32.  The operand
// lanes of the second line up with the output lanes of the first (block b =
// lanes 4b..4b+3 = one tet and four nodes), so the reciprocal cubes pass from
// one to the other in registers.
// Pairs whose rule is not G1 are masked out: for a tile of 16 tets whose
// centroids' bounding sphere (precomputed per tile) comes within r_band of
// a node tile's bounding sphere, every pair of that node tile is classified
// with the comparisons of fixed_rule
// (the band and ray-tracing kernels take the others); outside the band
// every pair is G1.  The cut distances are ordered (checked on the host),
// so a pair is G1 exactly when it is not incident and !(d^2 < g4^2); the
// incidence test is needed only when a tet's vertex can lie beyond the G4
// cut from its centroid.
//
// Workgroup = 4 waves = one block of 64 nodes (4 node tiles of 16) and one
// split of the tet range.  Every chunk of 256 tets is prepared once into LDS
// (double buffered); wave w takes tet tiles w, w+4, w+8, w+12 of the chunk
// against all four node tiles.  Lane l: node l%16 of a node tile, tets
// 4(l/16)+j, j < 4, of a tet tile.
// The records of chunk k+2 are loaded into registers while chunk k is
// computed and stored to LDS in the next step, so the loads' latency hides
// behind a whole chunk of work.
// PREC 0: FP32 accumulation throughout; PREC 1: the FP32 sums of every two
// chunks are folded into a compensated FP32 pair (value, error) by TwoSum.
// FP64 only assembles each node's result at the end: the four waves' pairs,
// the cross product with the node's offset from the block centre.
constexpr int kFarChunk = 256;

constexpr int kA1Stride = 80; // floats per tile in a1 (64 used; the pad spreads the banks of the stores)

struct FarLds {
    union {
        struct {
            float a1[2][16][kA1Stride];       // [buf][tile][k*16 + i]: -2p'_k (k < 3), |p'|^2 (k = 3) of tet i
            float a2[2][16][4][4][8];         // [buf][tile][c][q][2j + h]: component 4h + c of [W, W x p'] of tet 4q + j
            unsigned long long band[2][16];   // [buf][tile]: bit 16 nt + i = centroid of tet i within the band of node tile nt
        } c;
    };
    float accs[4][6][64];                     // [wave][component][lane]: compensated FP32 sums (value, error) of
    float accc[4][6][64];                     //   node 16 (lane / 16) + lane % 16
    float4 xn[64];                            // binary32 node coordinates (the rule's), by node of the block
    float4 nts[4];                            // bounding sphere of each node tile (radius < 0: no node)
};

typedef float f32x4 __attribute__((ext_vector_type(4)));

template <int PREC>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(4))) k_far_mfma(DevMesh m, Thresholds th, int splits,
                                                  int per_split, double *__restrict__ part)
{
    __shared__ FarLds S;
    const int tid = threadIdx.x;
    const int lane = tid & 63;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int q = lane >> 4, i16 = lane & 15, c4 = lane & 3;
    // Consecutive workgroup ids go to the eight XCDs in turn.  With fewer
    // than eight splits: id = block * splits + split.  With 8 S splits: XCD
    // x = id % 8 owns the splits x S .. x S + S - 1 (one eighth of the tets)
    // and takes them one after the other, every block on a split before the
    // next (id / 8 = sub * nblk + block), so the split's records (sized to
    // fit the XCD's L2 by the host) are read by all blocks while resident.
    int bl, split;
    if (splits >= 8) {
        const int per_xcd = splits >> 3;
        const int rest = (int)(blockIdx.x >> 3);
        const int sub = rest / m.nblk;
        bl = rest - sub * m.nblk;
        split = (int)(blockIdx.x & 7) * per_xcd + sub;
    } else {
        bl = blockIdx.x / splits;
        split = blockIdx.x - bl * splits;
    }
    const int b = m.blk0 + bl;
    const int t0 = split * per_split;
    const int t1 = min(m.T, t0 + per_split);
    const float4 bc = m.blk[b];

    // node operands: B = [x', 1] (component q of the lane), C = |x'|^2
    float B1[4], Cin[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) {
        const int i = b * kBlockNodes + 16 * nt + i16;
        float xp[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float cc = c == 0 ? bc.x : c == 1 ? bc.y : bc.z;
            xp[c] = i < m.nv ? (m.xh[c * m.npad + i] - cc) + m.xl[c * m.npad + i] : 0.f;
        }
        B1[nt] = q == 0 ? xp[0] : q == 1 ? xp[1] : q == 2 ? xp[2] : 1.f;
        Cin[nt] = i < m.nv ? (xp[0] * xp[0] + xp[1] * xp[1]) + xp[2] * xp[2] : 1e30f;
    }
    if (tid < 64) {
        const int i = b * kBlockNodes + tid;
        S.xn[tid] = make_float4(m.xh[i], m.xh[m.npad + i], m.xh[2 * m.npad + i], 0.f);
    }
    __syncthreads();
    if (tid < 4) {
        float lo[3] = {3e38f, 3e38f, 3e38f}, hi[3] = {-3e38f, -3e38f, -3e38f};
        const int nv = min(16, m.nv - (b * kBlockNodes + 16 * tid));
        for (int k = 0; k < nv; ++k) {
            const float4 x = S.xn[16 * tid + k];
            lo[0] = fminf(lo[0], x.x), hi[0] = fmaxf(hi[0], x.x);
            lo[1] = fminf(lo[1], x.y), hi[1] = fmaxf(hi[1], x.y);
            lo[2] = fminf(lo[2], x.z), hi[2] = fmaxf(hi[2], x.z);
        }
        const float cx = 0.5f * (lo[0] + hi[0]), cy = 0.5f * (lo[1] + hi[1]), cz = 0.5f * (lo[2] + hi[2]);
        float r2 = 0.f;
        for (int k = 0; k < nv; ++k) {
            const float4 x = S.xn[16 * tid + k];
            const float dx = x.x - cx, dy = x.y - cy, dz = x.z - cz;
            r2 = fmaxf(r2, (dx * dx + dy * dy) + dz * dz);
        }
        S.nts[tid] = nv > 0 ? make_float4(cx, cy, cz, sqrtf(r2) * (1.f + 1e-5f) + 1e-6f) : make_float4(0.f, 0.f, 0.f, -1.f);
    }
    __syncthreads();
    float4 nts[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) nts[nt] = S.nts[nt];

    f32x4 D0[4], D1[4];
#pragma unroll
    for (int nt = 0; nt < 4; ++nt) D0[nt] = D1[nt] = (f32x4){0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int r = 0; r < 6; ++r) S.accs[wave][r][lane] = S.accc[wave][r][lane] = 0.f; // node 16q + i16 after each fold

    // the record of tet c0 + tid, in flight in registers until stored (the
    // index is clamped so that the loads need no branch; tets past the end
    // of the split are replaced at the store)
    float4 pg;
    float2 pw;
    int pt;
    auto load = [&](int c0) {
        pt = c0 + tid;
        const int t = min(pt, t1 - 1);
        const float *g = m.g1 + (size_t)t * kRecG;
        pg = *(const float4 *)g;
        pw = *(const float2 *)(g + 4);
    };
    auto store = [&](int buf) {
        const int tile = tid >> 4, i = tid & 15, qq = i >> 2, j = i & 3;
        // a slot past the split keeps the clamped tet's position (finite
        // operands) with zero strength and |p'|^2 = 1e30: its terms are 0
        const bool pok = pt < t1;
        const float pr[6] = {pg.x, pg.y, pg.z, pok ? pg.w : 0.f, pok ? pw.x : 0.f, pok ? pw.y : 0.f};
        const float px = pr[0] - bc.x, py = pr[1] - bc.y, pz = pr[2] - bc.z;
        const float n2 = (px * px + py * py) + pz * pz;
        S.c.a1[buf][tile][i] = -2.f * px;
        S.c.a1[buf][tile][16 + i] = -2.f * py;
        S.c.a1[buf][tile][32 + i] = -2.f * pz;
        S.c.a1[buf][tile][48 + i] = pok ? n2 : 1e30f;
        const float comp[8] = {pr[3], pr[4], pr[5], pr[4] * pz - pr[5] * py, pr[5] * px - pr[3] * pz,
                               pr[3] * py - pr[4] * px, 0.f, 0.f};
#pragma unroll
        for (int c = 0; c < 4; ++c)
#pragma unroll
            for (int h = 0; h < 2; ++h) S.c.a2[buf][tile][c][qq][2 * j + h] = comp[4 * h + c];
        // the wave's 64 tets are tiles 4 wave + tl of the chunk; lane 4 tl + nt
        // tests the bounding sphere of tile tl against node tile nt
        bool near = false;
        if (lane < 16) {
            const int g = ((pt - lane) >> 4) + (lane >> 2);
            const float4 ns = S.nts[lane & 3];
            if (16 * g < t1 && ns.w >= 0.f) {
                const float4 ts = m.tsph[g];
                const float dx = ts.x - ns.x, dy = ts.y - ns.y, dz = ts.z - ns.z;
                const float rr = (ts.w + ns.w + th.r_band) * (1.f + 1e-5f);
                near = (dx * dx + dy * dy) + dz * dz < rr * rr;
            }
        }
        const unsigned long long bal = __ballot(near);
#pragma unroll
        for (int tl = 0; tl < 4; ++tl) {
            unsigned long long pk = 0;
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) pk |= ((bal >> (4 * tl + nt)) & 1ull) ? 0xffffull << (16 * nt) : 0ull;
            if (lane == 0) S.c.band[buf][4 * wave + tl] = pk;
        }
    };
    // sum the four tet streams of every node (lanes l, l^16, l^32, l^48) in
    // FP32, leaving node tile q's six sums in lane group q (a reduce-scatter
    // by lane swaps: lanes 0-31 keep node tiles 0, 1 and lanes 32-63 tiles
    // 2, 3, then even and odd groups split those), and fold them into the
    // compensated pairs by TwoSum (Knuth: t = s + x, the rounding error of
    // the addition recovered exactly from t, s and x)
    auto fold = [&]() {
        float y[2][6];
#pragma unroll
        for (int h = 0; h < 2; ++h)
#pragma unroll
            for (int r = 0; r < 6; ++r) {
                const float lo = r < 4 ? D0[h][r] : D1[h][r - 4];
                const float hi = r < 4 ? D0[h + 2][r] : D1[h + 2][r - 4];
                const auto sw = __builtin_amdgcn_permlane32_swap(__float_as_uint(lo), __float_as_uint(hi), false, false);
                y[h][r] = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
            }
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            const auto sw =
                __builtin_amdgcn_permlane16_swap(__float_as_uint(y[0][r]), __float_as_uint(y[1][r]), false, false);
            const float x = __uint_as_float(sw[0]) + __uint_as_float(sw[1]);
            const float a = S.accs[wave][r][lane];
            const float t = a + x;
            const float bp = t - a;
            const float e = (a - (t - bp)) + (x - bp);
            S.accs[wave][r][lane] = t;
            S.accc[wave][r][lane] += e;
        }
#pragma unroll
        for (int nt = 0; nt < 4; ++nt) D0[nt] = D1[nt] = (f32x4){0.f, 0.f, 0.f, 0.f};
    };

    if (t0 < t1) {
        load(t0);
        store(0);
        if (t0 + kFarChunk < t1) load(t0 + kFarChunk);
    }
    __syncthreads();
    int k = 0;
    for (int c0 = t0; c0 < t1; c0 += kFarChunk, ++k) {
        const int buf = k & 1;
        if (c0 + kFarChunk < t1) {
            store(buf ^ 1);
            if (c0 + 2 * kFarChunk < t1) load(c0 + 2 * kFarChunk);
        }
#pragma unroll 1
        for (int u = 0; u < 4; ++u) {
            const int tile = wave + 4 * u;
            const unsigned long long bw = S.c.band[buf][tile];
            const unsigned blo = __builtin_amdgcn_readfirstlane((unsigned)bw);
            const unsigned bhi = __builtin_amdgcn_readfirstlane((unsigned)(bw >> 32));
            const unsigned bmask[4] = {blo & 0xffffu, blo >> 16, bhi & 0xffffu, bhi >> 16};
            const float A1 = S.c.a1[buf][tile][lane];
            const float4 v0 = *(const float4 *)&S.c.a2[buf][tile][c4][q][0];
            const float4 v1 = *(const float4 *)&S.c.a2[buf][tile][c4][q][4];
            const float A2[4][2] = {{v0.x, v0.y}, {v0.z, v0.w}, {v1.x, v1.y}, {v1.z, v1.w}};
            // the matrix core and the vector ALUs of a SIMD do not overlap
            // here (each MFMA group costs its full pipe time), so a wave at
            // its MFMAs is given issue priority over the waves at vector work
            // and the matrix pipe runs its groups back to back
            f32x4 r2[4];
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
                r2[nt] = __builtin_amdgcn_mfma_f32_16x16x4f32(A1, B1[nt], (f32x4){Cin[nt], Cin[nt], Cin[nt], Cin[nt]},
                                                             0, 0, 0);
            __builtin_amdgcn_s_setprio(0);
            float sv[4][4];
#pragma unroll
            for (int nt = 0; nt < 4; ++nt)
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    const float iv = __builtin_amdgcn_rsqf(r2[nt][j]);
                    sv[nt][j] = iv * iv * iv;
                }
            // (one branch skips the masks of a tet tile clear of every node tile's band)
            if (blo | bhi)
#pragma unroll
            for (int nt = 0; nt < 4; ++nt) {
                if (!bmask[nt]) continue;
                // the matrix-core distance decides the pairs clear of the G4
                // cut; a wave with a pair near it (or with incidence to test)
                // takes the rule's own test for all its pairs
                bool g1[4], amb = false;
#pragma unroll
                for (int j = 0; j < 4; ++j) {
                    g1[j] = sv[nt][j] < th.s_g1;
                    amb = amb || (!g1[j] && !(sv[nt][j] > th.s_amb));
                }
                if (th.inc_far || __ballot(amb)) {
                    const float4 xn = S.xn[16 * nt + i16];
                    const int self = b * kBlockNodes + 16 * nt + i16;
#pragma unroll
                    for (int j = 0; j < 4; ++j) {
                        // the rule's centroid and ids from the tet records (a
                        // padding slot past the split reads the last tet: its
                        // strength is zero in the operands, any decision holds)
                        const int tg = min(c0 + tile * 16 + 4 * q + j, t1 - 1);
                        const float4 pc = *reinterpret_cast<const float4 *>(m.g1 + (size_t)tg * kRecG);
                        const float dx = xn.x - pc.x, dy = xn.y - pc.y, dz = xn.z - pc.z;
                        const float sx = dx * dx, sy = dy * dy, sz = dz * dz;
                        g1[j] = !((sx + sy) + sz < th.g4_2);
                        if (th.inc_far) {
                            const int4 id = m.tid[tg];
                            g1[j] = g1[j] && !((id.x == self) | (id.y == self) | (id.z == self) | (id.w == self));
                        }
                    }
                }
#pragma unroll
                for (int j = 0; j < 4; ++j) sv[nt][j] = g1[j] ? sv[nt][j] : 0.f;
            }
            __builtin_amdgcn_s_setprio(1);
#pragma unroll
            for (int j = 0; j < 4; ++j)
#pragma unroll
                for (int nt = 0; nt < 4; ++nt) {
                    D0[nt] = __builtin_amdgcn_mfma_f32_4x4x1f32(A2[j][0], sv[nt][j], D0[nt], 0, 0, 0);
                    D1[nt] = __builtin_amdgcn_mfma_f32_4x4x1f32(A2[j][1], sv[nt][j], D1[nt], 0, 0, 0);
                }
            __builtin_amdgcn_s_setprio(0);
        }
        if (PREC == 1 && (k & 1)) fold();
        __syncthreads();
    }
    fold();
    // combine the waves (each took a quarter of every chunk)
    __syncthreads();
    if (tid < 64) {
        double sw[6];
#pragma unroll
        for (int r = 0; r < 6; ++r) {
            sw[r] = 0.0;
#pragma unroll
            for (int w = 0; w < 4; ++w) sw[r] += (double)S.accs[w][r][tid] + (double)S.accc[w][r][tid];
        }
        const int i = b * kBlockNodes + tid;
        double xp[3] = {0.0, 0.0, 0.0};
        if (i < m.nv) {
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                const float cc = c == 0 ? bc.x : c == 1 ? bc.y : bc.z;
                xp[c] = (double)((m.xh[c * m.npad + i] - cc) + m.xl[c * m.npad + i]);
            }
        }
        double *o = part + (size_t)split * 3 * m.npad;
        o[i] = (sw[1] * xp[2] - sw[2] * xp[1]) - sw[3];
        o[m.npad + i] = (sw[2] * xp[0] - sw[0] * xp[2]) - sw[4];
        o[2 * m.npad + i] = (sw[0] * xp[1] - sw[1] * xp[0]) - sw[5];
    }
}

hipError_t launch_far_mfma(const DevMesh &m, const Thresholds &th, int precision, int splits, double *part,
                           hipStream_t s)
{
    if (splits < 1 || (splits > 8 && splits % 8) || precision < 0 || precision > 1) return hipErrorInvalidValue;
    const int per = ((m.T + splits - 1) / splits + kFarChunk - 1) / kFarChunk * kFarChunk;
    const dim3 grid(m.nblk * splits);
    if (precision == 0)
        hipLaunchKernelGGL(k_far_mfma<0>, grid, dim3(256), 0, s, m, th, splits, per, part);
    else
        hipLaunchKernelGGL(k_far_mfma<1>, grid, dim3(256), 0, s, m, th, splits, per, part);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Rows of bins (fixed y, z; x range clipped to the ball) intersecting the
// ball (c, R); next() yields the contiguous tet range of each row in turn.
struct RowIter {
    const DevMesh &m;
    float cx, cy, cz, R, inv;
    int iy, iz, iy0, iy1, iz1;
    __device__ RowIter(const DevMesh &mm, float x, float y, float z, float r) : m(mm), cx(x), cy(y), cz(z), R(r)
    {
        inv = 1.0f / m.bins.cs;
        iy0 = max(0, (int)floorf((cy - R - m.bins.lo[1]) * inv));
        iy1 = min(m.bins.dim[1] - 1, (int)floorf((cy + R - m.bins.lo[1]) * inv));
        iz = max(0, (int)floorf((cz - R - m.bins.lo[2]) * inv));
        iz1 = min(m.bins.dim[2] - 1, (int)floorf((cz + R - m.bins.lo[2]) * inv));
        iy = iy0;
    }
    __device__ __forceinline__ bool next(int &t0, int &t1)
    {
        for (; iz <= iz1; ++iz, iy = iy0) {
            const float zl = m.bins.lo[2] + iz * m.bins.cs, zh = zl + m.bins.cs;
            const float dz = cz < zl ? zl - cz : (cz > zh ? cz - zh : 0.f);
            for (; iy <= iy1; ++iy) {
                const float yl = m.bins.lo[1] + iy * m.bins.cs, yh = yl + m.bins.cs;
                const float dy = cy < yl ? yl - cy : (cy > yh ? cy - yh : 0.f);
                const float rem = R * R - dy * dy - dz * dz;
                if (rem < 0.f) continue;
                const float hw = sqrtf(rem);
                const int ix0 = max(0, (int)floorf((cx - hw - m.bins.lo[0]) * inv));
                const int ix1 = min(m.bins.dim[0] - 1, (int)floorf((cx + hw - m.bins.lo[0]) * inv));
                if (ix0 > ix1) continue;
                const int row = (iz * m.bins.dim[1] + iy) * m.bins.dim[0];
                t0 = m.cell_start[row + ix0];
                t1 = m.cell_start[row + ix1 + 1];
                ++iy;
                if (t0 < t1) return true;
                --iy;
            }
        }
        return false;
    }
};

__device__ __forceinline__ unsigned long long wave_sum_u64(unsigned long long v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

// ---------------------------------------------------------------------------
// Band corrections after k_gauss_all (which took every pair by G1).  One
// workgroup of kBandWaves waves per 64 consecutive (k-d ordered) nodes; lane
// = node, the waves take the bin rows of the block's neighbourhood in turn.
// For every tet whose centroid lies within r_band of the block's bounding
// sphere, lanes whose pair rule is not G1 subtract that G1 term, then lanes
// with G4 / G11 add that rule (ray-traced pairs are added by the ray-tracing
// kernels).  The waves' partial sums are combined in FP64 through LDS.
// (After k_far_mfma, which leaves out every pair that is not G1, the band
// runs in k_band_piece.)
constexpr int kBandWaves = 4;

template <int PREC>
__global__ void __launch_bounds__(64 * kBandWaves) k_band(DevMesh m, Thresholds th, double *__restrict__ band,
                                                          unsigned long long *__restrict__ cnt)
{
    __shared__ double red[kBandWaves][3][64];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6); // uniform within the wave
    // consecutive workgroup ids go to the eight XCDs in turn: give each XCD a
    // contiguous range of (spatially ordered) blocks, whose neighbourhoods
    // overlap in its L2
    const int per_xcd = (m.nblk + 7) >> 3;
    const int lb = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (lb >= m.nblk) return;
    const int blk = m.blk0 + lb;
    const int i = blk * kBlockNodes + lane;
    const bool valid = i < m.nv;
    const float x = m.xh[i], y = m.xh[m.npad + i], z = m.xh[2 * m.npad + i];
    const float4 bc = m.blk[blk];
    float sx = 0.f, sy = 0.f, sz = 0.f, ccx = 0.f, ccy = 0.f, ccz = 0.f;
    double dx = 0.0, dy = 0.0, dz = 0.0;
    unsigned long long n4 = 0, n11 = 0;
    RowIter rows(m, bc.x, bc.y, bc.z, th.r_band + bc.w);
    int t0, t1, row = 0;
    while (rows.next(t0, t1)) {
        if ((row++ % kBandWaves) != wave) continue;
        float ax = 0.f, ay = 0.f, az = 0.f;
        for (int t = t0; t < t1; ++t) {
            const float *g = m.g1 + (size_t)t * kRecG;
            // fixed_rule's comparisons on its own binary32 d^2; the incidence
            // test only where an incident pair can lie beyond the ray-tracing cut
            const float ex = x - g[0], ey = y - g[1], ez = z - g[2];
            const float qx = ex * ex, qy = ey * ey, qz = ez * ez;
            const float d2 = (qx + qy) + qz;
            bool near = d2 < th.rt2;
            if (th.inc_band) {
                const int4 id = m.tid[t];
                near = near || (id.x == i) | (id.y == i) | (id.z == i) | (id.w == i);
            }
            const bool in11 = valid && !near && d2 < th.g11_2;
            const bool in4 = valid && !near && d2 < th.g4_2 && !(d2 < th.g11_2);
            if (valid && (near || d2 < th.g4_2)) {
                float a = 0.f, b = 0.f, c = 0.f;
                gauss_point(x, y, z, g, a, b, c);
                ax -= a;
                ay -= b;
                az -= c;
            }
            if (in4) {
                const float *g4 = m.g4 + (size_t)t * 4 * kRecG;
#pragma unroll
                for (int q = 0; q < 4; ++q) gauss_point(x, y, z, g4 + q * kRecG, ax, ay, az);
                ++n4;
            }
            if (in11) {
                const float *g11 = m.g11 + (size_t)t * 11 * kRecG;
#pragma unroll
                for (int q = 0; q < 11; ++q) gauss_point(x, y, z, g11 + q * kRecG, ax, ay, az);
                ++n11;
            }
            // FP64 mode: every pair's terms added in FP64; compensated mode:
            // the FP32 sum of every 32 tets folded by TwoSum
            if (PREC == 2) {
                dx += (double)ax;
                dy += (double)ay;
                dz += (double)az;
                ax = ay = az = 0.f;
            } else if (PREC == 1 && ((t - t0) & 31) == 31) {
                two_sum(sx, ccx, ax);
                two_sum(sy, ccy, ay);
                two_sum(sz, ccz, az);
                ax = ay = az = 0.f;
            }
        }
        if (PREC == 1) {
            two_sum(sx, ccx, ax);
            two_sum(sy, ccy, ay);
            two_sum(sz, ccz, az);
        } else if (PREC == 0) {
            sx += ax;
            sy += ay;
            sz += az;
        }
    }
    if (PREC != 2) {
        dx = (double)sx + (double)ccx;
        dy = (double)sy + (double)ccy;
        dz = (double)sz + (double)ccz;
    }
    red[wave][0][lane] = dx;
    red[wave][1][lane] = dy;
    red[wave][2][lane] = dz;
    n4 = wave_sum_u64(n4);
    n11 = wave_sum_u64(n11);
    if (lane == 0 && cnt) {
        unsigned long long *c = cnt_copy(cnt, blockIdx.x);
        atomicAdd(&c[0], n4);
        atomicAdd(&c[1], n11);
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double v = red[0][c][lane];
#pragma unroll
            for (int w = 1; w < kBandWaves; ++w) v += red[w][c][lane];
            band[(size_t)c * m.npad + i] = v;
        }
    }
}

// Band pairs after k_far_mfma (no G1 terms to remove): k_band's blocks,
// waves, rows and rule masks, but each wave streams its rows in pieces of 32
// tets staged in its own LDS.  The centroids and G4 points of the next piece
// are loaded into registers while the current piece is evaluated, so a tet
// costs LDS broadcast reads instead of dependent scalar loads from L2 (the
// G11 points, needed for few tets, stay scalar loads).  The FP32 sums of a
// piece are folded into the compensated sums.
constexpr int kBandPiece = 32;

struct BandPieceLds {
    float4 cen[kBandPiece];     // centroid (x, y, z, 0)
    float4 pa[kBandPiece][4];   // G4 point q: position, W.x
    float4 pb[kBandPiece][2];   // G4 points 2e, 2e + 1: W.y, W.z of each
};

// Seven waves per SIMD (72 registers, a few spilled outside the point
// loop): the kernel waits on its record loads and LDS reads as well as
// issuing; at six waves it took 74.5 ms on the two-ring mesh, at seven 72.0.
template <int PREC>
__global__ void __launch_bounds__(64 * kBandWaves) __attribute__((amdgpu_waves_per_eu(7))) k_band_piece(DevMesh m, Thresholds th, double *__restrict__ band,
                                                                unsigned long long *__restrict__ cnt)
{
    __shared__ double red[kBandWaves][3][64];
    __shared__ BandPieceLds P[kBandWaves];
    const int lane = threadIdx.x & 63;
    const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
    const int per_xcd = (m.nblk + 7) >> 3;
    const int lb = (blockIdx.x & 7) * per_xcd + (blockIdx.x >> 3);
    if (lb >= m.nblk) return;
    const int blk = m.blk0 + lb;
    const int i = blk * kBlockNodes + lane;
    const bool valid = i < m.nv;
    const float x = m.xh[i], y = m.xh[m.npad + i], z = m.xh[2 * m.npad + i];
    const float4 bc = m.blk[blk];
    float sx = 0.f, sy = 0.f, sz = 0.f, ccx = 0.f, ccy = 0.f, ccz = 0.f;
    double dx = 0.0, dy = 0.0, dz = 0.0;
    unsigned long long n4 = 0, n11 = 0;
    RowIter rows(m, bc.x, bc.y, bc.z, th.r_band + bc.w);
    int row = 0, c0 = 0, c1 = 0, t0, t1;
    // lane l: tet c0 + l % 32 (clamped to the piece), G4 points 2h, 2h + 1
    // with h = l / 32; lanes below 32 also the centroid
    const int k = lane & (kBandPiece - 1), h = lane >> 5;
    float4 rc, ra0, ra1;
    float2 rb0, rb1;
#define BAND_FETCH()                                                                                   \
    do {                                                                                               \
        const int t_ = min(c0 + k, c1 - 1);                                                            \
        rc = *reinterpret_cast<const float4 *>(m.g1 + (size_t)t_ * kRecG);                            \
        const float *g_ = m.g4 + (size_t)t_ * 4 * kRecG + 2 * h * kRecG;                               \
        ra0 = *reinterpret_cast<const float4 *>(g_);                                                   \
        rb0 = *reinterpret_cast<const float2 *>(g_ + 4);                                               \
        ra1 = *reinterpret_cast<const float4 *>(g_ + kRecG);                                           \
        rb1 = *reinterpret_cast<const float2 *>(g_ + kRecG + 4);                                       \
    } while (0)
    // the first piece of this wave's rows
    bool have = false;
    while (rows.next(t0, t1)) {
        if ((row++ % kBandWaves) != wave) continue;
        c0 = t0;
        c1 = t1;
        have = true;
        break;
    }
    if (have) BAND_FETCH();
    while (have) {
        const int p0 = c0, pn = min(kBandPiece, c1 - c0);
        // the piece's tets within the scan radius of the block sphere (the
        // bin rows overreach it by about a quarter): no node of the block can
        // take any other by G4 or G11
        unsigned live;
        {
            const float qx = rc.x - bc.x, qy = rc.y - bc.y, qz = rc.z - bc.z;
            const float rs = (th.r_band + bc.w) * (1.f + 1e-5f);
            live = (unsigned)__ballot(h == 0 && k < pn && (qx * qx + qy * qy) + qz * qz < rs * rs);
        }
        if (h == 0) P[wave].cen[k] = make_float4(rc.x, rc.y, rc.z, 0.f);
        P[wave].pa[k][2 * h] = ra0;
        P[wave].pa[k][2 * h + 1] = ra1;
        P[wave].pb[k][h] = make_float4(rb0.x, rb0.y, rb1.x, rb1.y);
        // the next piece: the rest of this row, else this wave's next row
        if (c0 + kBandPiece < c1) {
            c0 += kBandPiece;
        } else {
            have = false;
            while (rows.next(t0, t1)) {
                if ((row++ % kBandWaves) != wave) continue;
                c0 = t0;
                c1 = t1;
                have = true;
                break;
            }
        }
        if (have) BAND_FETCH();
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
        __builtin_amdgcn_wave_barrier();
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        float ax = 0.f, ay = 0.f, az = 0.f;
        for (; live; live &= live - 1u) {
            const int j = __builtin_ctz(live);
            const int t = p0 + j;
            const float4 c = P[wave].cen[j];
            const float ex = x - c.x, ey = y - c.y, ez = z - c.z;
            const float qx = ex * ex, qy = ey * ey, qz = ez * ez;
            const float d2 = (qx + qy) + qz;
            bool near = d2 < th.rt2;
            if (th.inc_band) {
                const int4 id = m.tid[t];
                near = near || (id.x == i) | (id.y == i) | (id.z == i) | (id.w == i);
            }
            const bool in11 = valid && !near && d2 < th.g11_2;
            const bool in4 = valid && !near && d2 < th.g4_2 && !(d2 < th.g11_2);
            if (in4) {
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const float4 b = P[wave].pb[j][e];
                    const float4 a0 = P[wave].pa[j][2 * e], a1 = P[wave].pa[j][2 * e + 1];
                    const float g0[6] = {a0.x, a0.y, a0.z, a0.w, b.x, b.y};
                    const float g1[6] = {a1.x, a1.y, a1.z, a1.w, b.z, b.w};
                    gauss_point(x, y, z, g0, ax, ay, az);
                    gauss_point(x, y, z, g1, ax, ay, az);
                }
                ++n4;
            }
            if (in11) {
                const float *g11 = m.g11 + (size_t)t * 11 * kRecG;
#pragma unroll
                for (int q = 0; q < 11; ++q) gauss_point(x, y, z, g11 + q * kRecG, ax, ay, az);
                ++n11;
            }
            if (PREC == 2) { // FP64 mode: every pair's terms added in FP64
                dx += (double)ax;
                dy += (double)ay;
                dz += (double)az;
                ax = ay = az = 0.f;
            }
        }
        if (PREC == 1) {
            two_sum(sx, ccx, ax);
            two_sum(sy, ccy, ay);
            two_sum(sz, ccz, az);
        } else if (PREC == 0) {
            sx += ax;
            sy += ay;
            sz += az;
        }
        // the next piece's stores must follow this piece's reads
        __builtin_amdgcn_wave_barrier();
    }
#undef BAND_FETCH
    if (PREC != 2) {
        dx = (double)sx + (double)ccx;
        dy = (double)sy + (double)ccy;
        dz = (double)sz + (double)ccz;
    }
    red[wave][0][lane] = dx;
    red[wave][1][lane] = dy;
    red[wave][2][lane] = dz;
    n4 = wave_sum_u64(n4);
    n11 = wave_sum_u64(n11);
    if (lane == 0 && cnt) {
        unsigned long long *c = cnt_copy(cnt, blockIdx.x);
        atomicAdd(&c[0], n4);
        atomicAdd(&c[1], n11);
    }
    __syncthreads();
    if (wave == 0) {
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            double v = red[0][c][lane];
#pragma unroll
            for (int w = 1; w < kBandWaves; ++w) v += red[w][c][lane];
            band[(size_t)c * m.npad + i] = v;
        }
    }
}

hipError_t launch_band(const DevMesh &m, const Thresholds &th, int precision, int sub_g1, double *band,
                       unsigned long long *cnt, hipStream_t s)
{
    const dim3 blk(64 * kBandWaves);
    const dim3 grid(8 * ((m.nblk + 7) / 8));
    if (sub_g1) {
        if (precision == 0)
            hipLaunchKernelGGL(k_band<0>, grid, blk, 0, s, m, th, band, cnt);
        else if (precision == 1)
            hipLaunchKernelGGL(k_band<1>, grid, blk, 0, s, m, th, band, cnt);
        else
            hipLaunchKernelGGL(k_band<2>, grid, blk, 0, s, m, th, band, cnt);
    } else {
        if (precision == 0)
            hipLaunchKernelGGL(k_band_piece<0>, grid, blk, 0, s, m, th, band, cnt);
        else if (precision == 1)
            hipLaunchKernelGGL(k_band_piece<1>, grid, blk, 0, s, m, th, band, cnt);
        else
            hipLaunchKernelGGL(k_band_piece<2>, grid, blk, 0, s, m, th, band, cnt);
    }
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Ray tracing.  One wave (64 lanes) per node.
//
// 1. The tets whose centroid lies within r_rt of the node are classified
//    (64 at a time); those whose rule is RT are appended to an LDS list.
// 2. Every 64 listed tets form a batch; lane p prepares pair p: vertex
//    positions relative to the node (from the hi/lo split, so nearby
//    differences are exact to binary32), the six edge normals a_j x a_k in
//    a canonical order (smaller node id first), the four face volumes, a
//    cone bounding the directions that can reach the tet and the rectangle
//    of (row, column) ray indices covering that cone.
// 3. The rays of all rectangles of the batch are processed 64 at a time
//    (lane = one (pair, ray) item): cone test, then the six signed edge
//    volumes d . (a_j x a_k) decide which faces the ray crosses (a face is
//    crossed when its three edge values have one sign; a value of zero
//    counts as positive); every crossing at rho > 0 gives rho = vol_f / sum
//    and the area coordinates; the chord adds to the lane's accumulator.
//    Edge values tiny relative to the normal are recomputed in FP64 from
//    the FP64 relative positions and FP64 directions.
// 4. Lane accumulators are summed across the wave in FP64.
struct RtLds {
    float a[12][64];   // relative vertex positions, [j*3 + c][pair]
    float w[12][64];   // vertex vorticity
    float nrm[18][64]; // canonical edge normals, [e*3 + c][pair]
    float vol[4][64];  // face volumes a_p . (a_q x a_r), face f opposite vertex f
    float cone[4][64]; // unit axis, cos(alpha) (< -1: no culling)
    int meta[64];      // bits 0-2: incident vertex (4 = none); bits 3-8: edge orientation
    int rows[64];      // first row
    int cols[64];      // first column
    int ncol[64];      // columns per row
    int pref[64];      // inclusive prefix sum of the item counts
    int ids[4][64];    // vertex node ids (for the FP64 retest)
};

// LDS of k_rt: the pending list, and either one batch's pair data or (for
// the learned policy) the network's scratch, never live together.
template <bool LEARNED> struct RtShared {
    union {
        RtLds b;
        InferLds n;
    } u;
    int list[128]; // pending ray-traced tets
    int cand[128]; // pairs waiting for the selector
};
template <> struct RtShared<false> {
    union {
        RtLds b;
    } u;
    int list[128];
};

__device__ __forceinline__ float diamond(float c, float s)
{
    // monotone pseudo-angle in [0, 4) of the unit vector (c, s)
    if (s >= 0.f) return c >= 0.f ? s / (c + s) : 1.f - c / (-c + s);
    return c < 0.f ? 2.f - s / (-c - s) : 3.f + c / (c - s);
}

// first index in the ascending array a[0..n) with a[idx] > v (n if none)
__device__ __forceinline__ int upper_bound_f(const float *a, int n, float v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] <= v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

// first index in the ascending array a[0..n) with a[idx] >= v (n if none)
__device__ __forceinline__ int lower_bound_f(const float *a, int n, float v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

__device__ __forceinline__ void cross_canon(const float *A, const float *B, float *N)
{
    N[0] = fmaf(A[1], B[2], -(A[2] * B[1]));
    N[1] = fmaf(A[2], B[0], -(A[0] * B[2]));
    N[2] = fmaf(A[0], B[1], -(A[1] * B[0]));
}

// Pair setup for lane p (tet t, node self at (xh, xl)).  Returns the number
// of candidate rays.
__device__ int rt_setup(const DevMesh &m, const AngTab &ang, RtLds &L, int p, int t, int self, const float *xhv,
                        const float *xlv)
{
    const int4 id4 = m.tid[t];
    const int id[4] = {id4.x, id4.y, id4.z, id4.w};
    float a[4][3];
    int inc = 4;
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const int v = id[j];
        L.ids[j][p] = v;
        if (v == self) inc = j;
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const float vh = m.xh[c * m.npad + v], vl = m.xl[c * m.npad + v];
            a[j][c] = (vh - xhv[c]) + (vl - xlv[c]);
            L.a[j * 3 + c][p] = a[j][c];
            L.w[j * 3 + c][p] = m.om[c * m.npad + v];
        }
    }
    int sig = 0;
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        constexpr int ea[6] = {0, 0, 0, 1, 1, 2}, eb[6] = {1, 2, 3, 2, 3, 3};
        const int j = ea[e], k = eb[e];
        float N[3];
        if (id[j] < id[k]) cross_canon(a[j], a[k], N);
        else {
            cross_canon(a[k], a[j], N);
            sig |= 1 << e;
        }
#pragma unroll
        for (int c = 0; c < 3; ++c) L.nrm[e * 3 + c][p] = N[c];
    }
#pragma unroll
    for (int f = 0; f < 4; ++f) {
        const int pp = f == 0 ? 1 : 0, qq = f <= 1 ? 2 : 1, rr = f <= 2 ? 3 : 2; // ascending, without f
        float N[3];
        cross_canon(a[qq], a[rr], N);
        L.vol[f][p] = fmaf(a[pp][0], N[0], fmaf(a[pp][1], N[1], a[pp][2] * N[2]));
    }
    L.meta[p] = inc | (sig << 3);

    // bounding cone of the directions reaching the tet
    float u[4][3], U[3] = {0.f, 0.f, 0.f};
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float r2 = fmaf(a[j][0], a[j][0], fmaf(a[j][1], a[j][1], a[j][2] * a[j][2]));
        const float s = (j == inc) ? 0.f : __builtin_amdgcn_rsqf(r2);
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            u[j][c] = a[j][c] * s;
            U[c] += u[j][c];
        }
    }
    const float uu = fmaf(U[0], U[0], fmaf(U[1], U[1], U[2] * U[2]));
    float cosa = 2.f;
    if (uu > 0.f) {
        const float s = __builtin_amdgcn_rsqf(uu);
#pragma unroll
        for (int c = 0; c < 3; ++c) U[c] *= s;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j != inc) cosa = fminf(cosa, fmaf(U[0], u[j][0], fmaf(U[1], u[j][1], U[2] * u[j][2])));
    }
    cosa -= 1e-5f; // margin covering the rounding of the cone itself
    const bool cull = uu > 0.f && cosa > 0.02f;
    L.cone[0][p] = U[0];
    L.cone[1][p] = U[1];
    L.cone[2][p] = U[2];
    L.cone[3][p] = cull ? cosa : -2.f;

    // rectangle of ray indices covering the cone
    int r0 = 0, nr = ang.N, c0 = 0, nc = ang.M2;
    if (cull) {
        const float sina = sqrtf(fmaxf(0.f, 1.f - cosa * cosa));
        const float rxy = sqrtf(fmaxf(0.f, 1.f - U[2] * U[2]));
        const bool north = U[2] >= cosa, south = -U[2] >= cosa;
        const float chi = north ? 2.f : fmaf(U[2], cosa, rxy * sina) + 1e-5f;
        const float clo = south ? -2.f : fmaf(U[2], cosa, -rxy * sina) - 1e-5f;
        // rows: cphi descending; rows n with clo <= cphi[n] <= chi
        int lo = 0, hi = ang.N;
        while (lo < hi) { // first n with cphi[n] <= chi
            const int mid = (lo + hi) >> 1;
            if (ang.cphi[mid] > chi) lo = mid + 1;
            else hi = mid;
        }
        r0 = lo;
        lo = r0;
        hi = ang.N;
        while (lo < hi) { // first n with cphi[n] < clo
            const int mid = (lo + hi) >> 1;
            if (ang.cphi[mid] >= clo) lo = mid + 1;
            else hi = mid;
        }
        nr = lo - r0;
        if (!(north || south) && rxy > 0.f && sina < rxy) {
            const float sb = sina / rxy;
            const float cb = sqrtf(fmaxf(0.f, 1.f - sb * sb));
            const float ct = U[0] / rxy, st = U[1] / rxy;
            // endpoints at azimuth theta_U -+ beta
            const float dlo0 = diamond(fmaf(ct, cb, st * sb), fmaf(st, cb, -ct * sb)) - 2e-4f;
            const float dhi0 = diamond(fmaf(ct, cb, -st * sb), fmaf(st, cb, ct * sb)) + 2e-4f;
            const float dlo = dlo0 < 0.f ? dlo0 + 4.f : dlo0;
            const float dhi = dhi0 >= 4.f ? dhi0 - 4.f : dhi0;
            const int jlo = lower_bound_f(ang.dia, ang.M2, dlo); // first column with dia >= dlo
            const int jhi = upper_bound_f(ang.dia, ang.M2, dhi) - 1; // last column with dia <= dhi
            c0 = jlo;
            if (dlo <= dhi) nc = max(0, jhi - jlo + 1);
            else nc = min(ang.M2, (ang.M2 - jlo) + (jhi + 1));
            if (c0 >= ang.M2) c0 -= ang.M2;
        }
    }
    L.rows[p] = r0;
    L.cols[p] = c0;
    L.ncol[p] = nc;
    return nr > 0 && nc > 0 ? nr * nc : 0;
}

// Faces of a tetrahedron: face F is opposite vertex F; its vertices p < q < r
// in local order; edge indices of (p,q), (q,r), (p,r) with the numbering
// 01->0 02->1 03->2 12->3 13->4 23->5.
template <int F> struct Face;
template <> struct Face<0> { static constexpr int p = 1, q = 2, r = 3, epq = 3, eqr = 5, epr = 4; };
template <> struct Face<1> { static constexpr int p = 0, q = 2, r = 3, epq = 1, eqr = 5, epr = 2; };
template <> struct Face<2> { static constexpr int p = 0, q = 1, r = 3, epq = 0, eqr = 4, epr = 2; };
template <> struct Face<3> { static constexpr int p = 0, q = 1, r = 2, epq = 0, eqr = 3, epr = 1; };

struct Chord {
    float rho_n, rho_f, wn[3], wf[3];
    int nh;
};

// Crossing of face F by the ray d: ce[e] = [d, a_j, a_k] (j < k local),
// se[e] its sign (+1 for zero, decided on the canonical value).
template <int F>
__device__ __forceinline__ void face_cross(const RtLds &L, int p, const float (&ce)[6], const int (&se)[6],
                                           Chord &ch)
{
    using FF = Face<F>;
    const int s1 = se[FF::epq], s2 = se[FF::eqr], s3 = -se[FF::epr];
    if (s1 != s2 || s2 != s3) return;
    const float E1 = ce[FF::epq], E2 = ce[FF::eqr], E3 = -ce[FF::epr];
    const float S = (E1 + E2) + E3;
    const float rho = L.vol[F][p] / S;
    if (!(rho > 0.f) || !(rho < 3.0e38f)) return;
    const float lp = E2 / S, lq = E3 / S, lr = E1 / S;
    float w[3];
#pragma unroll
    for (int c = 0; c < 3; ++c)
        w[c] = fmaf(lp, L.w[FF::p * 3 + c][p], fmaf(lq, L.w[FF::q * 3 + c][p], lr * L.w[FF::r * 3 + c][p]));
    const bool first = ch.nh == 0;
    const bool un = first || rho < ch.rho_n;
    const bool uf = first || rho > ch.rho_f;
    ch.rho_n = un ? rho : ch.rho_n;
    ch.rho_f = uf ? rho : ch.rho_f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        ch.wn[c] = un ? w[c] : ch.wn[c];
        ch.wf[c] = uf ? w[c] : ch.wf[c];
    }
    ++ch.nh;
}

// Sign of [d, a_j, a_k] recomputed in FP64 (positions from the hi/lo split,
// FP64 ray direction); canonical operand order (smaller node id first).
__device__ __forceinline__ int edge_sign_f64(const DevMesh &m, const double *d64, int v0, int v1, const float *xhv,
                                          const float *xlv)
{
    double A[3], B[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double xn = (double)xhv[c] + (double)xlv[c];
        A[c] = ((double)m.xh[c * m.npad + v0] + (double)m.xl[c * m.npad + v0]) - xn;
        B[c] = ((double)m.xh[c * m.npad + v1] + (double)m.xl[c * m.npad + v1]) - xn;
    }
    const double N0 = A[1] * B[2] - A[2] * B[1];
    const double N1 = A[2] * B[0] - A[0] * B[2];
    const double N2 = A[0] * B[1] - A[1] * B[0];
    const double c64 = d64[0] * N0 + d64[1] * N1 + d64[2] * N2;
    return c64 >= 0.0 ? 1 : -1;
}

// One (pair, ray) item; adds to (ax, ay, az).  Returns 1 if the ray hits.
__device__ __forceinline__ int rt_item(const DevMesh &m, const AngTab &ang, const RtLds &L, int p, int l,
                                       const float *omx, const float *xhv, const float *xlv, float &ax,
                                       float &ay, float &az, int &retests)
{
    const float4 d = ang.dir[l];
    const float cosa = L.cone[3][p];
    if (cosa > -1.5f) {
        const float dc = fmaf(d.x, L.cone[0][p], fmaf(d.y, L.cone[1][p], d.z * L.cone[2][p]));
        if (dc < cosa) return 0;
    }
    const int meta = L.meta[p];
    const int inc = meta & 7;
    const int sig = meta >> 3;
    float ce[6];
    int se[6];
#pragma unroll
    for (int e = 0; e < 6; ++e) {
        constexpr int ea[6] = {0, 0, 0, 1, 1, 2}, eb[6] = {1, 2, 3, 2, 3, 3};
        ce[e] = 0.f;
        se[e] = 1;
        if (inc == ea[e] || inc == eb[e]) continue; // edge through the node: its faces are skipped
        const float nx = L.nrm[e * 3][p], ny = L.nrm[e * 3 + 1][p], nz = L.nrm[e * 3 + 2][p];
        const float c = fmaf(d.x, nx, fmaf(d.y, ny, d.z * nz));
        int sg = c >= 0.f ? 1 : -1;
        if (fabsf(c) <= 1e-5f * (fabsf(nx) + fabsf(ny) + fabsf(nz))) {
            const int vj = L.ids[ea[e]][p], vk = L.ids[eb[e]][p];
            const bool flip = (sig >> e) & 1;
            sg = edge_sign_f64(m, ang.dir64 + 3 * (size_t)l, flip ? vk : vj, flip ? vj : vk, xhv, xlv);
            ++retests;
        }
        const bool flip = (sig >> e) & 1;
        se[e] = flip ? -sg : sg;
        ce[e] = flip ? -c : c;
    }
    Chord ch;
    ch.nh = 0;
    ch.rho_n = ch.rho_f = 0.f;
#pragma unroll
    for (int c = 0; c < 3; ++c) ch.wn[c] = ch.wf[c] = 0.f;
    if (inc == 4 || inc == 0) face_cross<0>(L, p, ce, se, ch);
    if (inc == 4 || inc == 1) face_cross<1>(L, p, ce, se, ch);
    if (inc == 4 || inc == 2) face_cross<2>(L, p, ce, se, ch);
    if (inc == 4 || inc == 3) face_cross<3>(L, p, ce, se, ch);
    float len;
    if (ch.nh == 0) return 0;
    if (inc != 4) {
        if (ch.nh < 1) return 0;
        // chord from the node (rho = 0, omega_x) to the opposite face
        len = ch.rho_f;
#pragma unroll
        for (int c = 0; c < 3; ++c) ch.wn[c] = omx[c];
    } else if (ch.nh == 1) {
        // one crossing ahead: the point lies inside the tet (a target that is
        // not a vertex of it); the chord starts at the point itself, where the
        // vorticity is the tet's linear field at the point: barycentric
        // weights from the face volumes [a_p, a_q, a_r] (alternating signs)
        const float v0 = L.vol[0][p], v1 = -L.vol[1][p], v2 = L.vol[2][p], v3 = -L.vol[3][p];
        const float D = (v0 + v1) + (v2 + v3);
        if (!(fabsf(D) > 0.f)) return 0;
        const float iD = 1.0f / D;
#pragma unroll
        for (int c = 0; c < 3; ++c)
            ch.wn[c] = (fmaf(v0, L.w[c][p], v1 * L.w[3 + c][p]) + fmaf(v2, L.w[6 + c][p], v3 * L.w[9 + c][p])) * iD;
        len = ch.rho_f;
    } else {
        len = ch.rho_f - ch.rho_n;
    }
    const float h = 0.5f * d.w * len;
    const float sx = ch.wn[0] + ch.wf[0], sy = ch.wn[1] + ch.wf[1], sz = ch.wn[2] + ch.wf[2];
    ax = fmaf(h, fmaf(d.y, sz, -(d.z * sy)), ax);
    ay = fmaf(h, fmaf(d.z, sx, -(d.x * sz)), ay);
    az = fmaf(h, fmaf(d.x, sy, -(d.y * sx)), az);
    return 1;
}

__device__ __forceinline__ double wave_sum_f64(double v)
{
    for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
    return v;
}

__device__ __forceinline__ int wave_incl_scan(int v, int lane)
{
    for (int o = 1; o < 64; o <<= 1) {
        const int u = __shfl_up(v, o, 64);
        if (lane >= o) v += u;
    }
    return v;
}

struct RtAcc {
    float ax, ay, az, sx, sy, sz, cx, cy, cz;
    double dx, dy, dz;
    unsigned long long pairs, hits;
    int retests;
};

// One batch of mcount (<= 64) listed tets: setup, then all candidate rays.
template <int PREC>
__device__ __forceinline__ void acc_add(RtAcc &A, float a0, float a1, float a2)
{
    if (PREC == 0) {
        A.ax += a0;
        A.ay += a1;
        A.az += a2;
    } else if (PREC == 1) {
        two_sum(A.sx, A.cx, a0);
        two_sum(A.sy, A.cy, a1);
        two_sum(A.sz, A.cz, a2);
    } else {
        A.dx += (double)a0;
        A.dy += (double)a1;
        A.dz += (double)a2;
    }
}

template <int PREC>
__device__ __forceinline__ void rt_batch(const DevMesh &m, const AngTab &ang, RtLds &L, const int *list, int mcount,
                                         int lane, int self, const float *xhv, const float *xlv, const float *omx,
                                         RtAcc &A)
{
    int cntp = 0;
    if (lane < mcount) cntp = rt_setup(m, ang, L, lane, list[lane], self, xhv, xlv);
    const int incl = wave_incl_scan(cntp, lane);
    L.pref[lane] = incl;
    __syncthreads();
    const int total = __shfl(incl, 63, 64);
    for (int k0 = 0; k0 < total; k0 += 64) {
        const int k = k0 + lane;
        if (k < total) {
            int lo = 0, hi = mcount - 1;
            while (lo < hi) {
                const int mid = (lo + hi) >> 1;
                if (L.pref[mid] > k) hi = mid;
                else lo = mid + 1;
            }
            const int p = lo;
            const int r = k - (p ? L.pref[p - 1] : 0);
            const int nc = L.ncol[p];
            int row = (int)(((float)r + 0.5f) * (1.0f / (float)nc));
            if (row * nc > r) --row;
            if ((row + 1) * nc <= r) ++row;
            int col = L.cols[p] + (r - row * nc);
            if (col >= ang.M2) col -= ang.M2;
            const int l = (L.rows[p] + row) * ang.M2 + col;
            float a0 = 0.f, a1 = 0.f, a2 = 0.f;
            A.hits += rt_item(m, ang, L, p, l, omx, xhv, xlv, a0, a1, a2, A.retests);
            acc_add<PREC>(A, a0, a1, a2);
        }
    }
    A.pairs += mcount;
    __syncthreads();
}

// The first np (<= NQ) points of a Gauss record g at x, all NQ records
// loaded before any is used (point min(q, np - 1) for q >= np, its term
// dropped; np = 0 adds nothing).
template <int NQ>
__device__ __forceinline__ void gauss_terms(const float *x, const float *g, int np, float &a0, float &a1, float &a2)
{
    float4 ra[NQ];
    float2 rb[NQ];
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        const int qq = min(q, max(np - 1, 0));
        ra[q] = *reinterpret_cast<const float4 *>(g + qq * kRecG);
        rb[q] = *reinterpret_cast<const float2 *>(g + qq * kRecG + 4);
    }
#pragma unroll
    for (int q = 0; q < NQ; ++q) {
        if (q >= np) continue;
        const float rec[6] = {ra[q].x, ra[q].y, ra[q].z, ra[q].w, rb[q].x, rb[q].y};
        gauss_point(x[0], x[1], x[2], rec, a0, a1, a2);
    }
}

// Learned rule choice for a batch of n <= 64 candidate pairs (lane p: tet
// cand[p], p < n): pairs the fixed rule ray-traces whose tet does not
// contain the node.  The pair takes the cheapest Gauss rule whose predicted
// probability of meeting the error budget (the softmax mass of the classes
// up to it) is at least conf_min; if none, it stays ray traced.  Pairs given
// a Gauss rule are evaluated here (no other kernel adds a term for a pair the
// fixed rule ray-traces).  Returns the lane's rule (RULE_RT for p >= n) and
// its tet in *t_out.
template <int PREC>
__device__ __forceinline__ int learned_batch(const DevMesh &m, const LearnParams &lp, InferLds &L, const int *cand,
                                             int n, int lane, const float *xhv, const float *xlv, RtAcc &A,
                                             unsigned long long *n_by_rule, int *t_out)
{
    const PackedNet *W = lp.net;
    const bool act = lane < n;
    const int t = cand[act ? lane : 0];
    *t_out = t;
    const int4 id4 = m.tid[t];
    const int id[4] = {id4.x, id4.y, id4.z, id4.w};
    float a[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const float4 r0 = m.nrec[2 * id[j]], r1 = m.nrec[2 * id[j] + 1];
        a[j][0] = (r0.x - xhv[0]) + (r0.w - xlv[0]);
        a[j][1] = (r0.y - xhv[1]) + (r1.x - xlv[1]);
        a[j][2] = (r0.z - xhv[2]) + (r1.y - xlv[2]);
    }
    float f[16];
    pair_features(a, lp.hbar, false, f);
#pragma unroll
    for (int q = 0; q < 16; ++q) L.x[lane][q] = (__bf16)(act ? (f[q] - W->mu[q]) * W->isg[q] : 0.f);
    __syncthreads();
    mlp_forward_packed(W, L.x, L.z3, lane);
    __syncthreads();
    int rule = RULE_RT;
    if (act) {
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
        const float need = lp.conf_min * se;
        // cumulative sums in class order; the cheapest sufficient class wins
        const float c0 = e[0], c1 = c0 + e[1], c2 = c1 + e[2];
        rule = c2 >= need ? RULE_G11 : RULE_RT;
        rule = c1 >= need ? RULE_G4 : rule;
        rule = c0 >= need ? RULE_G1 : rule;
    }
    // the Gauss terms of the moved pairs: every lane runs the wave's largest
    // rule, unrolled so that the record loads issue together (a lane with a
    // smaller rule reloads its last point and drops the extra terms)
    const int np = !act || rule == RULE_RT ? 0 : rule == RULE_G1 ? 1 : rule == RULE_G4 ? 4 : 11;
    const float *g = np == 11 ? m.g11 + (size_t)t * 11 * kRecG
                     : np == 4 ? m.g4 + (size_t)t * 4 * kRecG : m.g1 + (size_t)t * kRecG;
    float a0 = 0.f, a1 = 0.f, a2 = 0.f;
    if (__ballot(np == 11)) gauss_terms<11>(xhv, g, np, a0, a1, a2);
    else if (__ballot(np == 4)) gauss_terms<4>(xhv, g, np, a0, a1, a2);
    else if (__ballot(np == 1)) gauss_terms<1>(xhv, g, np, a0, a1, a2);
    if (np > 0) {
        acc_add<PREC>(A, a0, a1, a2);
        n_by_rule[0] += rule == RULE_G1;
        n_by_rule[1] += rule == RULE_G4;
        n_by_rule[2] += rule == RULE_G11;
    }
    __syncthreads();
    return rule;
}

// Append the tets t of the lanes with take to list[n..] (wave-uniform n).
__device__ __forceinline__ void list_append(int *list, int &n, bool take, int t, int lane)
{
    const unsigned long long mk = __ballot(take);
    if (take) list[n + __popcll(mk & ((1ull << lane) - 1ull))] = t;
    n += __popcll(mk);
}

// Drop the first `used` entries of list[0..n) (wave-uniform).
__device__ __forceinline__ void list_shift(int *list, int &n, int used, int lane)
{
    const int rest = n - used;
    int keep[2];
#pragma unroll
    for (int k = 0; k < 2; ++k) keep[k] = lane + 64 * k < rest ? list[used + lane + 64 * k] : 0;
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 2; ++k)
        if (lane + 64 * k < rest) list[lane + 64 * k] = keep[k];
    __syncthreads();
    n = rest;
}

// workgroups of k_rt over a node list: two rounds of the chip's wave slots
// at this kernel's four waves per SIMD (the walk's fallback on a moved
// mesh is about 30% of the nodes), few enough that an empty list costs
// nothing beside the kernels that run concurrently
constexpr int kRtListGrid = 8192;

template <int PREC, bool LEARNED>
__global__ void __launch_bounds__(64) k_rt(DevMesh m, Thresholds th, AngTab ang, LearnParams lp, int all_pairs,
                                           double *__restrict__ rtv, unsigned long long *__restrict__ cnt,
                                           const int *__restrict__ node_list, const int *__restrict__ node_count)
{
    __shared__ RtShared<LEARNED> S;
    const int lane = threadIdx.x;
    // with a node list (whose length only the device knows) a grid of at
    // most kRtListGrid workgroups strides over it; without one, one
    // workgroup per node
    const int count = node_list ? *node_count : m.n;
    for (int nk = blockIdx.x; nk < count; nk += gridDim.x) {
        const int self = node_list ? node_list[nk] : nk;
        float xhv[3], xlv[3], omx[3];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            xhv[c] = m.xh[c * m.npad + self];
            xlv[c] = m.xl[c * m.npad + self];
            omx[c] = m.om[c * m.npad + self];
        }
        RtAcc A;
        A.ax = A.ay = A.az = A.sx = A.sy = A.sz = A.cx = A.cy = A.cz = 0.f;
        A.dx = A.dy = A.dz = 0.0;
        A.pairs = A.hits = 0;
        A.retests = 0;
        unsigned long long n_by_rule[3] = {0, 0, 0};
        int nlist = 0, ncand = 0; // uniform

        RowIter rows(m, xhv[0], xhv[1], xhv[2], th.r_rt);
        int t0 = 0, t1 = all_pairs ? m.T : 0;
        bool have = all_pairs ? (m.T > 0) : rows.next(t0, t1);
        while (have) {
            for (int b0 = t0; b0 < t1; b0 += 64) {
                const int t = b0 + lane;
                bool is_rt = false, inc = false;
                if (t < t1) {
                    const int4 id = m.tid[t];
                    inc = (id.x == self) | (id.y == self) | (id.z == self) | (id.w == self);
                    if (all_pairs) is_rt = true;
                    else {
                        const float *g = m.g1 + (size_t)t * kRecG;
                        is_rt = fixed_rule(xhv[0], xhv[1], xhv[2], g[0], g[1], g[2], id, self, th) == RULE_RT;
                    }
                }
                if constexpr (LEARNED) {
                    // the selector's pairs wait for a full batch; the rest are listed now
                    const bool cand = is_rt && !inc;
                    list_append(S.cand, ncand, cand, t, lane);
                    is_rt = is_rt && !cand;
                }
                list_append(S.list, nlist, is_rt, t, lane);
                __syncthreads();
                if (nlist >= 64) {
                    rt_batch<PREC>(m, ang, S.u.b, S.list, 64, lane, self, xhv, xlv, omx, A);
                    list_shift(S.list, nlist, 64, lane);
                }
                if constexpr (LEARNED) {
                    if (ncand >= 64) {
                        int tt;
                        const bool keep = learned_batch<PREC>(m, lp, S.u.n, S.cand, 64, lane, xhv, xlv, A, n_by_rule,
                                                              &tt) == RULE_RT;
                        list_shift(S.cand, ncand, 64, lane);
                        list_append(S.list, nlist, keep, tt, lane);
                        __syncthreads();
                        if (nlist >= 64) {
                            rt_batch<PREC>(m, ang, S.u.b, S.list, 64, lane, self, xhv, xlv, omx, A);
                            list_shift(S.list, nlist, 64, lane);
                        }
                    }
                }
            }
            have = all_pairs ? false : rows.next(t0, t1);
        }
        if constexpr (LEARNED) {
            if (ncand > 0) {
                int tt;
                const bool keep = learned_batch<PREC>(m, lp, S.u.n, S.cand, ncand, lane, xhv, xlv, A, n_by_rule, &tt) ==
                                      RULE_RT && lane < ncand;
                list_append(S.list, nlist, keep, tt, lane);
                __syncthreads();
                if (nlist >= 64) {
                    rt_batch<PREC>(m, ang, S.u.b, S.list, 64, lane, self, xhv, xlv, omx, A);
                    list_shift(S.list, nlist, 64, lane);
                }
            }
        }
        if (nlist > 0) rt_batch<PREC>(m, ang, S.u.b, S.list, nlist, lane, self, xhv, xlv, omx, A);

        double vx, vy, vz;
        if (PREC == 0) {
            vx = A.ax;
            vy = A.ay;
            vz = A.az;
        } else if (PREC == 1) {
            vx = (double)A.sx + (double)A.cx;
            vy = (double)A.sy + (double)A.cy;
            vz = (double)A.sz + (double)A.cz;
        } else {
            vx = A.dx;
            vy = A.dy;
            vz = A.dz;
        }
        vx = wave_sum_f64(vx);
        vy = wave_sum_f64(vy);
        vz = wave_sum_f64(vz);
        const unsigned long long hits = wave_sum_u64(A.hits);
        const unsigned long long rts = wave_sum_u64((unsigned long long)A.retests);
        unsigned long long lr[3];
#pragma unroll
        for (int k = 0; k < 3; ++k) lr[k] = LEARNED ? wave_sum_u64(n_by_rule[k]) : 0;
        if (lane == 0) {
            rtv[self] = vx;
            rtv[m.npad + self] = vy;
            rtv[2 * m.npad + self] = vz;
            if (cnt) {
                unsigned long long *c = cnt_copy(cnt, self);
                atomicAdd(&c[2], A.pairs);
                atomicAdd(&c[3], hits);
                atomicAdd(&c[4], rts);
                if (LEARNED)
                    for (int k = 0; k < 3; ++k) atomicAdd(&c[5 + k], lr[k]);
            }
        }
        __syncthreads(); // the next node reuses the shared arrays
    }
}

// ---------------------------------------------------------------------------
// Ray tracing by walking the mesh (face-manifold meshes: every interior
// face shared by two tets).  Where the boundary is not convex a ray that
// leaves the mesh may enter it again, so a node with a ray that leaves
// before its stop distance (or starts outside) is left to k_rt.
// One wave per node; lane = ray.  Every ray leaves the node through the one
// incident tet whose opposite face it crosses, then crosses face neighbours
// outward: the exit face of one tet is the entry face of the next, decided
// by the same shared edge values, so chords join exactly.  A tet adds its
// chord when its pair with the node is ray traced: for the fixed rule the
// rule's own test on the tet's centroid, for the learned selector that test
// and then a sorted LDS list of the pairs it left ray traced (a subset of
// the fixed rule's), for the pure ray-tracing policy
// every tet.  The walk stops at the boundary or once the ray is farther than
// any ray-traced tet reaches (the largest centroid distance among them plus
// the largest vertex-centroid distance, at most r_stop = r_rt plus that
// distance; the learned selector, which takes pairs off, shortens the
// walks).
//
// A step carries the entry face: its three nodes, their positions relative
// to the node and vorticity, and its three edge values, which all have the
// sign s of the crossing.  The tet across has one more node V (the XOR of
// its four node ids and the face's three), so a step loads one node record
// and forms the three edge values [d, V, P_k]; the exit face is (V, P_k,
// P_k+1) for the one k with [d, V, P_k] of sign s and [d, V, P_k+1] of sign
// -s (the faces through V share those edges, so no two qualify; none does
// only when the ray meets V itself, and the ray ends there).
constexpr int kIncCap = 48;    // incident tets per node (more: left to k_rt)
constexpr int kMaxSteps = 1 << 13; // tets per ray: bounds a walk that stalls on a degenerate crossing

struct WalkLds {
    int list[kSelListCap]; // learned policy: its ray-traced tets, sorted
    // incident tets: the three vertices of the face opposite the node
    float ia[kIncCap][9];  // positions relative to the node
    float iw[kIncCap][9];  // vorticity
    float in[kIncCap][9];  // canonical normals of the edges pq, qr, pr
    float inn[kIncCap][3]; // below this magnitude an edge value takes its sign from FP64: 1e-5 (|nx| + |ny| + |nz|)
    int iid[kIncCap][3];   // node ids of p, q, r
    int imeta[kIncCap];    // bits 0-2: flip of pq, qr, pr
    int inb[kIncCap];      // tet across the face (-1: boundary)
    float ivol[kIncCap];   // [a_p, a_q, a_r]
    float4 icone[kIncCap]; // cone around the face seen from the node: unit axis, cos(half angle) (-2: none)
};

// The learned policy's walk also holds a bounding sphere (radius: the
// largest vertex-centroid distance) of every listed tet that does not
// contain the node: centroid relative to the node and its squared norm.  A
// ray can meet such a tet only inside its sphere, so each ray walks only to
// the far side of the last sphere it passes through (not at all past its
// start if it passes through none).
struct WalkLdsListed : WalkLds {
    float4 lc[kSelListCap];
};


// value [d, A, B] in the given order; when it is too small for its binary32
// sign to be certain (|value| below 1e-5 of the normal's 1-norm; the
// rounding error of either order is near 1e-7 of it), the sign comes from
// FP64 in the canonical order (smaller node id first), so every test of an
// edge takes the same decision whichever tet or order it is evaluated in.
__device__ __forceinline__ float edge_val(const float4 &d, const float *A, int ia, const float *B, int ib,
                                          const DevMesh &m, const double *d64, const float *xhv, const float *xlv,
                                          int &sgn, int &retests)
{
    float N[3];
    cross_canon(A, B, N);
    const float c = fmaf(d.x, N[0], fmaf(d.y, N[1], d.z * N[2]));
    int sg = c >= 0.f ? 1 : -1;
    if (fabsf(c) <= 1e-5f * (fabsf(N[0]) + fabsf(N[1]) + fabsf(N[2]))) {
        const bool flip = ia > ib;
        const int s64 = edge_sign_f64(m, d64, flip ? ib : ia, flip ? ia : ib, xhv, xlv);
        sg = flip ? -s64 : s64;
        ++retests;
    }
    sgn = sg;
    return c;
}

__device__ __forceinline__ bool in_sorted(const int *a, int n, int v)
{
    int lo = 0, hi = n;
    while (lo < hi) {
        const int mid = (lo + hi) >> 1;
        if (a[mid] < v) lo = mid + 1;
        else hi = mid;
    }
    return lo < n && a[lo] == v;
}

// Count the ray-traced tets the wave found and track the farthest centroid
// (g: the tet's centroid).
__device__ __forceinline__ void walk_reach_add(int &n, bool take, const float4 &g, const float *xhv, float &dmax)
{
    n += __popcll(__ballot(take));
    if (take) {
        const float dx = xhv[0] - g.x, dy = xhv[1] - g.y, dz = xhv[2] - g.z;
        dmax = fmaxf(dmax, sqrtf((dx * dx + dy * dy) + dz * dz));
    }
}

// ---------------------------------------------------------------------------
// The learned policy's selection pass (walk meshes): one wave per node scans
// the tets its fixed rule ray-traces, runs the selector on the non-incident
// ones 64 at a time, adds the Gauss terms of the pairs it moves to rtv, and
// leaves the pairs still ray traced (incident ones included) in
// sel_list[node][kSelCap] with their count and farthest centroid distance
// for k_rt_walk, and the node's counts of pairs moved to each Gauss rule
// (added to the counters by the walk once it completes the node: a node the
// walk leaves to k_rt is counted there).  A node with more than kSelCap
// such pairs, or without incident tets the walk can start from, is marked
// with count -1 and left to k_rt (nothing is written for it here).
constexpr int kSelCap = kSelListCap;

__device__ __forceinline__ void sel_add(const DevMesh &m, int *list, int &n, bool take, int t, int lane,
                                        const float *xhv, float &dmax)
{
    const unsigned long long mk = __ballot(take);
    const int pos = n + __popcll(mk & ((1ull << lane) - 1ull));
    if (take && pos < kSelCap) list[pos] = t;
    n += __popcll(mk);
    if (take) {
        const float *g = m.g1 + (size_t)t * kRecG;
        const float dx = xhv[0] - g[0], dy = xhv[1] - g[1], dz = xhv[2] - g[2];
        dmax = fmaxf(dmax, sqrtf((dx * dx + dy * dy) + dz * dz));
    }
}

template <int PREC>
__global__ void __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(3))) k_select(DevMesh m, Thresholds th, LearnParams lp, double *__restrict__ rtv,
                                               int *__restrict__ sel_list, int *__restrict__ sel_n,
                                               float *__restrict__ sel_dmax, int *__restrict__ sel_cnt)
{
    __shared__ InferLds L;
    __shared__ int cand[128];
    const int lane = threadIdx.x;
    const int self = blockIdx.x;
    const int ninc = m.inc_start[self + 1] - m.inc_start[self];
    if (ninc == 0 || ninc > kIncCap) {
        if (lane == 0) sel_n[self] = -1;
        return;
    }
    float xhv[3], xlv[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xhv[c] = m.xh[c * m.npad + self];
        xlv[c] = m.xl[c * m.npad + self];
    }
    RtAcc A;
    A.ax = A.ay = A.az = A.sx = A.sy = A.sz = A.cx = A.cy = A.cz = 0.f;
    A.dx = A.dy = A.dz = 0.0;
    A.pairs = A.hits = 0;
    A.retests = 0;
    unsigned long long n_by_rule[3] = {0, 0, 0};
    int *list = sel_list + (size_t)self * kSelCap;
    int nlist = 0, ncand = 0;
    float dmax = 0.f;
    RowIter rows(m, xhv[0], xhv[1], xhv[2], th.r_rt);
    int t0, t1;
    while (rows.next(t0, t1)) {
        for (int b0 = t0; b0 < t1; b0 += 64) {
            const int t = b0 + lane;
            bool is_rt = false, inc = false;
            if (t < t1) {
                const int4 id = m.tid[t];
                inc = (id.x == self) | (id.y == self) | (id.z == self) | (id.w == self);
                const float *g = m.g1 + (size_t)t * kRecG;
                is_rt = fixed_rule(xhv[0], xhv[1], xhv[2], g[0], g[1], g[2], id, self, th) == RULE_RT;
            }
            const bool c = is_rt && !inc;
            list_append(cand, ncand, c, t, lane);
            sel_add(m, list, nlist, is_rt && !c, t, lane, xhv, dmax);
            __syncthreads();
            if (ncand >= 64) {
                int tt;
                const bool keep = learned_batch<PREC>(m, lp, L, cand, 64, lane, xhv, xlv, A, n_by_rule, &tt) == RULE_RT;
                list_shift(cand, ncand, 64, lane);
                sel_add(m, list, nlist, keep, tt, lane, xhv, dmax);
            }
        }
    }
    if (ncand > 0) {
        int tt;
        const bool keep =
            learned_batch<PREC>(m, lp, L, cand, ncand, lane, xhv, xlv, A, n_by_rule, &tt) == RULE_RT && lane < ncand;
        sel_add(m, list, nlist, keep, tt, lane, xhv, dmax);
    }
    for (int o = 32; o > 0; o >>= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, o, 64));
    if (nlist > kSelCap) {
        if (lane == 0) sel_n[self] = -1;
        return;
    }
    double vx, vy, vz;
    if (PREC == 0) {
        vx = A.ax;
        vy = A.ay;
        vz = A.az;
    } else if (PREC == 1) {
        vx = (double)A.sx + (double)A.cx;
        vy = (double)A.sy + (double)A.cy;
        vz = (double)A.sz + (double)A.cz;
    } else {
        vx = A.dx;
        vy = A.dy;
        vz = A.dz;
    }
    vx = wave_sum_f64(vx);
    vy = wave_sum_f64(vy);
    vz = wave_sum_f64(vz);
    unsigned long long lr[3];
#pragma unroll
    for (int k = 0; k < 3; ++k) lr[k] = wave_sum_u64(n_by_rule[k]);
    if (lane == 0) {
        rtv[self] = vx;
        rtv[m.npad + self] = vy;
        rtv[2 * m.npad + self] = vz;
        sel_n[self] = nlist;
        sel_dmax[self] = dmax;
        for (int k = 0; k < 3; ++k) sel_cnt[3 * (size_t)self + k] = (int)lr[k];
    }
}

// LISTED: the ray-traced tets of every node come from k_select (which also
// wrote the node's Gauss terms to rtv: the walk adds to them).
template <int PREC, bool LISTED>
__global__ void __launch_bounds__(64) k_rt_walk(DevMesh m, Thresholds th, AngTab ang, int all_pairs, float r_stop,
                                                int exit_fb, double *__restrict__ rtv,
                                                unsigned long long *__restrict__ cnt, int *__restrict__ fallback,
                                                int *__restrict__ n_fallback, const int *__restrict__ sel_list,
                                                const int *__restrict__ sel_n, const float *__restrict__ sel_dmax,
                                                const int *__restrict__ sel_cnt)
{
    __shared__ typename std::conditional<LISTED, WalkLdsListed, WalkLds>::type W;
    const int lane = threadIdx.x;
    const int self = blockIdx.x;
    float xhv[3], xlv[3], omx[3];
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        xhv[c] = m.xh[c * m.npad + self];
        xlv[c] = m.xl[c * m.npad + self];
        omx[c] = m.om[c * m.npad + self];
    }
    RtAcc A;
    A.ax = A.ay = A.az = A.sx = A.sy = A.sz = A.cx = A.cy = A.cz = 0.f;
    A.dx = A.dy = A.dz = 0.0;
    A.pairs = A.hits = 0;
    A.retests = 0;

    // ---- A. ray-traced tets of the node (not needed when every pair is):
    // their count and the farthest centroid; the learned policy's list
    int nlist = 0, n_lc = 0;
    float stop = r_stop;
    if (!all_pairs) {
        float dmax = 0.f;
        if constexpr (LISTED) {
            nlist = sel_n[self];
            if (nlist < 0) {
                if (lane == 0) fallback[atomicAdd(n_fallback, 1)] = self;
                return;
            }
            for (int k0 = 0; k0 < nlist; k0 += 64) {
                const int k = k0 + lane;
                bool take = false;
                float4 c = make_float4(0.f, 0.f, 0.f, 0.f);
                if (k < nlist) {
                    const int t = sel_list[(size_t)self * kSelCap + k];
                    W.list[k] = t;
                    const int4 id = m.tid[t];
                    const float *g = m.g1 + (size_t)t * kRecG;
                    c.x = (g[0] - xhv[0]) - xlv[0];
                    c.y = (g[1] - xhv[1]) - xlv[1];
                    c.z = (g[2] - xhv[2]) - xlv[2];
                    c.w = (c.x * c.x + c.y * c.y) + c.z * c.z;
                    take = !((id.x == self) | (id.y == self) | (id.z == self) | (id.w == self));
                }
                const unsigned long long mk = __ballot(take);
                if (take) W.lc[n_lc + __popcll(mk & ((1ull << lane) - 1ull))] = c;
                n_lc += __popcll(mk);
            }
            dmax = sel_dmax[self];
            // sort the list (bitonic, padded with INT_MAX)
            int np2 = 1;
            while (np2 < nlist) np2 <<= 1;
            for (int k = nlist + lane; k < np2; k += 64) W.list[k] = 0x7fffffff;
            __syncthreads();
            for (int size = 2; size <= np2; size <<= 1)
                for (int stride = size >> 1; stride > 0; stride >>= 1) {
                    for (int k = lane; k < np2 / 2; k += 64) {
                        const int i = 2 * k - (k & (stride - 1));
                        const int j = i + stride;
                        const bool up = (i & size) == 0;
                        const int a = W.list[i], b = W.list[j];
                        if ((a > b) == up) {
                            W.list[i] = b;
                            W.list[j] = a;
                        }
                    }
                    __syncthreads();
                }
        } else {
            // chunks of 64 tets of a bin row, the next chunk's ids and
            // centroids loaded while the current one is tested
            RowIter rows(m, xhv[0], xhv[1], xhv[2], th.r_rt);
            int t0 = 0, t1 = 0;
            bool have = rows.next(t0, t1);
            int b0 = t0;
            int4 id_n = make_int4(-1, -1, -1, -1);
            float4 g_n = make_float4(0.f, 0.f, 0.f, 0.f);
            if (have && b0 + lane < t1) {
                id_n = m.tid[b0 + lane];
                g_n = *reinterpret_cast<const float4 *>(m.g1 + (size_t)(b0 + lane) * kRecG);
            }
            while (have) {
                const bool tv = b0 + lane < t1;
                const int4 id = id_n;
                const float4 g = g_n;
                if (b0 + 64 < t1) {
                    b0 += 64;
                } else {
                    have = rows.next(t0, t1);
                    b0 = t0;
                }
                if (have && b0 + lane < t1) {
                    id_n = m.tid[b0 + lane];
                    g_n = *reinterpret_cast<const float4 *>(m.g1 + (size_t)(b0 + lane) * kRecG);
                }
                const bool is_rt = tv && fixed_rule(xhv[0], xhv[1], xhv[2], g.x, g.y, g.z, id, self, th) == RULE_RT;
                walk_reach_add(nlist, is_rt, g, xhv, dmax);
            }
            for (int o = 32; o > 0; o >>= 1) dmax = fmaxf(dmax, __shfl_xor(dmax, o, 64));
        }
        stop = fminf(r_stop, (dmax + th.vc) * (1.f + 1e-4f) + 1e-6f);
    }

    // ---- B. incident tets: the face opposite the node, its neighbour
    const int i0 = m.inc_start[self], i1 = m.inc_start[self + 1];
    const int ninc = i1 - i0;
    // a point that is no vertex of the mesh (inside a tet, or outside the
    // mesh) has no incident tet to start from: the candidate kernel takes it
    if (ninc > kIncCap || ninc == 0) {
        if (lane == 0) fallback[atomicAdd(n_fallback, 1)] = self;
        return;
    }
    if (lane < ninc) {
        const int t = m.inc_list[i0 + lane];
        const int4 id4 = m.tid[t];
        const int id[4] = {id4.x, id4.y, id4.z, id4.w};
        const int4 nb4 = m.nbr[t];
        const int nb[4] = {nb4.x, nb4.y, nb4.z, nb4.w};
        int f = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (id[j] == self) f = j;
        int v[3], k = 0;
#pragma unroll
        for (int j = 0; j < 4; ++j)
            if (j != f) v[k++] = j;
        float a[3][3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const int nid = id[v[q]];
            W.iid[lane][q] = nid;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                a[q][c] = (m.xh[c * m.npad + nid] - xhv[c]) + (m.xl[c * m.npad + nid] - xlv[c]);
                W.ia[lane][3 * q + c] = a[q][c];
                W.iw[lane][3 * q + c] = m.om[c * m.npad + nid];
            }
        }
        // edges pq (0,1), qr (1,2), pr (0,2) in canonical order
        const int ep[3][2] = {{0, 1}, {1, 2}, {0, 2}};
        int flips = 0;
#pragma unroll
        for (int e = 0; e < 3; ++e) {
            const int x0 = ep[e][0], x1 = ep[e][1];
            float N[3];
            if (id[v[x0]] < id[v[x1]]) cross_canon(a[x0], a[x1], N);
            else {
                cross_canon(a[x1], a[x0], N);
                flips |= 1 << e;
            }
#pragma unroll
            for (int c = 0; c < 3; ++c) W.in[lane][3 * e + c] = N[c];
            W.inn[lane][e] = 1e-5f * (fabsf(N[0]) + fabsf(N[1]) + fabsf(N[2]));
        }
        float N[3];
        cross_canon(a[1], a[2], N);
        W.ivol[lane] = fmaf(a[0][0], N[0], fmaf(a[0][1], N[1], a[0][2] * N[2]));
        W.imeta[lane] = flips;
        W.inb[lane] = nb[f];
        // the directions that enter this tet form the spherical triangle of
        // the face; a cap narrower than a hemisphere that holds its three
        // corners holds all of it
        float u[3][3], ax[3] = {0.f, 0.f, 0.f};
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            const float il = 1.f / sqrtf((a[q][0] * a[q][0] + a[q][1] * a[q][1]) + a[q][2] * a[q][2]);
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                u[q][c] = a[q][c] * il;
                ax[c] += u[q][c];
            }
        }
        const float iax = 1.f / sqrtf((ax[0] * ax[0] + ax[1] * ax[1]) + ax[2] * ax[2]);
        float cmin = 1.f;
#pragma unroll
        for (int q = 0; q < 3; ++q) cmin = fminf(cmin, (ax[0] * u[q][0] + ax[1] * u[q][1] + ax[2] * u[q][2]) * iax);
        W.icone[lane] = make_float4(ax[0] * iax, ax[1] * iax, ax[2] * iax, cmin > 0.02f ? cmin - 1e-5f : -2.f);
    }
    __syncthreads();

    // ---- C. rays, 8 x 8 blocks of (row, column) per step so that the rays
    // of the wave point into a small solid angle
    const int bcols = (ang.M2 + 7) >> 3, nblk = ((ang.N + 7) >> 3) * bcols;
    // exit_fb (a mesh whose boundary is not convex): a ray that leaves the
    // mesh before its stop distance (or never enters it) could enter it again
    // beyond; the node is then left to the candidate kernel, which finds
    // every tet a ray meets
    bool early = false;
    for (int bi = 0; bi < nblk; ++bi) {
        if (exit_fb && __ballot(early)) {
            if (lane == 0) fallback[atomicAdd(n_fallback, 1)] = self;
            return;
        }
        const int row = 8 * (bi / bcols) + (lane >> 3), col = 8 * (bi % bcols) + (lane & 7);
        const bool valid = row < ang.N && col < ang.M2;
        const int l = valid ? row * ang.M2 + col : 0;
        const float4 d = ang.dir[l];
        const double *d64 = ang.dir64 + 3 * (size_t)l;
        // start: the incident tet whose opposite face the ray crosses (tets
        // whose cone no ray of the wave enters are skipped)
        int start = -1, sg = 1;
        float rho = 0.f, w_in[3] = {0.f, 0.f, 0.f}, cf[3] = {0.f, 0.f, 0.f};
        for (int i = 0; i < ninc; ++i) {
            if (!__ballot(valid && start < 0)) break;
            const float4 cone = W.icone[i];
            const bool pass = valid && start < 0 && fmaf(d.x, cone.x, fmaf(d.y, cone.y, d.z * cone.z)) >= cone.w;
            if (!__ballot(pass)) continue;
            if (!pass) continue;
            const int meta = W.imeta[i];
            float ce[3];
            int se[3];
#pragma unroll
            for (int e = 0; e < 3; ++e) {
                const float nx = W.in[i][3 * e], ny = W.in[i][3 * e + 1], nz = W.in[i][3 * e + 2];
                const float c = fmaf(d.x, nx, fmaf(d.y, ny, d.z * nz));
                int sg = c >= 0.f ? 1 : -1;
                if (fabsf(c) <= W.inn[i][e]) {
                    const int ep0[3] = {0, 1, 0}, ep1[3] = {1, 2, 2};
                    const int u0 = W.iid[i][ep0[e]], u1 = W.iid[i][ep1[e]];
                    const bool fl = (meta >> e) & 1;
                    sg = edge_sign_f64(m, d64, fl ? u1 : u0, fl ? u0 : u1, xhv, xlv);
                    ++A.retests;
                }
                const bool fl = (meta >> e) & 1;
                se[e] = fl ? -sg : sg;
                ce[e] = fl ? -c : c;
            }
            // face (p, q, r): [d,p,q] = ce0, [d,q,r] = ce1, [d,r,p] = -ce2
            if (se[0] != se[1] || se[1] != -se[2]) continue;
            const float E1 = ce[0], E2 = ce[1], E3 = -ce[2];
            const float Sm = (E1 + E2) + E3;
            // one reciprocal for the chord and the three weights, as in the
            // walk's steps
            const float inv = __builtin_amdgcn_rcpf(Sm);
            const float r = W.ivol[i] * inv;
            if (!(r > 0.f) || !(r < 3.0e38f)) continue;
            const float lp_ = E2 * inv, lq = E3 * inv, lr = E1 * inv;
#pragma unroll
            for (int c = 0; c < 3; ++c)
                w_in[c] = fmaf(lp_, W.iw[i][c], fmaf(lq, W.iw[i][3 + c], lr * W.iw[i][6 + c]));
            rho = r;
            start = i;
            cf[0] = E1;
            cf[1] = E2;
            cf[2] = E3;
            sg = se[0];
        }
        if (!valid) continue;
        if (start < 0) {
            early = true;
            continue;
        }
        {
            const float h = 0.5f * d.w * rho;
            const float sx = omx[0] + w_in[0], sy = omx[1] + w_in[1], sz = omx[2] + w_in[2];
            acc_add<PREC>(A, h * fmaf(d.y, sz, -(d.z * sy)), h * fmaf(d.z, sx, -(d.x * sz)),
                          h * fmaf(d.x, sy, -(d.y * sx)));
            ++A.hits;
        }
        // the learned policy: this ray's last listed sphere
        float stop_r = stop;
        if constexpr (LISTED) {
            const float vcm = th.vc * (1.f + 1e-4f) + 1e-6f, vc2 = vcm * vcm;
            float sr = 0.f;
            for (int k = 0; k < n_lc; ++k) {
                const float4 c = W.lc[k];
                const float t = fmaf(c.x, d.x, fmaf(c.y, d.y, c.z * d.z));
                if (c.w - t * t <= vc2 && t + vcm > sr) sr = t + vcm;
            }
            stop_r = fminf(stop, sr * (1.f + 1e-4f) + 1e-6f);
        }
        // the entry face (P0, P1, P2) and its values [d,P0,P1], [d,P1,P2],
        // [d,P2,P0] (all of sign sg)
        int T = W.inb[start];
        int e[3];
        float P[3][3], Wv[3][3];
#pragma unroll
        for (int q = 0; q < 3; ++q) {
            e[q] = W.iid[start][q];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                P[q][c] = W.ia[start][3 * q + c];
                Wv[q][c] = W.iw[start][3 * q + c];
            }
        }
        // compensated mode: the chords of one ray summed in FP32, the ray's
        // sum added to the node's compensated sum
        float ray[3] = {0.f, 0.f, 0.f};
        int steps = 0;
        while (T >= 0 && rho < stop_r && steps < kMaxSteps) {
            ++steps;
            const int4 id4 = m.tid[T];
            const int4 nb4 = m.nbr[T];
            float4 cen = make_float4(0.f, 0.f, 0.f, 0.f);
            if (!all_pairs) cen = *reinterpret_cast<const float4 *>(m.g1 + (size_t)T * kRecG);
            // the node of T off the entry face
            const int v = (id4.x ^ id4.y ^ id4.z ^ id4.w) ^ (e[0] ^ e[1] ^ e[2]);
            const float4 r0 = m.nrec[2 * v], r1 = m.nrec[2 * v + 1];
            const float wz = m.om[2 * m.npad + v];
            const float av[3] = {(r0.x - xhv[0]) + (r0.w - xlv[0]), (r0.y - xhv[1]) + (r1.x - xlv[1]),
                                 (r0.z - xhv[2]) + (r1.y - xlv[2])};
            const float wv[3] = {r1.z, r1.w, wz};
            float cv[3];
            int sv[3];
#pragma unroll
            for (int k = 0; k < 3; ++k) cv[k] = edge_val(d, av, v, P[k], e[k], m, d64, xhv, xlv, sv[k], A.retests);
            const bool x0 = sv[0] == sg && sv[1] != sg;
            const bool x1 = sv[1] == sg && sv[2] != sg;
            const bool x2 = sv[2] == sg && sv[0] != sg;
            if (!(x0 || x1 || x2)) break; // the ray meets V: end it here
            // exit face (V, A, B) = (V, P_k, P_k+1); O = P_k+2 is the node of T off it
            float pa[3], pb[3], wa[3], wb[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                pa[c] = x0 ? P[0][c] : (x1 ? P[1][c] : P[2][c]);
                pb[c] = x0 ? P[1][c] : (x1 ? P[2][c] : P[0][c]);
                wa[c] = x0 ? Wv[0][c] : (x1 ? Wv[1][c] : Wv[2][c]);
                wb[c] = x0 ? Wv[1][c] : (x1 ? Wv[2][c] : Wv[0][c]);
            }
            const int ea = x0 ? e[0] : (x1 ? e[1] : e[2]);
            const int eb = x0 ? e[1] : (x1 ? e[2] : e[0]);
            const int eo = x0 ? e[2] : (x1 ? e[0] : e[1]);
            const float cVA = x0 ? cv[0] : (x1 ? cv[1] : cv[2]);
            const float cAB = x0 ? cf[0] : (x1 ? cf[1] : cf[2]);
            const float cBV = -(x0 ? cv[1] : (x1 ? cv[2] : cv[0]));
            const float Sm = (cVA + cAB) + cBV;
            float N[3];
            cross_canon(pa, pb, N);
            const float vol = fmaf(av[0], N[0], fmaf(av[1], N[1], av[2] * N[2]));
            const float inv = __builtin_amdgcn_rcpf(Sm);
            const float rout = vol * inv;
            if (!(rout < 3.0e38f) || !(rout > -3.0e38f)) break; // degenerate face: end the ray
            const float lv = cAB * inv, la = cBV * inv, lb = cVA * inv;
            float wout[3];
#pragma unroll
            for (int c = 0; c < 3; ++c) wout[c] = fmaf(lv, wv[c], fmaf(la, wa[c], lb * wb[c]));
            const float r_out = fmaxf(rout, rho);
            // the fixed rule's test: past its first segment a ray meets no tet
            // incident to the node (such a tet lies in its own cone from the
            // node), so only the distance comparison remains; the selector's
            // list holds only pairs the fixed rule ray-traces
            bool take = true;
            if (!all_pairs) {
                const float ex = xhv[0] - cen.x, ey = xhv[1] - cen.y, ez = xhv[2] - cen.z;
                const float qx = ex * ex, qy = ey * ey, qz = ez * ez;
                take = (qx + qy) + qz < th.rt2;
                if constexpr (LISTED) take = take && in_sorted(W.list, nlist, T);
            }
            if (take) {
                const float h = 0.5f * d.w * (r_out - rho);
                const float sx = w_in[0] + wout[0], sy = w_in[1] + wout[1], sz = w_in[2] + wout[2];
                const float a0 = h * fmaf(d.y, sz, -(d.z * sy)), a1 = h * fmaf(d.z, sx, -(d.x * sz)),
                            a2 = h * fmaf(d.x, sy, -(d.y * sx));
                if (PREC == 1) {
                    ray[0] += a0;
                    ray[1] += a1;
                    ray[2] += a2;
                } else {
                    acc_add<PREC>(A, a0, a1, a2);
                }
                ++A.hits;
            }
            // across the exit face: the face of T opposite O
            T = id4.x == eo ? nb4.x : (id4.y == eo ? nb4.y : (id4.z == eo ? nb4.z : nb4.w));
            rho = r_out;
            e[0] = v;
            e[1] = ea;
            e[2] = eb;
            cf[0] = cVA;
            cf[1] = cAB;
            cf[2] = cBV;
#pragma unroll
            for (int c = 0; c < 3; ++c) {
                P[0][c] = av[c];
                P[1][c] = pa[c];
                P[2][c] = pb[c];
                Wv[0][c] = wv[c];
                Wv[1][c] = wa[c];
                Wv[2][c] = wb[c];
                w_in[c] = wout[c];
            }
        }
        if (PREC == 1) acc_add<1>(A, ray[0], ray[1], ray[2]);
        early = early || (T < 0 && rho < stop_r);
    }
    if (exit_fb && __ballot(early)) {
        if (lane == 0) fallback[atomicAdd(n_fallback, 1)] = self;
        return;
    }
    A.pairs = all_pairs ? (unsigned long long)m.T : (unsigned long long)nlist;

    double vx, vy, vz;
    if (PREC == 0) {
        vx = A.ax;
        vy = A.ay;
        vz = A.az;
    } else if (PREC == 1) {
        vx = (double)A.sx + (double)A.cx;
        vy = (double)A.sy + (double)A.cy;
        vz = (double)A.sz + (double)A.cz;
    } else {
        vx = A.dx;
        vy = A.dy;
        vz = A.dz;
    }
    vx = wave_sum_f64(vx);
    vy = wave_sum_f64(vy);
    vz = wave_sum_f64(vz);
    const unsigned long long hits = wave_sum_u64(A.hits);
    const unsigned long long rts = wave_sum_u64((unsigned long long)A.retests);
    if (lane == 0) {
        if (LISTED) {
            vx += rtv[self];
            vy += rtv[m.npad + self];
            vz += rtv[2 * m.npad + self];
        }
        rtv[self] = vx;
        rtv[m.npad + self] = vy;
        rtv[2 * m.npad + self] = vz;
        if (cnt) {
            unsigned long long *c = cnt_copy(cnt, self);
            atomicAdd(&c[2], A.pairs);
            atomicAdd(&c[3], hits);
            atomicAdd(&c[4], rts);
            if (LISTED)
                for (int k = 0; k < 3; ++k) atomicAdd(&c[5 + k], (unsigned long long)sel_cnt[3 * (size_t)self + k]);
        }
    }
}

hipError_t launch_rt(const DevMesh &m, const Thresholds &th, const AngTab &ang, const LearnParams &lp,
                     int all_pairs, int precision, double *rtv, unsigned long long *cnt, const int *node_list,
                     const int *node_count, hipStream_t s)
{
    if (m.n == 0) return hipSuccess;
    const bool L = lp.net != nullptr;
    const int grid = node_list ? std::min(m.n, kRtListGrid) : m.n;
#define BS_RT(P, LL)                                                                                               \
    hipLaunchKernelGGL((k_rt<P, LL>), dim3(grid), dim3(64), 0, s, m, th, ang, lp, all_pairs, rtv, cnt, node_list, \
                       node_count)
    if (precision == 0) {
        if (L) BS_RT(0, true); else BS_RT(0, false);
    } else if (precision == 1) {
        if (L) BS_RT(1, true); else BS_RT(1, false);
    } else {
        if (L) BS_RT(2, true); else BS_RT(2, false);
    }
#undef BS_RT
    return hipGetLastError();
}

hipError_t launch_select(const DevMesh &m, const Thresholds &th, const LearnParams &lp, int precision, double *rtv,
                         int *sel_list, int *sel_n, float *sel_dmax, int *sel_cnt, hipStream_t s)
{
    if (m.n == 0) return hipSuccess;
    if (precision == 0)
        hipLaunchKernelGGL(k_select<0>, dim3(m.n), dim3(64), 0, s, m, th, lp, rtv, sel_list, sel_n, sel_dmax, sel_cnt);
    else if (precision == 1)
        hipLaunchKernelGGL(k_select<1>, dim3(m.n), dim3(64), 0, s, m, th, lp, rtv, sel_list, sel_n, sel_dmax, sel_cnt);
    else
        hipLaunchKernelGGL(k_select<2>, dim3(m.n), dim3(64), 0, s, m, th, lp, rtv, sel_list, sel_n, sel_dmax, sel_cnt);
    return hipGetLastError();
}

hipError_t launch_rt_walk(const DevMesh &m, const Thresholds &th, const AngTab &ang, int all_pairs, float r_stop,
                          int exit_fb, int precision, double *rtv, unsigned long long *cnt, int *fallback,
                          int *n_fallback, const int *sel_list, const int *sel_n, const float *sel_dmax,
                          const int *sel_cnt, hipStream_t s)
{
    if (m.n == 0) return hipSuccess;
    const bool L = sel_n != nullptr;
#define BS_RW(P, LL)                                                                                               \
    hipLaunchKernelGGL((k_rt_walk<P, LL>), dim3(m.n), dim3(64), 0, s, m, th, ang, all_pairs, r_stop, exit_fb, rtv, \
                       cnt, fallback, n_fallback, sel_list, sel_n, sel_dmax, sel_cnt)
    if (precision == 0) {
        if (L) BS_RW(0, true); else BS_RW(0, false);
    } else if (precision == 1) {
        if (L) BS_RW(1, true); else BS_RW(1, false);
    } else {
        if (L) BS_RW(2, true); else BS_RW(2, false);
    }
#undef BS_RW
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_combine(int n, int first, int npad, const int *__restrict__ node_orig,
                                                 const double *__restrict__ part, int splits,
                                                 const double *__restrict__ band, const double *__restrict__ rtv,
                                                 double *__restrict__ vel, int *__restrict__ nonfinite)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= n) return;
    const int o = node_orig[k];
    const int i = first + k;
    bool bad = false;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        double v = 0.0;
        for (int s = 0; s < splits; ++s) v += part[((size_t)s * 3 + c) * npad + i];
        if (band) v += band[(size_t)c * npad + i];
        if (rtv) v += rtv[(size_t)c * npad + i];
        vel[3 * (size_t)o + c] = v;
        bad |= !isfinite(v);
    }
    if (bad) atomicOr(nonfinite, 1);
}

hipError_t launch_combine(const DevMesh &m, const int *node_orig, const double *part, int splits,
                          const double *band, const double *rtv, double *vel, int *nonfinite, hipStream_t s)
{
    if (m.n == 0) return hipSuccess;
    hipLaunchKernelGGL(k_combine, dim3((m.n + 255) / 256), dim3(256), 0, s, m.n, m.blk0 * kBlockNodes, m.npad,
                       node_orig, part, splits, band, rtv, vel, nonfinite);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Static scratch of the no-allocation evaluation (bs_eval_velocity_noalloc):
// partial sums, counters and lists live here instead of in mesh-owned
// buffers.  In host code the array's name is only a stand-in for the symbol;
// its device address comes from hipGetSymbolAddress, looked up once per
// device with that device current.

static __device__ __align__(256) unsigned char scratch[kScratchBytes];

namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
void *g_scratch_addr[kMaxScratchDevices];
hipError_t g_scratch_rc[kMaxScratchDevices];
bool g_scratch_done[kMaxScratchDevices];
} // namespace

hipError_t scratch_setup(int device)
{
    if (device < 0 || device >= kMaxScratchDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_done[device]) {
        void *ptr = nullptr;
        const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
        g_scratch_rc[device] = e;
        g_scratch_addr[device] = e == hipSuccess ? ptr : nullptr;
        g_scratch_done[device] = true;
    }
    return g_scratch_rc[device];
}

void *scratch_ptr(int device)
{
    if (device < 0 || device >= kMaxScratchDevices) return nullptr;
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    return g_scratch_done[device] ? g_scratch_addr[device] : nullptr;
}

__global__ void __launch_bounds__(256) k_fill_zero(unsigned *__restrict__ p, size_t words)
{
    for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < words; i += (size_t)gridDim.x * 256) p[i] = 0u;
}

hipError_t launch_fill_zero(void *p, size_t words, hipStream_t s)
{
    if (words == 0) return hipSuccess;
    const unsigned blocks = (unsigned)std::min<size_t>((words + 255) / 256, 1024);
    hipLaunchKernelGGL(k_fill_zero, dim3(blocks), dim3(256), 0, s, (unsigned *)p, words);
    return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Velocity gradient of the piecewise-linear interpolant of nodal velocities
// (FP64).  Per tet: with E = [x1-x0, x2-x0, x3-x0] and D = [v1-v0, v2-v0,
// v3-v0] (columns), the interpolant's gradient is G = D E^-1, whose rows of
// E^-1 are the cross products of pairs of edges over det E; tg[t] holds
// |T| G (9 values, G[a][b] = dv_a/dx_b) and |T|.  Per node: the mean of G
// over its incident tets weighted by their volumes, in the incident list's
// order, written in input numbering (0 for a node without tets).
__global__ void __launch_bounds__(256) k_tet_grad(DevMesh m, const int *__restrict__ node_orig,
                                                  const double *__restrict__ vel, double *__restrict__ tg)
{
    const int t = blockIdx.x * 256 + threadIdx.x;
    if (t >= m.T) return;
    const int4 id4 = m.tid[t];
    const int id[4] = {id4.x, id4.y, id4.z, id4.w};
    double x[4][3], v[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j) {
        const size_t o = 3 * (size_t)node_orig[id[j]];
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            x[j][c] = (double)m.xh[c * m.npad + id[j]] + (double)m.xl[c * m.npad + id[j]];
            v[j][c] = vel[o + c];
        }
    }
    double e[3][3], dv[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k)
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            e[k][c] = x[k + 1][c] - x[0][c];
            dv[k][c] = v[k + 1][c] - v[0][c];
        }
    double r[3][3];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
        const double *p = e[(k + 1) % 3], *q = e[(k + 2) % 3];
        r[k][0] = p[1] * q[2] - p[2] * q[1];
        r[k][1] = p[2] * q[0] - p[0] * q[2];
        r[k][2] = p[0] * q[1] - p[1] * q[0];
    }
    const double det = e[0][0] * r[0][0] + e[0][1] * r[0][1] + e[0][2] * r[0][2];
    // |T| G = (|det| / 6) D E^-1 = (sign(det) / 6) sum_k dv_k r_k^T
    const double w = (det < 0.0 ? -1.0 : 1.0) / 6.0;
    double *o = tg + 10 * (size_t)t;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
        for (int b = 0; b < 3; ++b)
            o[3 * a + b] = w * ((dv[0][a] * r[0][b] + dv[1][a] * r[1][b]) + dv[2][a] * r[2][b]);
    o[9] = fabs(det) / 6.0;
}

__global__ void __launch_bounds__(256) k_node_grad(DevMesh m, const int *__restrict__ node_orig,
                                                   const double *__restrict__ tg, double *__restrict__ grad)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= m.n) return;
    double g[9] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0}, vs = 0.0;
    for (int p = m.inc_start[k]; p < m.inc_start[k + 1]; ++p) {
        const double *o = tg + 10 * (size_t)m.inc_list[p];
#pragma unroll
        for (int q = 0; q < 9; ++q) g[q] += o[q];
        vs += o[9];
    }
    const double inv = vs > 0.0 ? 1.0 / vs : 0.0;
    double *out = grad + 9 * (size_t)node_orig[k];
#pragma unroll
    for (int q = 0; q < 9; ++q) out[q] = g[q] * inv;
}

// Vortex stretching rate of every node, (omega . grad) v = G omega, from
// the nodal gradients (input order) and the nodal vorticity (FP64, input
// order), in the order ((G_a0 w0 + G_a1 w1) + G_a2 w2).
__global__ void __launch_bounds__(256) k_stretch(int n, const double *__restrict__ grad, const double *__restrict__ om,
                                                 double *__restrict__ rate)
{
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double *g = grad + 9 * (size_t)i;
    const double w0 = om[3 * (size_t)i], w1 = om[3 * (size_t)i + 1], w2 = om[3 * (size_t)i + 2];
#pragma unroll
    for (int a = 0; a < 3; ++a) rate[3 * (size_t)i + a] = (g[3 * a] * w0 + g[3 * a + 1] * w1) + g[3 * a + 2] * w2;
}

hipError_t launch_stretching(int n, const double *grad, const double *om, double *rate, hipStream_t s)
{
    if (n > 0) hipLaunchKernelGGL(k_stretch, dim3((n + 255) / 256), dim3(256), 0, s, n, grad, om, rate);
    return hipGetLastError();
}

hipError_t launch_velocity_gradient(const DevMesh &m, const int *node_orig, const double *vel, double *tg,
                                    double *grad, hipStream_t s)
{
    if (m.T > 0) hipLaunchKernelGGL(k_tet_grad, dim3((m.T + 255) / 256), dim3(256), 0, s, m, node_orig, vel, tg);
    if (m.n > 0) hipLaunchKernelGGL(k_node_grad, dim3((m.n + 255) / 256), dim3(256), 0, s, m, node_orig, tg, grad);
    return hipGetLastError();
}

} // namespace bsk
