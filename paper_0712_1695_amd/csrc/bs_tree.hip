// bs_tree.hip -- the treecode far field: the fast-multipole-like evaluation
// of the 1-point-rule pairs that the paper leaves to future work (Section 4),
// as a batched Barnes-Hut treecode with Cartesian multipole expansions.
//
// The host builds the plan (bs_host.cpp): the k-d tree of the tet centroids,
// cluster and block spheres, and per 64-node block the list of clusters it
// accepts and the leaves it sums pair by pair; k_tree_sources lays the
// sources out in tree order for it.  Per evaluation, here:
//   k_tree_p2m   moments of every leaf about its centre, FP64:
//                M_k = sum_t W_t (c_t - c)^k, |k| <= P;
//   k_tree_m2m   the same for every internal cluster, level by level from
//                the deepest, from its children by the binomial shift
//                (c_t - c_p)^k = sum_{a <= k} C(k, a) (c_t - c_ch)^a (c_ch - c_p)^(k-a);
//   k_tree_curl  the curl moments N_m = sum_c (-1)^(|m|-1) m_c e_c x M_{m-e_c},
//                1 <= |m| <= P+1, binary32, so that the expansion's velocity
//                is v(x) = sum_m a_m(x - c) N_m with a_m = d^m (1/|r|) / m!;
//   k_tree_m2p   one wave per (target block, chunk of its list), lane =
//                node: the accepted clusters' expansions, a_m by the
//                Lindsay-Krasny recurrence
//                n |r|^2 a_m + (2n-1) sum_c r_c a_{m-e_c} + (n-1) sum_c a_{m-2e_c} = 0
//                in registers, N_m as scalar operands, one TwoSum fold per
//                cluster;
//   k_tree_direct one wave per (target block, chunk of its list), lane =
//                node: the pairs of the block's direct leaves that the fixed
//                rule gives the 1-point rule (its binary32 test), one TwoSum
//                fold per leaf.
// Every chunk writes a partial buffer of its own; the combine kernel adds
// them in FP64 in a fixed order.  Waves take blocks in contiguous k-d ranges
// per XCD (workgroup ids are dealt to the eight XCDs in turn), so each XCD's
// L2 holds one region's clusters.
#include "bs_internal.h"

#include <utility>

namespace bsk {
namespace {

// ---- multi-indices (i, j, l): graded by n = i + j + l, then i and j
// descending; index of (i, j, l) in that order
constexpr int tc_index(int i, int j, int l)
{
    const int n = i + j + l;
    return n * (n + 1) * (n + 2) / 6 + (n - i) * (n - i + 1) / 2 + (n - i - j);
}

template <int D>
struct TcTable {
    int e[tree_ncoef(D)][3];   // exponents
    int dn[tree_ncoef(D)][3];  // index of m - e_c, or -1
    int dn2[tree_ncoef(D)][3]; // index of m - 2 e_c, or -1
    constexpr TcTable() : e{}, dn{}, dn2{}
    {
        int q = 0;
        for (int n = 0; n <= D; ++n)
            for (int i = n; i >= 0; --i)
                for (int j = n - i; j >= 0; --j) {
                    const int x[3] = {i, j, n - i - j};
                    for (int c = 0; c < 3; ++c) {
                        e[q][c] = x[c];
                        int y[3] = {x[0], x[1], x[2]};
                        y[c] -= 1;
                        dn[q][c] = x[c] >= 1 ? tc_index(y[0], y[1], y[2]) : -1;
                        y[c] -= 1;
                        dn2[q][c] = x[c] >= 2 ? tc_index(y[0], y[1], y[2]) : -1;
                    }
                    ++q;
                }
    }
};

template <int D>
struct TcTab {
    static constexpr TcTable<D> t{};
};

// exponents of graded index k (run-time)
__device__ __forceinline__ void tc_decode(int k, int &i, int &j, int &l)
{
    int n = 0;
    while ((n + 1) * (n + 2) * (n + 3) / 6 <= k) ++n;
    int rem = k - n * (n + 1) * (n + 2) / 6;
    i = n;
    while (rem >= n - i + 1) {
        rem -= n - i + 1;
        --i;
    }
    j = n - i - rem;
    l = n - i - j;
}

__device__ __forceinline__ double ipow(double x, int e)
{
    double r = 1.0;
    for (int k = 0; k < e; ++k) r *= x;
    return r;
}

// Fold a into the compensated pair (s, c) (Knuth's TwoSum).
__device__ __forceinline__ void tc_two_sum(float &s, float &c, float a)
{
    const float t = s + a;
    const float bp = t - s;
    const float err = (s - (t - bp)) + (a - bp);
    s = t;
    c += err;
}

// One Taylor coefficient a_Q from lower ones: al[n] = -(2n-1) / (n |r|^2),
// be[n] = -(n-1) / (n |r|^2).
template <int D, int Q>
__device__ __forceinline__ void taylor_one(float *a, float rx, float ry, float rz, const float *al, const float *be)
{
    if constexpr (Q > 0) {
        constexpr auto &t = TcTab<D>::t;
        constexpr int n = t.e[Q][0] + t.e[Q][1] + t.e[Q][2];
        constexpr int d0 = t.dn[Q][0], d1 = t.dn[Q][1], d2 = t.dn[Q][2];
        constexpr int f0 = t.dn2[Q][0], f1 = t.dn2[Q][1], f2 = t.dn2[Q][2];
        float s1 = 0.f;
        if constexpr (d0 >= 0) s1 = rx * a[d0];
        if constexpr (d1 >= 0) s1 = d0 >= 0 ? fmaf(ry, a[d1], s1) : ry * a[d1];
        if constexpr (d2 >= 0) s1 = (d0 >= 0 || d1 >= 0) ? fmaf(rz, a[d2], s1) : rz * a[d2];
        float v = al[n] * s1;
        if constexpr (f0 >= 0 || f1 >= 0 || f2 >= 0) {
            float s2 = 0.f;
            if constexpr (f0 >= 0) s2 = a[f0];
            if constexpr (f1 >= 0) s2 = f0 >= 0 ? s2 + a[f1] : a[f1];
            if constexpr (f2 >= 0) s2 = (f0 >= 0 || f1 >= 0) ? s2 + a[f2] : a[f2];
            v = fmaf(be[n], s2, v);
        }
        a[Q] = v;
    }
}

template <int D, int... Q>
__device__ __forceinline__ void taylor_all(float *a, float rx, float ry, float rz, const float *al, const float *be,
                                           std::integer_sequence<int, Q...>)
{
    (taylor_one<D, Q>(a, rx, ry, rz, al, be), ...);
}

template <int Q>
__device__ __forceinline__ void curl_one(const float *a, const float *__restrict__ N, float &vx, float &vy, float &vz)
{
    if constexpr (Q > 0) {
        vx = fmaf(a[Q], N[3 * (Q - 1)], vx);
        vy = fmaf(a[Q], N[3 * (Q - 1) + 1], vy);
        vz = fmaf(a[Q], N[3 * (Q - 1) + 2], vz);
    }
}

template <int... Q>
__device__ __forceinline__ void curl_all(const float *a, const float *__restrict__ N, float &vx, float &vy, float &vz,
                                         std::integer_sequence<int, Q...>)
{
    (curl_one<Q>(a, N, vx, vy, vz), ...);
}

// Velocity of one cluster's expansion at offset r = x - c (binary32).
template <int P>
__device__ __forceinline__ void expansion(float rx, float ry, float rz, const float *__restrict__ N, float &vx, float &vy,
                                          float &vz)
{
    constexpr int D = P + 1;
    constexpr int NK = tree_ncoef(D);
    const float r2 = fmaf(rx, rx, fmaf(ry, ry, rz * rz));
    const float inv = __builtin_amdgcn_rcpf(r2);
    float al[D + 1], be[D + 1];
#pragma unroll
    for (int n = 1; n <= D; ++n) {
        al[n] = (float)(-(2 * n - 1)) / (float)n * inv;
        be[n] = (float)(-(n - 1)) / (float)n * inv;
    }
    float a[NK];
    a[0] = __builtin_amdgcn_rsqf(r2);
    taylor_all<D>(a, rx, ry, rz, al, be, std::make_integer_sequence<int, NK>{});
    vx = vy = vz = 0.f;
    curl_all(a, N, vx, vy, vz, std::make_integer_sequence<int, NK>{});
}

// ---- moments (FP64)

template <int P>
__global__ void __launch_bounds__(256) k_tree_p2m(TreeView t)
{
    constexpr int NK = tree_ncoef(P);
    const int gid = blockIdx.x * 256 + threadIdx.x;
    if (gid >= t.nleaf * NK) return;
    const int q = gid / NK, k = gid - q * NK;
    const int j = t.leaves[q];
    const int2 r = t.nrange[j];
    int ei, ej, el;
    tc_decode(k, ei, ej, el);
    const double cx = t.c64[4 * j], cy = t.c64[4 * j + 1], cz = t.c64[4 * j + 2];
    double mx = 0.0, my = 0.0, mz = 0.0;
    for (int u = r.x; u < r.y; ++u) {
        const double *s = t.src64 + 8 * (size_t)u;
        const double f = ipow(s[0] - cx, ei) * ipow(s[1] - cy, ej) * ipow(s[2] - cz, el);
        mx += f * s[3];
        my += f * s[4];
        mz += f * s[5];
    }
    double *o = t.M + ((size_t)j * NK + k) * 3;
    o[0] = mx;
    o[1] = my;
    o[2] = mz;
}

__device__ __forceinline__ double binom(int n, int k)
{
    double r = 1.0;
    for (int q = 1; q <= k; ++q) r = r * (double)(n - k + q) / (double)q;
    return r;
}

template <int P>
__global__ void __launch_bounds__(256) k_tree_m2m(TreeView t, int node0, int node1)
{
    constexpr int NK = tree_ncoef(P);
    const int gid = blockIdx.x * 256 + threadIdx.x;
    const int j = node0 + gid / NK, k = gid % NK;
    if (j >= node1) return;
    const int2 ch = t.child[j];
    if (ch.x < 0) return; // a leaf: its moments come from k_tree_p2m
    int ei, ej, el;
    tc_decode(k, ei, ej, el);
    double mx = 0.0, my = 0.0, mz = 0.0;
    const int kids[2] = {ch.x, ch.y};
    for (int h = 0; h < 2; ++h) {
        const int c = kids[h];
        const double dx = t.c64[4 * c] - t.c64[4 * j], dy = t.c64[4 * c + 1] - t.c64[4 * j + 1],
                     dz = t.c64[4 * c + 2] - t.c64[4 * j + 2];
        const double *Mc = t.M + (size_t)c * NK * 3;
        for (int a = 0; a <= ei; ++a)
            for (int b = 0; b <= ej; ++b)
                for (int e = 0; e <= el; ++e) {
                    const double f = binom(ei, a) * binom(ej, b) * binom(el, e) * ipow(dx, ei - a) *
                                     ipow(dy, ej - b) * ipow(dz, el - e);
                    const double *m = Mc + 3 * tc_index(a, b, e);
                    mx += f * m[0];
                    my += f * m[1];
                    mz += f * m[2];
                }
    }
    double *o = t.M + ((size_t)j * NK + k) * 3;
    o[0] = mx;
    o[1] = my;
    o[2] = mz;
}

template <int P>
__global__ void __launch_bounds__(256) k_tree_curl(TreeView t)
{
    constexpr int NK = tree_ncoef(P);
    constexpr int NC = tree_ncoef(P + 1) - 1;
    const int gid = blockIdx.x * 256 + threadIdx.x;
    if (gid >= t.nnode * NC) return;
    const int j = gid / NC, q = 1 + gid % NC;
    int ei, ej, el;
    tc_decode(q, ei, ej, el);
    const double *M = t.M + (size_t)j * NK * 3;
    double nx = 0.0, ny = 0.0, nz = 0.0;
    if (ei >= 1) { // i e_x x M = i (0, -Mz, My)
        const double *m = M + 3 * tc_index(ei - 1, ej, el);
        ny -= ei * m[2];
        nz += ei * m[1];
    }
    if (ej >= 1) { // j e_y x M = j (Mz, 0, -Mx)
        const double *m = M + 3 * tc_index(ei, ej - 1, el);
        nx += ej * m[2];
        nz -= ej * m[0];
    }
    if (el >= 1) { // l e_z x M = l (-My, Mx, 0)
        const double *m = M + 3 * tc_index(ei, ej, el - 1);
        nx -= el * m[1];
        ny += el * m[0];
    }
    const double sg = ((ei + ej + el - 1) & 1) ? -1.0 : 1.0;
    float *o = t.N + ((size_t)j * NC + (q - 1)) * 3;
    o[0] = (float)(sg * nx);
    o[1] = (float)(sg * ny);
    o[2] = (float)(sg * nz);
}

// ---- evaluation

// Work item of this wave: (target block, chunk of its list).  Workgroup ids
// are dealt to the eight XCDs in turn, and XCD x takes logical workgroups
// [x per_xcd, (x+1) per_xcd), so each XCD walks one contiguous range of k-d
// blocks; the chunks of a block are neighbours.  Each block's list is cut
// into `chunks` parts (many short waves rather than one per block, so that
// the last waves do not run alone).  Returns the block, or -1 past the end.
__device__ __forceinline__ int tree_item(int per_xcd, int nblk, int chunks, int &chunk)
{
    const int g = blockIdx.x;
    const int lg = (g & 7) * per_xcd + (g >> 3);
    // the wave's index, made uniform for the compiler: every list index and
    // record address below is then wave-uniform (scalar loads, scalar loop
    // control) rather than per lane
    const int w = 4 * lg + __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
    const int b = w / chunks;
    chunk = w - b * chunks;
    return b < nblk ? b : -1;
}

// Entries [q0, q1) of list [a, b) for chunk c of `chunks`.
__device__ __forceinline__ void chunk_range(int a, int b, int c, int chunks, int &q0, int &q1)
{
    const int len = b - a;
    q0 = a + (int)(((long long)len * c) / chunks);
    q1 = a + (int)(((long long)len * (c + 1)) / chunks);
}

template <int P, int PREC>
__global__ void __launch_bounds__(256) k_tree_m2p(DevMesh m, TreeView t, int per_xcd, int chunks,
                                                   double *__restrict__ part)
{
    int chunk;
    const int b = tree_item(per_xcd, m.nblk, chunks, chunk);
    if (b < 0) return;
    constexpr int NC = tree_ncoef(P + 1) - 1;
    const int gb = m.blk0 + b;
    const int p = 64 * gb + (threadIdx.x & 63);
    const int np = m.npad;
    const float xh = m.xh[p], yh = m.xh[np + p], zh = m.xh[2 * np + p];
    const float xl = m.xl[p], yl = m.xl[np + p], zl = m.xl[2 * np + p];
    float sx = 0.f, sy = 0.f, sz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
    double dx = 0.0, dy = 0.0, dz = 0.0;
    int a0, a1;
    chunk_range(t.acc_start[gb], t.acc_start[gb + 1], chunk, chunks, a0, a1);
    for (int q = a0; q < a1; ++q) {
        const int j = t.acc[q];
        const float *cr = t.crec + 8 * (size_t)j;
        const float rx = (xh - cr[0]) + (xl - cr[3]);
        const float ry = (yh - cr[1]) + (yl - cr[4]);
        const float rz = (zh - cr[2]) + (zl - cr[5]);
        float vx, vy, vz;
        expansion<P>(rx, ry, rz, t.N + (size_t)j * NC * 3, vx, vy, vz);
        if (PREC == 0) {
            sx += vx;
            sy += vy;
            sz += vz;
        } else if (PREC == 1) {
            tc_two_sum(sx, cx, vx);
            tc_two_sum(sy, cy, vy);
            tc_two_sum(sz, cz, vz);
        } else {
            dx += (double)vx;
            dy += (double)vy;
            dz += (double)vz;
        }
    }
    if (PREC != 2) {
        dx = (double)sx + (double)cx;
        dy = (double)sy + (double)cy;
        dz = (double)sz + (double)cz;
    }
    double *o = part + (size_t)chunk * 3 * np;
    o[p] = dx;
    o[np + p] = dy;
    o[2 * np + p] = dz;
}

template <int PREC, int INC>
__global__ void __launch_bounds__(256) k_tree_direct(DevMesh m, TreeView t, float g4_2, int per_xcd, int chunks,
                                                      double *__restrict__ part)
{
    int chunk;
    const int b = tree_item(per_xcd, m.nblk, chunks, chunk);
    if (b < 0) return;
    const int gb = m.blk0 + b;
    const int p = 64 * gb + (threadIdx.x & 63);
    const int np = m.npad;
    const float x = m.xh[p], y = m.xh[np + p], z = m.xh[2 * np + p];
    float sx = 0.f, sy = 0.f, sz = 0.f, cx = 0.f, cy = 0.f, cz = 0.f;
    double dx = 0.0, dy = 0.0, dz = 0.0;
    int l0, l1;
    chunk_range(t.dir_start[gb], t.dir_start[gb + 1], chunk, chunks, l0, l1);
    for (int q = l0; q < l1; ++q) {
        const int2 r = t.nrange[t.dir[q]];
        float ax = 0.f, ay = 0.f, az = 0.f;
#pragma unroll 2
        for (int u = r.x; u < r.y; ++u) {
            const float *g = t.g1t + 8 * (size_t)u;
            // the rule's binary32 distance (each operation rounded, no FMA)
            const float ex = x - g[0], ey = y - g[1], ez = z - g[2];
            const float qx = ex * ex, qy = ey * ey, qz = ez * ez;
            const float d2 = (qx + qy) + qz;
            bool on = !(d2 < g4_2);
            if (INC) {
                const int4 id = t.tidt[u];
                on = on && id.x != p && id.y != p && id.z != p && id.w != p;
            }
            const float iv = __builtin_amdgcn_rsqf(d2);
            const float s = on ? iv * iv * iv : 0.f;
            const float ux = ex * s, uy = ey * s, uz = ez * s;
            if (PREC == 2) {
                dx += (double)fmaf(g[4], uz, -g[5] * uy);
                dy += (double)fmaf(g[5], ux, -g[3] * uz);
                dz += (double)fmaf(g[3], uy, -g[4] * ux);
            } else {
                ax = fmaf(g[4], uz, fmaf(-g[5], uy, ax));
                ay = fmaf(g[5], ux, fmaf(-g[3], uz, ay));
                az = fmaf(g[3], uy, fmaf(-g[4], ux, az));
            }
        }
        if (PREC == 0) {
            sx += ax;
            sy += ay;
            sz += az;
        } else if (PREC == 1) {
            tc_two_sum(sx, cx, ax);
            tc_two_sum(sy, cy, ay);
            tc_two_sum(sz, cz, az);
        }
    }
    if (PREC != 2) {
        dx = (double)sx + (double)cx;
        dy = (double)sy + (double)cy;
        dz = (double)sz + (double)cz;
    }
    double *o = part + (size_t)chunk * 3 * np;
    o[p] = dx;
    o[np + p] = dy;
    o[2 * np + p] = dz;
}

// Per-tet sources in tree order (position k, input tet order[k]): FP64
// centroid (((v0+v1)+v2)+v3)/4 and strength |T|/(4 pi) (((w0+w1)+w2)+w3)/4,
// their binary32 roundings, and the vertex slots; every operation as the
// host's, in FP64 without contraction.
__global__ void __launch_bounds__(256) k_tree_sources(int T, const int *__restrict__ order,
                                                      const int4 *__restrict__ tets, const double *__restrict__ x64,
                                                      const double *__restrict__ w64, const int *__restrict__ rank,
                                                      double *__restrict__ src64, float *__restrict__ g1t,
                                                      int4 *__restrict__ tidt)
{
    const int k = blockIdx.x * 256 + threadIdx.x;
    if (k >= T) return;
    const int4 t4 = tets[order[k]];
    const int id[4] = {t4.x, t4.y, t4.z, t4.w};
    double v[4][3];
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) v[j][c] = x64[3 * (size_t)id[j] + c];
    double e[3][3];
#pragma unroll
    for (int j = 0; j < 3; ++j)
#pragma unroll
        for (int c = 0; c < 3; ++c) e[j][c] = v[j + 1][c] - v[0][c];
    const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                       e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                       e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
    const double f = fabs(det) / 6.0 / (4.0 * M_PI);
    double *o = src64 + 8 * (size_t)k;
    float *g = g1t + 8 * (size_t)k;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        const double cen = (((v[0][c] + v[1][c]) + v[2][c]) + v[3][c]) * 0.25;
        const double w = (((w64[3 * (size_t)id[0] + c] + w64[3 * (size_t)id[1] + c]) + w64[3 * (size_t)id[2] + c]) +
                          w64[3 * (size_t)id[3] + c]) * 0.25;
        o[c] = cen;
        o[3 + c] = f * w;
        g[c] = (float)cen;
        g[3 + c] = (float)(f * w);
    }
    o[6] = o[7] = 0.0;
    g[6] = g[7] = 0.f;
    tidt[k] = make_int4(rank[id[0]], rank[id[1]], rank[id[2]], rank[id[3]]);
}

template <int P>
hipError_t moments_p(const TreeView &t, const int *level_start, int nlevel, hipStream_t s)
{
    constexpr int NK = tree_ncoef(P);
    constexpr int NC = tree_ncoef(P + 1) - 1;
    if (t.nleaf > 0) {
        const int64_t n = (int64_t)t.nleaf * NK;
        hipLaunchKernelGGL((k_tree_p2m<P>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t);
    }
    for (int L = nlevel - 1; L >= 0; --L) {
        const int a = level_start[L], b = level_start[L + 1];
        if (b <= a) continue;
        const int64_t n = (int64_t)(b - a) * NK;
        hipLaunchKernelGGL((k_tree_m2m<P>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t, a, b);
    }
    if (t.nnode > 0) {
        const int64_t n = (int64_t)t.nnode * NC;
        hipLaunchKernelGGL((k_tree_curl<P>), dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, t);
    }
    return hipGetLastError();
}

template <int P, int PREC>
void launch_m2p(const DevMesh &m, const TreeView &t, int per_xcd, int chunks, double *part, hipStream_t s)
{
    hipLaunchKernelGGL((k_tree_m2p<P, PREC>), dim3(8 * per_xcd), dim3(256), 0, s, m, t, per_xcd, chunks, part);
}

template <int PREC>
void launch_m2p_prec(const DevMesh &m, const TreeView &t, int per_xcd, int chunks, double *part, hipStream_t s)
{
    if (t.order == 2) launch_m2p<2, PREC>(m, t, per_xcd, chunks, part, s);
    else if (t.order == 4) launch_m2p<4, PREC>(m, t, per_xcd, chunks, part, s);
    else launch_m2p<6, PREC>(m, t, per_xcd, chunks, part, s);
}

template <int PREC>
void launch_direct(const DevMesh &m, const TreeView &t, float g4_2, int inc, int per_xcd, int chunks, double *part,
                   hipStream_t s)
{
    if (inc)
        hipLaunchKernelGGL((k_tree_direct<PREC, 1>), dim3(8 * per_xcd), dim3(256), 0, s, m, t, g4_2, per_xcd, chunks,
                           part);
    else
        hipLaunchKernelGGL((k_tree_direct<PREC, 0>), dim3(8 * per_xcd), dim3(256), 0, s, m, t, g4_2, per_xcd, chunks,
                           part);
}

} // namespace

hipError_t launch_tree_sources(int T, const int *order, const int4 *tets, const double *x64, const double *w64,
                               const int *rank, double *src64, float *g1t, int4 *tidt, hipStream_t s)
{
    if (T <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_tree_sources, dim3((unsigned)((T + 255) / 256)), dim3(256), 0, s, T, order, tets, x64, w64, rank,
                       src64, g1t, tidt);
    return hipGetLastError();
}

hipError_t launch_tree_moments(const TreeView &t, const int *level_start, int nlevel, hipStream_t s)
{
    if (t.order == 2) return moments_p<2>(t, level_start, nlevel, s);
    if (t.order == 4) return moments_p<4>(t, level_start, nlevel, s);
    if (t.order == 6) return moments_p<6>(t, level_start, nlevel, s);
    return hipErrorInvalidValue;
}

hipError_t launch_tree_far(const DevMesh &m, const TreeView &t, float g4_2, int inc, int precision, int chunks,
                           double *part, hipStream_t s)
{
    if (t.order != 2 && t.order != 4 && t.order != 6) return hipErrorInvalidValue;
    if (chunks < 1 || chunks > kTreeMaxChunks) return hipErrorInvalidValue;
    if (m.nblk <= 0) return hipSuccess;
    const int wg = (m.nblk * chunks + 3) / 4;
    const int per_xcd = (wg + 7) / 8;
    double *p0 = part, *p1 = part + 3 * (size_t)m.npad * chunks;
    if (precision == 0) {
        launch_m2p_prec<0>(m, t, per_xcd, chunks, p0, s);
        launch_direct<0>(m, t, g4_2, inc, per_xcd, chunks, p1, s);
    } else if (precision == 1) {
        launch_m2p_prec<1>(m, t, per_xcd, chunks, p0, s);
        launch_direct<1>(m, t, g4_2, inc, per_xcd, chunks, p1, s);
    } else {
        launch_m2p_prec<2>(m, t, per_xcd, chunks, p0, s);
        launch_direct<2>(m, t, g4_2, inc, per_xcd, chunks, p1, s);
    }
    return hipGetLastError();
}

} // namespace bsk
