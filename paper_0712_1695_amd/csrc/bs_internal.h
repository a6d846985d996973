// bs_internal.h -- device data layout and kernel launch interface of the
// Biot-Savart node-velocity library (shared by bs_host.cpp and
// bs_kernels.hip; not part of the public ABI).
//
// Layout in HBM (all arrays owned by one bs_mesh):
//   nodes, sorted along a Morton curve (spatially coherent waves):
//     xh[3][npad], xl[3][npad]  binary32 hi/lo split of the FP64 coordinates
//                               (x = xh + xl to ~2^-48 relative)
//     om[3][npad]               nodal vorticity, binary32
//     blk[nblk]                 per 64-node block: bounding-sphere centre, radius
//   tetrahedra, sorted by spatial bin of the centroid:
//     g1[T][8]    1-point rule: centroid p, strength W = |T| omega(p) / 4pi, pad
//     g4[T][4][8] 4-point rule: p_q, W_q = w_q |T| omega(p_q) / 4pi, pad
//     g11[T][11][8] 11-point rule, same record
//     tid[T]      the four vertex indices (sorted-node numbering), input order
//     nbr[T]      the tet across each face (sorted numbering), -1 on the boundary
//     inc_start[n+1], inc_list: the tets incident to every node
//     cell_start[ncell + 1] first tet of every bin (bins in x-fastest order)
//   angular tables (per policy): one entry per ray of the full sphere,
//     index l = n * 2M + j (polar row n, azimuth column j in [0, 2M)):
//     dir[l] = (d.xyz, kappa) binary32, dir64[l][3] FP64 directions,
//     cphi[N] cos(polar angle) per row, dia[2M] pseudo-angle per column.
//   outputs: part[S][3][npad] FP64 far-field partials per tet split,
//            band[3][npad], rtv[3][npad] FP64 near partials, vel[n][3].
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bsk {

constexpr int kRecG = 8;        // floats per Gauss point record
constexpr int kBlockNodes = 64; // nodes per band-kernel block (one wave)

struct Bins {
    float lo[3];   // lower corner of the bin grid
    float cs;      // bin edge length
    int dim[3];    // bins per axis
    int pad;
};

struct Thresholds {
    float rt2, g11_2, g4_2; // squared cut distances, binary32
    float r_band;           // scan radius of the band kernel (>= d_g4 hbar, max vertex-centroid distance)
    float r_rt;             // scan radius of the ray-tracing kernel
    float vc;               // largest vertex-centroid distance of any tet (with margin)
    int inc_far;            // 1 if a tet having the node as a vertex can lie beyond the G4 cut
    int inc_band;           // 1 if it can lie beyond the ray-tracing cut (by the rule's binary32 d^2)
    // bounds on d^-3 from the matrix-core distance: below s_g1 the pair is
    // surely beyond the G4 cut by the rule's binary32 test, above s_amb surely
    // within it; between them (or NaN) the rule's test decides
    float s_g1, s_amb;
};

struct AngTab {
    const float4 *dir;    // [N * 2M] direction + kappa
    const double *dir64;  // [N * 2M][3]
    const float *cphi;    // [N] cos(phi_n), descending
    const float *dia;     // [2M] pseudo-angle of theta'_j, ascending in [0, 4)
    int N, M2;            // rows, columns (2M)
};

struct PackedNet; // the selector's weights in MFMA operand order (bs_mlp_dev.h)
// bytes of a PackedNet: w1, w2, w3 (BF16 operand vectors), b1, b2, b3, mu, isg (FP32)
constexpr int kPackedNetBytes = 2 * (2 * 64 * 8 + 2 * 4 * 64 * 8 + 4 * 64 * 8) + 4 * (64 + 64 + 4 + 16 + 16);

// Learned rule selector: packed network (device), confidence threshold,
// mean edge length (feature scale).  net == nullptr: fixed rule.
struct LearnParams {
    const PackedNet *net;
    float conf_min;
    float hbar;
};

// A view of the mesh for one evaluation.  The targets are the nodes
// [64 blk0, nv) of the node arrays in blocks blk0 .. blk0+nblk-1, n of them:
// the mesh's own nodes (blk0 = 0, nv = n), or points placed after them
// (bs_eval_points; no tet has them as a vertex).
struct DevMesh {
    int n, npad, T, nblk;
    int blk0, nv;
    const float *xh, *xl, *om;
    const float4 *nrec;    // [npad][2] node records (xh.x, xh.y, xh.z, xl.x), (xl.y, xl.z, om.x, om.y)
    const float4 *blk;
    const float *g1, *g4, *g11;
    const int4 *tid;
    const int *cell_start;
    const int4 *nbr;       // [T] face neighbours (sorted numbering; face f opposite vertex f; -1 boundary)
    const float4 *tsph;    // [ceil(T/16)] bounding sphere of the centroids of each tile of 16 sorted tets
    const int *inc_start;  // [n+1] CSR of the tets incident to each node
    const int *inc_list;
    Bins bins;
};

// Counters accumulated by the kernels (device, 64-bit):
// [0] G4 pairs, [1] G11 pairs, [2] RT pairs, [3] RT hit lines, [4] FP64 retests,
// [5..7] pairs the learned selector moved from RT to G1 / G4 / G11.
// Kept in kCntStripes copies, one 128-byte cache line each, a node or block
// adding to copy (its index mod kCntStripes): atomics of every node on one
// line serialise in the L2 and bound the per-node kernels.  The host sums
// the copies.
constexpr int kNumCounters = 8;
constexpr int kCntStripes = 64;
constexpr int kCntStride = 16; // 64-bit counters per copy (128 bytes)
constexpr int kCntWords = kCntStripes * kCntStride;

// Launchers (return hipSuccess or the launch error).
hipError_t launch_gauss_all(const DevMesh &m, int rule_pts, int precision, int splits, double *part,
                            hipStream_t s);
// Far field of the fixed-rule policies (G1 pairs only), precision 0 or 1.
hipError_t launch_far_mfma(const DevMesh &m, const Thresholds &th, int precision, int splits, double *part,
                           hipStream_t s);
// sub_g1: also remove the G1 term of non-G1 pairs (after launch_gauss_all).
hipError_t launch_band(const DevMesh &m, const Thresholds &th, int precision, int sub_g1, double *band,
                       unsigned long long *cnt, hipStream_t s);
hipError_t launch_rt(const DevMesh &m, const Thresholds &th, const AngTab &ang, const LearnParams &lp,
                     int all_pairs, int precision, double *rtv, unsigned long long *cnt, const int *node_list,
                     const int *node_count, hipStream_t s);
// The learned policy's selection pass for the walk: Gauss terms of the pairs
// the selector moves (written to rtv) and the pairs still ray traced
// (sel_list[n][kSelListCap], sel_n[n] = count or -1: left to launch_rt).
constexpr int kSelListCap = 128;
hipError_t launch_select(const DevMesh &m, const Thresholds &th, const LearnParams &lp, int precision, double *rtv,
                         int *sel_list, int *sel_n, float *sel_dmax, int *sel_cnt, hipStream_t s);
// Walk variant (face-manifold meshes); nodes it cannot hold are appended to
// fallback[*n_fallback] for launch_rt in node-list mode: with exit_fb (a
// boundary that is not convex) also every node with a ray that leaves the
// mesh before its stop distance.  With sel_n the ray-traced tets come from
// launch_select, the walk adds to rtv and, for the nodes it completes, adds
// sel_cnt[3 node + k] (pairs moved to G1, G4, G11) to the counters.
hipError_t launch_rt_walk(const DevMesh &m, const Thresholds &th, const AngTab &ang, int all_pairs, float r_stop,
                          int exit_fb, int precision, double *rtv, unsigned long long *cnt, int *fallback,
                          int *n_fallback, const int *sel_list, const int *sel_n, const float *sel_dmax,
                          const int *sel_cnt, hipStream_t s);
// Nodal velocity gradient (grad[input node][3][3], FP64) of the linear
// interpolant of vel ([input node][3]) on each tet, volume-weighted over the
// node's tets; tg: scratch of 10 doubles per tet.
hipError_t launch_velocity_gradient(const DevMesh &m, const int *node_orig, const double *vel, double *tg,
                                    double *grad, hipStream_t s);
// Vortex stretching rate rate[i] = grad[i] om[i] (input order, FP64).
hipError_t launch_stretching(int n, const double *grad, const double *om, double *rate, hipStream_t s);
hipError_t launch_combine(const DevMesh &m, const int *node_orig, const double *part, int splits,
                          const double *band, const double *rtv, double *vel, int *nonfinite, hipStream_t s);

// Treecode far field (BS_FAR_TREECODE): the plan the host builds and the
// per-evaluation moment buffers.  Clusters are numbered breadth first, so
// every tree level is a contiguous range of ids; tets are in tree order
// (each cluster a contiguous range).  Lists are indexed by global block id
// (node blocks, then the evaluation points' blocks from blk0 of their view).
struct TreeView {
    int order;            // expansion order P (2, 4 or 6)
    int nnode, nleaf;
    const int2 *nrange;   // [nnode] tet range [x, y) in tree order
    const int2 *child;    // [nnode] children, (-1, -1) for a leaf
    const int *leaves;    // [nleaf] leaf ids
    const double *c64;    // [nnode][4] centre (FP64)
    const float *crec;    // [nnode][8] centre split hi.xyz, lo.xyz (binary32), 0, 0
    const double *src64;  // [T][8] centroid xyz, W xyz (FP64), 0, 0, tree order
    const float *g1t;     // [T][8] binary32 centroid, W, 0, 0, tree order
    const int4 *tidt;     // [T] vertex slots, tree order
    double *M;            // [nnode][ncoef(P)][3] moments about the centre (FP64)
    float *N;             // [nnode][ncoef(P+1) - 1][3] curl moments (binary32)
    const int *acc_start, *acc; // per block: accepted clusters (CSR)
    const int *dir_start, *dir; // per block: leaves summed pair by pair (CSR)
};
// Multi-indices of degree <= d.
constexpr int tree_ncoef(int d) { return (d + 1) * (d + 2) * (d + 3) / 6; }
// The sources in tree order (order[k]: input tet at position k; tets: input
// connectivity; x64, w64: FP64 node positions and vorticity, input order;
// rank: node slot of every input node) into src64, g1t and tidt.
hipError_t launch_tree_sources(int T, const int *order, const int4 *tets, const double *x64, const double *w64,
                               const int *rank, double *src64, float *g1t, int4 *tidt, hipStream_t s);
// Moments of every cluster for the current sources: P2M at the leaves, then
// M2M level by level (levels [level_start[L], level_start[L+1]), nlevel of
// them), then the curl moments.
hipError_t launch_tree_moments(const TreeView &t, const int *level_start, int nlevel, hipStream_t s);
// Expansions into part[0 .. chunks) and direct leaves into part[chunks ..
// 2 chunks) ([2 chunks][3][npad]) for the view's blocks, each block's lists
// cut into `chunks` parts (1 .. kTreeMaxChunks).  g4_2: the rule's binary32
// squared 4-point cut; inc: test incidence in direct leaves (a tet vertex
// can lie beyond the cut).
constexpr int kTreeMaxChunks = 8;
hipError_t launch_tree_far(const DevMesh &m, const TreeView &t, float g4_2, int inc, int precision, int chunks,
                           double *part, hipStream_t s);

// Zero `words` 32-bit words at p (a kernel, so that the clearing can sit in
// a captured graph where memset nodes are avoided).
hipError_t launch_fill_zero(void *p, size_t words, hipStream_t s);

// The library's static device scratch: kScratchBytes per device, held by
// every device the library runs on until the process ends.  scratch_setup
// looks up its device address once per device (call it with that device
// current); scratch_ptr returns that address, or nullptr when the lookup
// failed or was not made.
constexpr size_t kScratchBytes = (size_t)64 << 20;
hipError_t scratch_setup(int device);
void *scratch_ptr(int device);

} // namespace bsk
