// bs_host.cpp -- host side of the Biot-Savart node-velocity library: input
// validation, the O(n_tets) per-element precompute in FP64, spatial ordering,
// angular tables and the launch sequence of one velocity evaluation.
//
// Per-element precompute (Section 2: vorticity linear within each element;
// Introduction: Gauss rules for distant elements):
//   |T| = |det(v1-v0, v2-v0, v3-v0)| / 6, centroid (((v0+v1)+v2)+v3)/4 in
//   input vertex order, rule points p_q = sum_j lambda_qj v_j and strengths
//   W_q = w_q |T| omega(p_q) / 4pi for the 1-, 4- and 11-point rules.
// Angular tables (Section 2, eq. 3 and Section 2.2 item 3): Gauss-Legendre
//   nodes t_n, weights w_n; phi_n = (1 + t_n) pi/2, theta_m = (1 + t_m) pi/2,
//   line direction s_nm, weight k_nm = (pi/16) sin(phi_n) w_n w_m (the
//   half-sphere measure of eq. 2 times 1/4pi; the printed 1/(16 pi^2) does not
//   integrate the half sphere to 1/2).  Each line gives two rays, +s and -s,
//   both with weight k_nm.
#include "bs_internal.h"
#include "bs_learn.h"

#include "../../include/bs.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <atomic>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <thread>
#include <vector>

namespace {

thread_local std::string g_err;

int fail(int code, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_err = buf;
    return code;
}

int hip_fail(hipError_t e, const char *what)
{
    if (e == hipErrorOutOfMemory) return fail(BS_E_NOMEM, "%s: %s", what, hipGetErrorString(e));
    return fail(BS_E_DEVICE, "%s: %s", what, hipGetErrorString(e));
}

// --------------------------------------------------------------- quadrature

// Gauss-Legendre on [-1, 1]: Newton on P_n for the positive half; the
// negative nodes are exact mirrors so that the line set is symmetric.
void gauss_legendre(int n, std::vector<double> &t, std::vector<double> &w)
{
    t.assign(n, 0.0);
    w.assign(n, 0.0);
    const int half = (n + 1) / 2;
    for (int i = 0; i < half; ++i) {
        double x = std::cos(M_PI * (i + 0.75) / (n + 0.5)); // i-th largest root
        double dpn = 1.0;
        for (int it = 0; it < 60; ++it) {
            double pm = 1.0, p = x;
            for (int k = 2; k <= n; ++k) {
                const double pk = ((2 * k - 1) * x * p - (k - 1) * pm) / k;
                pm = p;
                p = pk;
            }
            if (n == 1) {
                p = x;
                pm = 1.0;
            }
            dpn = n * (x * p - pm) / (x * x - 1.0);
            const double dx = p / dpn;
            x -= dx;
            if (std::fabs(dx) <= 1e-17) break;
        }
        {
            double pm = 1.0, p = x;
            for (int k = 2; k <= n; ++k) {
                const double pk = ((2 * k - 1) * x * p - (k - 1) * pm) / k;
                pm = p;
                p = pk;
            }
            if (n == 1) {
                p = x;
                pm = 1.0;
            }
            dpn = n * (x * p - pm) / (x * x - 1.0);
        }
        const double wi = 2.0 / ((1.0 - x * x) * dpn * dpn);
        if (2 * i + 1 == n) x = 0.0;
        t[n - 1 - i] = x;
        t[i] = -x;
        w[n - 1 - i] = wi;
        w[i] = wi;
    }
}

// Symmetric tetrahedral rules as barycentric points and weights (sum 1).
struct TetRule {
    int n;
    double lam[11][4];
    double w[11];
};

TetRule tet_rule(int k)
{
    TetRule r{};
    r.n = k;
    if (k == 1) {
        for (int j = 0; j < 4; ++j) r.lam[0][j] = 0.25;
        r.w[0] = 1.0;
    } else if (k == 4) {
        // degree 2: one orbit (a, b, b, b) with weight 1/4
        const double s5 = std::sqrt(5.0);
        const double a = (5.0 + 3.0 * s5) / 20.0, b = (5.0 - s5) / 20.0;
        for (int q = 0; q < 4; ++q) {
            for (int j = 0; j < 4; ++j) r.lam[q][j] = (q == j) ? a : b;
            r.w[q] = 0.25;
        }
    } else {
        // degree 4 (Keast): centroid, orbit (11/14, 1/14, 1/14, 1/14),
        // orbit (c, c, d, d) with c, d = (1 +- sqrt(5/14))/4
        int q = 0;
        for (int j = 0; j < 4; ++j) r.lam[q][j] = 0.25;
        r.w[q++] = -148.0 / 1875.0;
        for (int v = 0; v < 4; ++v, ++q) {
            for (int j = 0; j < 4; ++j) r.lam[q][j] = (v == j) ? 11.0 / 14.0 : 1.0 / 14.0;
            r.w[q] = 343.0 / 7500.0;
        }
        const double g = std::sqrt(5.0 / 14.0);
        const double c = (1.0 + g) / 4.0, d = (1.0 - g) / 4.0;
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j, ++q) {
                for (int l = 0; l < 4; ++l) r.lam[q][l] = (l == i || l == j) ? c : d;
                r.w[q] = 56.0 / 375.0;
            }
    }
    return r;
}

// --------------------------------------------------------------- helpers

template <typename F>
void parallel_for(int64_t n, F &&f)
{
    unsigned hw = std::thread::hardware_concurrency();
    int nt = (int)std::min<unsigned>(hw ? hw : 1, 16);
    if (n < 4096 || nt <= 1) {
        f(0, n);
        return;
    }
    std::vector<std::thread> th;
    const int64_t chunk = (n + nt - 1) / nt;
    for (int k = 0; k < nt; ++k) {
        const int64_t a = k * chunk, b = std::min(n, a + chunk);
        if (a >= b) break;
        th.emplace_back([&, a, b] { f(a, b); });
    }
    for (auto &t : th) t.join();
}

// f(i) for every i in [0, count), items dealt to up to 16 threads.
template <class F>
void parallel_items(int64_t count, F &&f)
{
    const unsigned hw = std::thread::hardware_concurrency();
    const int64_t nt = std::min<int64_t>(std::min<unsigned>(hw ? hw : 1u, 16u), count);
    if (nt <= 1) {
        for (int64_t i = 0; i < count; ++i) f(i);
        return;
    }
    std::atomic<int64_t> next{0};
    std::vector<std::thread> th;
    for (int64_t k = 0; k < nt; ++k)
        th.emplace_back([&] {
            for (int64_t i; (i = next.fetch_add(1)) < count;) f(i);
        });
    for (auto &t : th) t.join();
}

// Stable counting sort of the keys key(i) in [0, nkeys) of items
// i in [0, count): start[nkeys + 1] (CSR offsets) and out[start[key] ..] =
// the items of each key in increasing i, as a sequential pass would leave
// them; contiguous ranges of i are counted and placed by separate threads
// (at most 16, fewer when a per-thread count array would be large).
template <class K>
void stable_bucket(int64_t count, int64_t nkeys, K &&key, std::vector<int32_t> &start, std::vector<int32_t> &out)
{
    start.assign((size_t)nkeys + 1, 0);
    out.resize((size_t)count);
    const int64_t nc = std::max<int64_t>(1, std::min<int64_t>({16, (int64_t)((1ll << 25) / std::max<int64_t>(nkeys, 1)),
                                                                 count / 4096 + 1}));
    std::vector<std::vector<int32_t>> cnt((size_t)nc);
    auto lo = [&](int64_t c) { return count * c / nc; };
    parallel_items(nc, [&](int64_t c) {
        auto &h = cnt[(size_t)c];
        h.assign((size_t)nkeys, 0);
        for (int64_t i = lo(c); i < lo(c + 1); ++i) h[(size_t)key(i)]++;
    });
    // start of every key; then each chunk's first slot per key
    for (int64_t k = 0; k < nkeys; ++k) {
        int32_t tot = 0;
        for (int64_t c = 0; c < nc; ++c) tot += cnt[(size_t)c][(size_t)k];
        start[(size_t)k + 1] = start[(size_t)k] + tot;
    }
    for (int64_t k = 0; k < nkeys; ++k) {
        int32_t at = start[(size_t)k];
        for (int64_t c = 0; c < nc; ++c) {
            const int32_t v = cnt[(size_t)c][(size_t)k];
            cnt[(size_t)c][(size_t)k] = at;
            at += v;
        }
    }
    parallel_items(nc, [&](int64_t c) {
        auto &h = cnt[(size_t)c];
        for (int64_t i = lo(c); i < lo(c + 1); ++i) out[(size_t)h[(size_t)key(i)]++] = (int32_t)i;
    });
}

// Pinned host memory (hipHostMalloc), grown on demand and kept: the
// staging of the records uploaded at every rebuild.
struct PinnedBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

int pinned_reserve(PinnedBuf &b, size_t bytes)
{
    if (b.p && b.bytes >= bytes) return BS_OK;
    if (b.p) (void)hipHostFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    hipError_t e = hipHostMalloc(&b.p, std::max<size_t>(bytes, 256), hipHostMallocDefault);
    if (e != hipSuccess) {
        b.p = nullptr;
        return hip_fail(e, "hipHostMalloc (record staging)");
    }
    b.bytes = std::max<size_t>(bytes, 256);
    return BS_OK;
}

// Node slots (nodes, then evaluation points from the next multiple of 1024,
// padded to a multiple of 1024) are indexed in 32-bit int by the kernels as
// c * npad + i for c < 3: 3 * 2^29 stays below 2^31.  The tet count is held
// below 2^29 so that the CSR of incident tets (4 per tet) fits int32.
constexpr int64_t kMaxNodeSlots = (int64_t)1 << 29;
constexpr int64_t kMaxTets = (int64_t)1 << 29;

inline int64_t round_up_1024(int64_t v) { return ((v + 1023) / 1024) * 1024; }

struct DBuf {
    void *p = nullptr;
    size_t bytes = 0;
};

int dalloc(DBuf &b, size_t bytes)
{
    if (b.p && b.bytes >= bytes) return BS_OK;
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
    if (bytes == 0) bytes = 256;
    hipError_t e = hipMalloc(&b.p, bytes);
    if (e != hipSuccess) {
        b.p = nullptr;
        return hip_fail(e, "hipMalloc");
    }
    b.bytes = bytes;
    return BS_OK;
}

void dfree(DBuf &b)
{
    if (b.p) (void)hipFree(b.p);
    b.p = nullptr;
    b.bytes = 0;
}

} // namespace

// --------------------------------------------------------------- mesh object

struct bs_mesh {
    int device = -1;
    int64_t n = 0, T = 0;
    int npad = 0, nblk = 0;
    std::vector<int32_t> tets;     // input connectivity
    std::vector<double> xyz, omega; // current FP64 inputs
    double hbar = 0.0, max_vc = 0.0;
    double max_abs = 0.0; // largest coordinate magnitude of any node or evaluation point
    int64_t reoriented = 0;
    std::vector<int8_t> orient; // sign of det per tet at upload (inversion check on updates)
    std::vector<int32_t> h_rank, h_order, h_cell_start; // node rank, tet order, bins (host copies)
    std::vector<float> h_cen32;                         // binary32 centroids, input tet order
    std::vector<float> h_xh;                            // binary32 node coordinates, input node order
    std::vector<int32_t> nbr_in;  // [T][4] face neighbours (input tet numbering, -1 boundary)
    std::vector<int32_t> inc_in_start, inc_in_list; // corners 4t + j of every input node, by node (built once)
    std::vector<int64_t> edge_keys; // unique edges, sorted (lo * (n + 1) + hi); built on first use
    PinnedBuf h_g1, h_g4, h_g11; // pinned host staging of the Gauss records (reused between builds)
    std::vector<int4> h_tid;
    bool manifold = true;         // every face shared by at most two tets
    bool convex = false;          // boundary is one closed, locally convex surface (rays never re-enter)
    bsk::Bins bins{};
    // device buffers
    DBuf tsph; // bounding spheres of 16-tet tiles
    DBuf xh, xl, om, nrec, blk, node_orig, g1, g4, g11, tid, cell_start, nbr, inc_start, inc_list;
    DBuf part, band, rtv, vel, cnt, nonfinite, fallback;
    // evaluation points (bs_eval_points): FP64 copy, count, first node index
    // and first block in the node arrays, their order and output
    std::vector<double> tgt;
    int64_t tn = 0;
    int t0 = 0, tblk0 = 0, tnblk = 0;
    DBuf torig, tlist, tvel;
    bool last_targets = false; // the last evaluation was of the points
    int last_rt = 0;           // ray tracing of the last evaluation: 0 none, 1 candidate kernel, 2 walk
    bool vel_valid = false;    // vel holds the nodes' velocities at the current positions and vorticity
    DBuf gvel, tgrad, ngrad;   // velocity gradient: input velocities, per-tet |T| G and |T|, nodal G
    DBuf om64, srate;          // FP64 nodal vorticity (input order) and the stretching rate G omega
    // treecode far field (BS_FAR_TREECODE): the plan of the current positions
    // and policy (tree, spheres, interaction lists) and the moment buffers
    struct TreePlan {
        bool valid = false;
        double theta = 0.0, d_g4 = 0.0;
        int order = 0, nnode = 0, nleaf = 0;
        std::vector<int> level_start; // tree level L: clusters [level_start[L], level_start[L+1])
        int64_t exp_nodes = 0, dir_nodes = 0, exp_pts = 0, dir_pts = 0; // expansion terms, direct pairs
        int64_t cov_nodes = 0, cov_pts = 0; // pairs the expansions sum
        DBuf nrange, child, leaves, c64, crec, src64, g1t, tidt, M, N, acc_start, acc, dir_start, dir;
        DBuf torder, tin, x64, rank; // tree order, input connectivity, FP64 positions, node slots (device)
        bool tin_valid = false;      // the connectivity is on the device (it never changes)
    } tree;
    std::vector<int32_t> h_torig; // evaluation points in their k-d order (host copy)
    int rt_mode = 0; // 0: walk (face-manifold meshes), 1: always the candidate kernel
    int far_mode = 0; // 0: matrix-core far field (fixed-rule policies, FP32 modes), 1: vector-ALU kernel
    int serial = 0;   // 1: every kernel on the caller's stream
    DBuf dir, dir64, cphi, dia;
    int part_splits = 0;
    // policy
    bs_policy pol{};
    int ang_N = 0, ang_M = 0;
    DBuf mlp; // the learned policy's network in the fused inference's operand order
    DBuf sel; // learned policy on walk meshes: ray-traced lists, their counts and farthest centroids
    // timing: 0 start, 1 far field done (caller's stream); 2-3 band (aux[0]);
    // 4-5 ray tracing (aux[1]); 6-7 combine (caller's stream)
    hipEvent_t ev[8] = {nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr, nullptr};
    hipEvent_t ev_fork = nullptr; // treecode: the moments are done, band and ray tracing may start
    hipStream_t aux[2] = {nullptr, nullptr}; // the band and ray-tracing kernels run beside the far field
};

namespace {

int check_device(int *dev)
{
    int count = 0;
    hipError_t e = hipGetDeviceCount(&count);
    if (e != hipSuccess || count == 0)
        return fail(BS_E_DEVICE, "no HIP device available (hipGetDeviceCount: %s, count %d)", hipGetErrorString(e), count);
    int d = 0;
    e = hipGetDevice(&d);
    if (e != hipSuccess) return hip_fail(e, "hipGetDevice");
    hipDeviceProp_t prop;
    e = hipGetDeviceProperties(&prop, d);
    if (e != hipSuccess) return hip_fail(e, "hipGetDeviceProperties");
    if (std::strncmp(prop.gcnArchName, "gfx950", 6) != 0)
        return fail(BS_E_DEVICE, "device %d is %s, this library is built for gfx950", d, prop.gcnArchName);
    *dev = d;
    return BS_OK;
}

// Mean edge length over unique edges: keys (min id, max id) of the input
// numbering, lengths summed in increasing key order.
// Mean length of the unique edges, summed in the order of their sorted keys.
// The edge set depends on the connectivity alone, fixed for the mesh's
// lifetime, so it is sorted once and kept (moving the nodes, as every
// stage of the Lagrangian step does, only re-measures the lengths).
double mean_edge(bs_mesh *m)
{
    const int64_t n = m->n, T = m->T;
    const int32_t *tets = m->tets.data();
    const double *xyz = m->xyz.data();
    if (m->edge_keys.empty() && T > 0) {
        // sorted by the smaller node (a counting sort), then by the larger
        // within each node's few edges: the order of a full sort of the keys
        static const int ea[6] = {0, 0, 0, 1, 1, 2}, eb[6] = {1, 2, 3, 2, 3, 3};
        std::vector<int64_t> start((size_t)n + 1, 0);
        for (int64_t t = 0; t < T; ++t)
            for (int e = 0; e < 6; ++e) start[(size_t)std::min(tets[4 * t + ea[e]], tets[4 * t + eb[e]]) + 1]++;
        for (int64_t i = 0; i < n; ++i) start[(size_t)i + 1] += start[(size_t)i];
        std::vector<int32_t> hi((size_t)(6 * T));
        {
            std::vector<int64_t> fill(start.begin(), start.end() - 1);
            for (int64_t t = 0; t < T; ++t)
                for (int e = 0; e < 6; ++e) {
                    const int32_t a = tets[4 * t + ea[e]], b = tets[4 * t + eb[e]];
                    hi[(size_t)fill[(size_t)std::min(a, b)]++] = std::max(a, b);
                }
        }
        std::vector<int64_t> keys;
        keys.reserve((size_t)(6 * T) / 2);
        for (int64_t i = 0; i < n; ++i) {
            int32_t *b0 = hi.data() + start[(size_t)i], *b1 = hi.data() + start[(size_t)i + 1];
            std::sort(b0, b1);
            for (int32_t *p = b0; p < b1; ++p)
                if (p == b0 || *p != p[-1]) keys.push_back(i * (n + 1) + *p);
        }
        m->edge_keys.swap(keys);
    }
    double sum = 0.0;
    for (const int64_t key : m->edge_keys) {
        const int64_t lo = key / (n + 1), hi = key % (n + 1);
        const double dx = xyz[3 * hi] - xyz[3 * lo], dy = xyz[3 * hi + 1] - xyz[3 * lo + 1],
                     dz = xyz[3 * hi + 2] - xyz[3 * lo + 2];
        sum += std::sqrt(dx * dx + dy * dy + dz * dz);
    }
    return m->edge_keys.empty() ? 0.0 : sum / (double)m->edge_keys.size();
}

// Signed 6-volume of tet t (FP64) and its longest squared edge.
double tet_det(const bs_mesh *m, int64_t t, double *h2)
{
    const int32_t *id = &m->tets[4 * t];
    double v[4][3];
    for (int j = 0; j < 4; ++j)
        for (int c = 0; c < 3; ++c) v[j][c] = m->xyz[3 * (int64_t)id[j] + c];
    double e[3][3];
    for (int j = 0; j < 3; ++j)
        for (int c = 0; c < 3; ++c) e[j][c] = v[j + 1][c] - v[0][c];
    if (h2) {
        double h = 0.0;
        for (int a = 0; a < 4; ++a)
            for (int b = a + 1; b < 4; ++b) {
                const double dx = v[b][0] - v[a][0], dy = v[b][1] - v[a][1], dz = v[b][2] - v[a][2];
                h = std::max(h, dx * dx + dy * dy + dz * dz);
            }
        *h2 = h;
    }
    return e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) - e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
           e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
}

// Lower *cur to v (atomically).
void atomic_min(std::atomic<int64_t> &cur, int64_t v)
{
    int64_t c = cur.load();
    while (v < c && !cur.compare_exchange_weak(c, v)) {
    }
}

// Every coordinate and vorticity finite, every tet of non-zero volume and,
// after the first call, of the orientation it was uploaded with.  The tets
// are checked in parallel; the error names the first failing node or tet,
// as a check in order would.
int validate_geometry(bs_mesh *m)
{
    const int64_t n = m->n, T = m->T;
    std::atomic<int64_t> bad_x{INT64_MAX};
    parallel_for(3 * n, [&](int64_t a, int64_t b) {
        for (int64_t i = a; i < b; ++i)
            if (!std::isfinite(m->xyz[(size_t)i]) || !std::isfinite(m->omega[(size_t)i])) {
                atomic_min(bad_x, i);
                return;
            }
    });
    if (bad_x.load() != INT64_MAX)
        return fail(BS_E_NONFINITE, "non-finite coordinate or vorticity at node %lld", (long long)(bad_x.load() / 3));
    const bool have_orient = !m->orient.empty();
    if (!have_orient) m->orient.resize((size_t)T);
    std::atomic<int64_t> bad_t{INT64_MAX}, neg{0};
    parallel_for(T, [&](int64_t a, int64_t b) {
        int64_t ng = 0;
        for (int64_t t = a; t < b; ++t) {
            double h2;
            const double det = tet_det(m, t, &h2);
            const int8_t sg = det < 0 ? -1 : 1;
            if (!(std::fabs(det) > 1e-12 * h2 * std::sqrt(h2)) || (have_orient && m->orient[(size_t)t] != sg)) {
                atomic_min(bad_t, t);
                return;
            }
            ng += det < 0;
            if (!have_orient) m->orient[(size_t)t] = sg;
        }
        neg += ng;
    });
    const int64_t t = bad_t.load();
    if (t != INT64_MAX) {
        if (!have_orient) m->orient.clear();
        double h2;
        const double det = tet_det(m, t, &h2);
        if (!(std::fabs(det) > 1e-12 * h2 * std::sqrt(h2)))
            return fail(BS_E_DEGENERATE, "tetrahedron %lld has zero volume", (long long)t);
        return fail(BS_E_DEGENERATE, "tetrahedron %lld inverted relative to its uploaded orientation", (long long)t);
    }
    m->reoriented = neg.load();
    return BS_OK;
}

// Face neighbours of every tet (input numbering): the face opposite local
// vertex f of tet t is keyed by its sorted node triple.
void build_neighbours(bs_mesh *m)
{
    const int64_t T = m->T;
    m->nbr_in.assign((size_t)(4 * T), -1);
    m->manifold = true;
    struct FK {
        int32_t a, b, c;
        int64_t tf;
    };
    // faces in the order of (a, b, c, tf): a counting sort by the smallest
    // node a, then a sort of each node's few faces
    const int64_t n = m->n;
    std::vector<int64_t> start((size_t)n + 1, 0);
    for (int64_t t = 0; t < T; ++t)
        for (int f = 0; f < 4; ++f) {
            int32_t a = INT32_MAX;
            for (int j = 0; j < 4; ++j)
                if (j != f) a = std::min(a, m->tets[(size_t)(4 * t + j)]);
            start[(size_t)a + 1]++;
        }
    for (int64_t i = 0; i < n; ++i) start[(size_t)i + 1] += start[(size_t)i];
    std::vector<FK> fk((size_t)(4 * T));
    {
        std::vector<int64_t> fill(start.begin(), start.end() - 1);
        for (int64_t t = 0; t < T; ++t)
            for (int f = 0; f < 4; ++f) {
                int32_t v[3], k = 0;
                for (int j = 0; j < 4; ++j)
                    if (j != f) v[k++] = m->tets[(size_t)(4 * t + j)];
                std::sort(v, v + 3);
                fk[(size_t)fill[(size_t)v[0]]++] = {v[0], v[1], v[2], 4 * t + f};
            }
    }
    for (int64_t i = 0; i < n; ++i)
        std::sort(fk.begin() + start[(size_t)i], fk.begin() + start[(size_t)i + 1], [](const FK &x, const FK &y) {
            return x.b != y.b ? x.b < y.b : x.c != y.c ? x.c < y.c : x.tf < y.tf;
        });
    for (size_t i = 0; i < fk.size();) {
        size_t j = i + 1;
        while (j < fk.size() && fk[j].a == fk[i].a && fk[j].b == fk[i].b && fk[j].c == fk[i].c) ++j;
        if (j - i == 2) {
            m->nbr_in[(size_t)fk[i].tf] = (int32_t)(fk[i + 1].tf / 4);
            m->nbr_in[(size_t)fk[i + 1].tf] = (int32_t)(fk[i].tf / 4);
        } else if (j - i > 2) {
            m->manifold = false;
        }
        i = j;
    }
}

// The boundary is one connected, closed surface whose every edge is convex
// (a locally convex closed surface bounds a convex body): a ray leaving the
// mesh never re-enters it.
bool boundary_convex(const bs_mesh *m)
{
    if (!m->manifold) return false;
    const int64_t T = m->T;
    const double *X = m->xyz.data();
    struct BF {
        int32_t v[3]; // oriented outward
    };
    std::vector<BF> bf;
    for (int64_t t = 0; t < T; ++t)
        for (int f = 0; f < 4; ++f) {
            if (m->nbr_in[(size_t)(4 * t + f)] >= 0) continue;
            int32_t v[3], k = 0;
            for (int j = 0; j < 4; ++j)
                if (j != f) v[k++] = m->tets[(size_t)(4 * t + j)];
            const int32_t o = m->tets[(size_t)(4 * t + f)];
            double e1[3], e2[3], d[3];
            for (int c = 0; c < 3; ++c) {
                e1[c] = X[3 * (int64_t)v[1] + c] - X[3 * (int64_t)v[0] + c];
                e2[c] = X[3 * (int64_t)v[2] + c] - X[3 * (int64_t)v[0] + c];
                d[c] = X[3 * (int64_t)o + c] - X[3 * (int64_t)v[0] + c];
            }
            const double nx = e1[1] * e2[2] - e1[2] * e2[1], ny = e1[2] * e2[0] - e1[0] * e2[2],
                         nz = e1[0] * e2[1] - e1[1] * e2[0];
            if (nx * d[0] + ny * d[1] + nz * d[2] > 0) std::swap(v[1], v[2]);
            bf.push_back({{v[0], v[1], v[2]}});
        }
    if (bf.empty()) return false;
    // edges of boundary faces: (min, max) -> faces
    struct EK {
        int64_t key;
        int32_t face, other; // the face's third vertex
    };
    std::vector<EK> ek;
    ek.reserve(3 * bf.size());
    const int64_t n1 = m->n + 1;
    for (size_t i = 0; i < bf.size(); ++i)
        for (int e = 0; e < 3; ++e) {
            const int32_t a = bf[i].v[e], b = bf[i].v[(e + 1) % 3], c = bf[i].v[(e + 2) % 3];
            ek.push_back({(int64_t)std::min(a, b) * n1 + std::max(a, b), (int32_t)i, c});
        }
    std::sort(ek.begin(), ek.end(), [](const EK &x, const EK &y) { return x.key < y.key || (x.key == y.key && x.face < y.face); });
    std::vector<int32_t> parent(bf.size());
    for (size_t i = 0; i < bf.size(); ++i) parent[i] = (int32_t)i;
    auto find = [&](int32_t x) {
        while (parent[(size_t)x] != x) x = parent[(size_t)x] = parent[(size_t)parent[(size_t)x]];
        return x;
    };
    for (size_t i = 0; i < ek.size();) {
        size_t j = i + 1;
        while (j < ek.size() && ek[j].key == ek[i].key) ++j;
        if (j - i != 2) return false; // open or non-manifold boundary
        const BF &F = bf[(size_t)ek[i].face];
        const int32_t g = ek[i + 1].other; // vertex of the neighbouring face off the shared edge
        double e1[3], e2[3], d[3], l2 = 0;
        for (int c = 0; c < 3; ++c) {
            e1[c] = X[3 * (int64_t)F.v[1] + c] - X[3 * (int64_t)F.v[0] + c];
            e2[c] = X[3 * (int64_t)F.v[2] + c] - X[3 * (int64_t)F.v[0] + c];
            d[c] = X[3 * (int64_t)g + c] - X[3 * (int64_t)F.v[0] + c];
            l2 += d[c] * d[c] + e1[c] * e1[c];
        }
        const double nx = e1[1] * e2[2] - e1[2] * e2[1], ny = e1[2] * e2[0] - e1[0] * e2[2],
                     nz = e1[0] * e2[1] - e1[1] * e2[0];
        const double nn = std::sqrt(nx * nx + ny * ny + nz * nz);
        // outward normal: g must not lie outside the plane of F
        if (nx * d[0] + ny * d[1] + nz * d[2] > 1e-9 * nn * std::sqrt(l2)) return false;
        const int32_t ra = find(ek[i].face), rb = find(ek[i + 1].face);
        if (ra != rb) parent[(size_t)ra] = rb;
        i = j;
    }
    const int32_t r0 = find(0);
    for (size_t i = 1; i < bf.size(); ++i)
        if (find((int32_t)i) != r0) return false;
    return true;
}

// Everything that depends on coordinates and vorticity: node order, bins,
// per-tet records.  Connectivity is already validated.
// Order of n points (FP64 [n][3]) in which recursive median splits across
// the longest axis, at multiples of 64, leave every consecutive 64 spatially
// compact.
std::vector<int32_t> kd_leaf_order(const double *X, int64_t n)
{
    std::vector<int32_t> orig((size_t)n);
    for (int64_t i = 0; i < n; ++i) orig[(size_t)i] = (int32_t)i;
    struct Range {
        int64_t a, b;
    };
    // the ranges of one level are split in parallel: each split depends only
    // on its own range, so the order is that of splitting them one by one
    std::vector<Range> level{{0, n}};
    while (!level.empty()) {
        std::vector<int64_t> ks(level.size(), 0);
        parallel_items((int64_t)level.size(), [&](int64_t q) {
            const Range r = level[(size_t)q];
            const int64_t len = r.b - r.a;
            if (len <= bsk::kBlockNodes) return;
            double lo3[3] = {1e300, 1e300, 1e300}, hi3[3] = {-1e300, -1e300, -1e300};
            for (int64_t k = r.a; k < r.b; ++k)
                for (int c = 0; c < 3; ++c) {
                    const double v = X[3 * (int64_t)orig[(size_t)k] + c];
                    lo3[c] = std::min(lo3[c], v);
                    hi3[c] = std::max(hi3[c], v);
                }
            int ax = 0;
            for (int c = 1; c < 3; ++c)
                if (hi3[c] - lo3[c] > hi3[ax] - lo3[ax]) ax = c;
            int64_t k = ((len / 2 + bsk::kBlockNodes / 2) / bsk::kBlockNodes) * bsk::kBlockNodes;
            k = std::min(std::max<int64_t>(k, bsk::kBlockNodes), len - 1);
            std::nth_element(orig.begin() + r.a, orig.begin() + r.a + k, orig.begin() + r.b, [&](int32_t u, int32_t v) {
                const double xu = X[3 * (int64_t)u + ax], xv = X[3 * (int64_t)v + ax];
                return xu < xv || (xu == xv && u < v);
            });
            ks[(size_t)q] = k;
        });
        std::vector<Range> next;
        for (size_t q = 0; q < level.size(); ++q)
            if (ks[q]) {
                next.push_back({level[q].a, level[q].a + ks[q]});
                next.push_back({level[q].a + ks[q], level[q].b});
            }
        level.swap(next);
    }
    return orig;
}

// Bounding spheres of the 64-point blocks of points [p0, p0 + count) of the
// binary32 SoA coordinates (stride npad): centre of the box, radius with a
// margin.
void block_spheres(const std::vector<float> &xh, int npad, int64_t p0, int64_t count, float4 *out)
{
    const int nb = (int)((count + bsk::kBlockNodes - 1) / bsk::kBlockNodes);
    for (int b = 0; b < nb; ++b) {
        float bl[3] = {3e38f, 3e38f, 3e38f}, bh[3] = {-3e38f, -3e38f, -3e38f};
        const int64_t a = p0 + (int64_t)b * bsk::kBlockNodes, e = p0 + std::min<int64_t>(count, (int64_t)(b + 1) * bsk::kBlockNodes);
        for (int64_t p = a; p < e; ++p)
            for (int c = 0; c < 3; ++c) {
                bl[c] = std::min(bl[c], xh[(size_t)c * npad + p]);
                bh[c] = std::max(bh[c], xh[(size_t)c * npad + p]);
            }
        float cc[3];
        for (int c = 0; c < 3; ++c) cc[c] = 0.5f * (bl[c] + bh[c]);
        double r2 = 0.0;
        for (int64_t p = a; p < e; ++p) {
            double d2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                const double d = (double)xh[(size_t)c * npad + p] - cc[c];
                d2 += d * d;
            }
            r2 = std::max(r2, d2);
        }
        out[b] = make_float4(cc[0], cc[1], cc[2], (float)(std::sqrt(r2) * (1 + 1e-5) + 1e-6));
    }
}

bool uses_treecode(const bs_policy &P)
{
    return P.far_field == BS_FAR_TREECODE && (P.kind == BS_POLICY_FIXED || P.kind == BS_POLICY_LEARNED);
}

// The treecode's sphere of the points P[idx[k]], k in [a, b) (FP64 [.][3]):
// centre the midpoint of their bounding box, radius the largest distance to
// it, each operation in this order.
void tree_sphere(const double *P, const int32_t *idx, int64_t a, int64_t b, double c[3], double &r)
{
    double lo[3] = {INFINITY, INFINITY, INFINITY}, hi[3] = {-INFINITY, -INFINITY, -INFINITY};
    for (int64_t k = a; k < b; ++k)
        for (int q = 0; q < 3; ++q) {
            const double v = P[3 * (int64_t)idx[k] + q];
            lo[q] = std::min(lo[q], v);
            hi[q] = std::max(hi[q], v);
        }
    for (int q = 0; q < 3; ++q) c[q] = 0.5 * (lo[q] + hi[q]);
    double r2 = 0.0;
    for (int64_t k = a; k < b; ++k) {
        const double *x = P + 3 * (int64_t)idx[k];
        const double dx = x[0] - c[0], dy = x[1] - c[1], dz = x[2] - c[2];
        r2 = std::max(r2, (dx * dx + dy * dy) + dz * dz);
    }
    r = std::sqrt(r2);
}

// Breadth-first k-d tree of points C ([T][3] FP64): the node order's split
// rule (longest side of the bounding box, the k smallest by (coordinate,
// index) first, k the multiple of 64 nearest half the range), leaves of at
// most 64.  order: point at each tree position; range and child per cluster;
// level_start: first cluster of every level, then the count.
void tree_kd(const double *C, int64_t T, std::vector<int32_t> &order, std::vector<int2> &range,
             std::vector<int2> &child, std::vector<int> &level_start)
{
    order.resize((size_t)T);
    for (int64_t i = 0; i < T; ++i) order[(size_t)i] = (int32_t)i;
    range.assign(1, make_int2(0, (int)T));
    child.assign(1, make_int2(-1, -1));
    level_start.assign(1, 0);
    int l0 = 0;
    for (;;) {
        const int l1 = (int)range.size();
        std::vector<int> ks((size_t)(l1 - l0), 0);
        parallel_items(l1 - l0, [&](int64_t q) {
            const int a = range[(size_t)(l0 + q)].x, b = range[(size_t)(l0 + q)].y, len = b - a;
            if (len <= bsk::kBlockNodes) return;
            double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
            for (int k = a; k < b; ++k)
                for (int c = 0; c < 3; ++c) {
                    const double v = C[3 * (int64_t)order[(size_t)k] + c];
                    lo[c] = std::min(lo[c], v);
                    hi[c] = std::max(hi[c], v);
                }
            int ax = 0;
            for (int c = 1; c < 3; ++c)
                if (hi[c] - lo[c] > hi[ax] - lo[ax]) ax = c;
            int k = ((len / 2 + bsk::kBlockNodes / 2) / bsk::kBlockNodes) * bsk::kBlockNodes;
            k = std::min(std::max(k, bsk::kBlockNodes), len - 1);
            std::nth_element(order.begin() + a, order.begin() + a + k, order.begin() + b, [&](int32_t u, int32_t v) {
                const double xu = C[3 * (int64_t)u + ax], xv = C[3 * (int64_t)v + ax];
                return xu < xv || (xu == xv && u < v);
            });
            ks[(size_t)q] = k;
        });
        for (int q = 0; q < l1 - l0; ++q) {
            if (!ks[(size_t)q]) continue;
            const int2 r = range[(size_t)(l0 + q)];
            child[(size_t)(l0 + q)] = make_int2((int)range.size(), (int)range.size() + 1);
            range.push_back(make_int2(r.x, r.x + ks[(size_t)q]));
            range.push_back(make_int2(r.x + ks[(size_t)q], r.y));
            child.push_back(make_int2(-1, -1));
            child.push_back(make_int2(-1, -1));
        }
        level_start.push_back(l1);
        if ((int)range.size() == l1) break;
        l0 = l1;
    }
}

// Does a block (centre cB, radius rB) accept a cluster (cS, rS)?  The
// treecode's test, each FP64 operation in this order.
inline bool tree_accepts(const double *cB, double rB, const double *cS, double rS, double theta, double kappa)
{
    const double dx = cB[0] - cS[0], dy = cB[1] - cS[1], dz = cB[2] - cS[2];
    const double D2 = (dx * dx + dy * dy) + dz * dz;
    const double rho = std::max(rS / theta, rS + kappa);
    return D2 >= (rB + rho) * (rB + rho);
}

// The treecode plan of the current positions and policy (BS_FAR_TREECODE):
// tree of the tet centroids, cluster and block spheres, interaction lists of
// every node block and evaluation-point block, per-tet sources in tree
// order, and the moment buffers; uploaded on stream s.
int build_tree_plan(bs_mesh *m, hipStream_t s)
{
    auto &tp = m->tree;
    tp.valid = false;
    const bs_policy &P = m->pol;
    const int64_t n = m->n, T = m->T, tn = m->tn;
    const double *X = m->xyz.data();
    if (T <= 0) {
        tp.theta = P.tree_theta;
        tp.order = P.tree_order;
        tp.d_g4 = P.d_g4;
        tp.nnode = tp.nleaf = 0;
        tp.exp_nodes = tp.dir_nodes = tp.exp_pts = tp.dir_pts = tp.cov_nodes = tp.cov_pts = 0;
        tp.valid = true;
        return BS_OK;
    }
    // FP64 centroids of the 1-point rule's sources (the tree's points; the
    // sources themselves are laid out on the device by k_tree_sources)
    std::vector<double> cen((size_t)(3 * T));
    parallel_for(T, [&](int64_t a, int64_t b) {
        for (int64_t t = a; t < b; ++t) {
            const int32_t *id = &m->tets[(size_t)(4 * t)];
            for (int c = 0; c < 3; ++c)
                cen[(size_t)(3 * t + c)] = (((X[3 * (int64_t)id[0] + c] + X[3 * (int64_t)id[1] + c]) +
                                             X[3 * (int64_t)id[2] + c]) + X[3 * (int64_t)id[3] + c]) * 0.25;
        }
    });
    std::vector<int32_t> order;
    std::vector<int2> range, child;
    tree_kd(cen.data(), T, order, range, child, tp.level_start);
    const int nnode = (int)range.size();
    std::vector<int> leaves;
    for (int j = 0; j < nnode; ++j)
        if (child[(size_t)j].x < 0) leaves.push_back(j);
    std::vector<double> c64((size_t)4 * nnode);
    std::vector<float> crec((size_t)8 * nnode, 0.f);
    parallel_items(nnode, [&](int64_t j) {
        double c[3], r;
        tree_sphere(cen.data(), order.data(), range[(size_t)j].x, range[(size_t)j].y, c, r);
        for (int q = 0; q < 3; ++q) {
            c64[(size_t)(4 * j + q)] = c[q];
            const float h = (float)c[q];
            crec[(size_t)(8 * j + q)] = h;
            crec[(size_t)(8 * j + 3 + q)] = (float)(c[q] - (double)h);
        }
        c64[(size_t)(4 * j + 3)] = r;
    });

    // target blocks: the nodes' (0 .. nblk-1) and the points' (tblk0 ..)
    const double kappa = std::max(P.d_g4 * m->hbar, m->max_vc) * (1.0 + 1e-3);
    const int nbt = std::max(m->nblk, m->tblk0 + m->tnblk);
    std::vector<int32_t> orig((size_t)n);
    for (int64_t i = 0; i < n; ++i) orig[(size_t)m->h_rank[(size_t)i]] = (int32_t)i;
    std::vector<std::vector<int>> acc((size_t)nbt), dir((size_t)nbt);
    std::vector<int> bcount((size_t)nbt, 0);
    parallel_items(nbt, [&](int64_t b) {
        const double *Pt;
        const int32_t *idx;
        int64_t cnt;
        if (b < m->nblk) {
            Pt = X;
            idx = orig.data() + 64 * b;
            cnt = std::min<int64_t>(64, n - 64 * b);
        } else if (b >= m->tblk0 && b < m->tblk0 + m->tnblk) {
            Pt = m->tgt.data();
            idx = m->h_torig.data() + 64 * (b - m->tblk0);
            cnt = std::min<int64_t>(64, tn - 64 * (b - m->tblk0));
        } else {
            return;
        }
        bcount[(size_t)b] = (int)cnt;
        double cB[3], rB;
        tree_sphere(Pt, idx, 0, cnt, cB, rB);
        std::vector<int> stack{0};
        while (!stack.empty()) {
            const int j = stack.back();
            stack.pop_back();
            if (tree_accepts(cB, rB, &c64[(size_t)(4 * j)], c64[(size_t)(4 * j + 3)], P.tree_theta, kappa))
                acc[(size_t)b].push_back(j);
            else if (child[(size_t)j].x < 0)
                dir[(size_t)b].push_back(j);
            else {
                stack.push_back(child[(size_t)j].y);
                stack.push_back(child[(size_t)j].x);
            }
        }
    });
    {
        // the lists are indexed in 32 bits on the device
        int64_t na = 0, nd = 0;
        for (int b = 0; b < nbt; ++b) {
            na += (int64_t)acc[(size_t)b].size();
            nd += (int64_t)dir[(size_t)b].size();
        }
        if (na > INT32_MAX || nd > INT32_MAX)
            return fail(BS_E_NOMEM, "treecode interaction lists too long for 32-bit indexing (%lld, %lld entries)",
                        (long long)na, (long long)nd);
    }
    std::vector<int> acc_start((size_t)nbt + 1, 0), dir_start((size_t)nbt + 1, 0);
    tp.exp_nodes = tp.dir_nodes = tp.exp_pts = tp.dir_pts = tp.cov_nodes = tp.cov_pts = 0;
    for (int b = 0; b < nbt; ++b) {
        acc_start[(size_t)b + 1] = acc_start[(size_t)b] + (int)acc[(size_t)b].size();
        dir_start[(size_t)b + 1] = dir_start[(size_t)b] + (int)dir[(size_t)b].size();
        int64_t dt = 0, ct = 0;
        for (int j : dir[(size_t)b]) dt += range[(size_t)j].y - range[(size_t)j].x;
        for (int j : acc[(size_t)b]) ct += range[(size_t)j].y - range[(size_t)j].x;
        const int64_t ex = (int64_t)acc[(size_t)b].size() * bcount[(size_t)b], dp = dt * bcount[(size_t)b],
                      cv = ct * bcount[(size_t)b];
        if (b < m->nblk) {
            tp.exp_nodes += ex;
            tp.dir_nodes += dp;
            tp.cov_nodes += cv;
        } else {
            tp.exp_pts += ex;
            tp.dir_pts += dp;
            tp.cov_pts += cv;
        }
    }
    std::vector<int> acc_list((size_t)std::max(1, acc_start.back())), dir_list((size_t)std::max(1, dir_start.back()));
    for (int b = 0; b < nbt; ++b) {
        std::copy(acc[(size_t)b].begin(), acc[(size_t)b].end(), acc_list.begin() + acc_start[(size_t)b]);
        std::copy(dir[(size_t)b].begin(), dir[(size_t)b].end(), dir_list.begin() + dir_start[(size_t)b]);
    }


    const int NK = bsk::tree_ncoef(P.tree_order), NC = bsk::tree_ncoef(P.tree_order + 1) - 1;
    int rc;
    if ((rc = dalloc(tp.nrange, sizeof(int2) * range.size())) || (rc = dalloc(tp.child, sizeof(int2) * child.size())) ||
        (rc = dalloc(tp.leaves, 4 * leaves.size())) || (rc = dalloc(tp.c64, 8 * c64.size())) ||
        (rc = dalloc(tp.crec, 4 * crec.size())) || (rc = dalloc(tp.src64, 8 * 8 * (size_t)T)) ||
        (rc = dalloc(tp.g1t, 4 * 8 * (size_t)T)) || (rc = dalloc(tp.tidt, sizeof(int4) * (size_t)T)) ||
        (rc = dalloc(tp.torder, 4 * (size_t)T)) || (rc = dalloc(tp.tin, 16 * (size_t)T)) ||
        (rc = dalloc(tp.x64, 8 * 3 * (size_t)n)) || (rc = dalloc(tp.rank, 4 * (size_t)n)) ||
        (rc = dalloc(tp.M, 8 * 3 * (size_t)nnode * NK)) || (rc = dalloc(tp.N, 4 * 3 * (size_t)nnode * NC)) ||
        (rc = dalloc(tp.acc_start, 4 * acc_start.size())) || (rc = dalloc(tp.acc, 4 * acc_list.size())) ||
        (rc = dalloc(tp.dir_start, 4 * dir_start.size())) || (rc = dalloc(tp.dir, 4 * dir_list.size())))
        return rc;
    hipError_t e;
#define BS_UP(buf, vec)                                                                                            \
    if ((e = hipMemcpyAsync(tp.buf.p, (vec).data(), sizeof((vec)[0]) * (vec).size(), hipMemcpyHostToDevice, s)) != \
        hipSuccess)                                                                                                \
        return hip_fail(e, "upload tree " #buf);
    BS_UP(nrange, range)
    BS_UP(child, child)
    BS_UP(leaves, leaves)
    BS_UP(c64, c64)
    BS_UP(crec, crec)
    BS_UP(torder, order)
    BS_UP(x64, m->xyz)
    BS_UP(rank, m->h_rank)
    if (!tp.tin_valid) {
        BS_UP(tin, m->tets)
        tp.tin_valid = true;
    }
    BS_UP(acc_start, acc_start)
    BS_UP(acc, acc_list)
    BS_UP(dir_start, dir_start)
    BS_UP(dir, dir_list)
#undef BS_UP
    if ((e = bsk::launch_tree_sources((int)T, (const int *)tp.torder.p, (const int4 *)tp.tin.p, (const double *)tp.x64.p,
                                      (const double *)m->om64.p, (const int *)tp.rank.p, (double *)tp.src64.p,
                                      (float *)tp.g1t.p, (int4 *)tp.tidt.p, s)))
        return hip_fail(e, "treecode sources");
    if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "upload tree");
    tp.nnode = nnode;
    tp.nleaf = (int)leaves.size();
    tp.theta = P.tree_theta;
    tp.order = P.tree_order;
    tp.d_g4 = P.d_g4;
    tp.valid = true;
    return BS_OK;
}

// Parts each target block's treecode lists are cut into: about four waves
// per wave slot of the chip (256 CUs x 4 SIMDs x 8) over the node blocks.
int tree_chunks(const bs_mesh *m)
{
    const int nb = std::max(1, m->nblk);
    return std::max(1, std::min(bsk::kTreeMaxChunks, (32768 + nb - 1) / nb));
}

bsk::TreeView tree_view(bs_mesh *m)
{
    bsk::TreeView t{};
    auto &tp = m->tree;
    t.order = tp.order;
    t.nnode = tp.nnode;
    t.nleaf = tp.nleaf;
    t.nrange = (const int2 *)tp.nrange.p;
    t.child = (const int2 *)tp.child.p;
    t.leaves = (const int *)tp.leaves.p;
    t.c64 = (const double *)tp.c64.p;
    t.crec = (const float *)tp.crec.p;
    t.src64 = (const double *)tp.src64.p;
    t.g1t = (const float *)tp.g1t.p;
    t.tidt = (const int4 *)tp.tidt.p;
    t.M = (double *)tp.M.p;
    t.N = (float *)tp.N.p;
    t.acc_start = (const int *)tp.acc_start.p;
    t.acc = (const int *)tp.acc.p;
    t.dir_start = (const int *)tp.dir_start.p;
    t.dir = (const int *)tp.dir.p;
    return t;
}

// A thread joined when the object goes out of scope (every return path).
struct JoinedThread {
    std::thread t;
    template <class F>
    explicit JoinedThread(F &&f) : t(std::forward<F>(f))
    {
    }
    void join()
    {
        if (t.joinable()) t.join();
    }
    ~JoinedThread() { join(); }
};

int build_device_mesh(bs_mesh *m, hipStream_t s)
{
    int rc;
    m->vel_valid = false;
    const int64_t n = m->n, T = m->T;
    const double *X = m->xyz.data(), *W = m->omega.data();
    // two serial passes that depend on the positions and connectivity only
    // run beside the node ordering: the mean edge length (summed in the
    // sorted order of the unique edges, as the oracle sums it) and the
    // boundary's convexity
    double hbar = 0.0;
    bool convex = false;
    JoinedThread th_hbar([&] { hbar = T > 0 ? mean_edge(m) : 0.0; });
    JoinedThread th_convex([&] { convex = T > 0 && boundary_convex(m); });

    // ---- nodes ordered by a k-d split into leaves of 64 (one band-kernel
    // block per leaf); evaluation points (bs_eval_points) follow the nodes
    // from t0 = n rounded up to 1024, ordered the same way among themselves
    const std::vector<int32_t> orig = kd_leaf_order(X, n);
    std::vector<int32_t> rank((size_t)n);
    for (int64_t i = 0; i < n; ++i) rank[(size_t)orig[(size_t)i]] = (int32_t)i;
    const int64_t tn = m->tn;
    const std::vector<int32_t> torig = kd_leaf_order(m->tgt.data(), tn);
    m->h_torig = torig;
    m->tree.valid = false;
    const int64_t t0 = tn > 0 ? ((n + 1023) / 1024) * 1024 : n;
    const int npad = (int)(((t0 + tn + 1023) / 1024) * 1024);
    const int nblk = (int)((n + bsk::kBlockNodes - 1) / bsk::kBlockNodes);
    const int tblk0 = (int)(t0 / bsk::kBlockNodes);
    const int tnblk = (int)((tn + bsk::kBlockNodes - 1) / bsk::kBlockNodes);
    m->npad = npad;
    m->nblk = nblk;
    m->t0 = (int)t0;
    m->tblk0 = tblk0;
    m->tnblk = tnblk;
    std::vector<float> xh((size_t)3 * npad), xl((size_t)3 * npad), om((size_t)3 * npad);
    double max_abs = 0.0;
    for (int64_t p = 0; p < npad; ++p) {
        const bool is_t = p >= t0 && p < t0 + tn;
        const int64_t i = p < n ? orig[(size_t)p] : is_t ? torig[(size_t)(p - t0)] : (n > 0 ? orig[0] : 0);
        for (int c = 0; c < 3; ++c) {
            const double x = is_t ? m->tgt[3 * i + c] : (n > 0 ? X[3 * i + c] : 0.0);
            const float h = (float)x;
            max_abs = std::max(max_abs, std::fabs(x));
            xh[(size_t)c * npad + p] = h;
            xl[(size_t)c * npad + p] = (float)(x - (double)h);
            om[(size_t)c * npad + p] = (is_t || n == 0) ? 0.f : (float)W[3 * i + c];
        }
    }
    std::vector<float4> nrec((size_t)2 * npad);
    for (int64_t p = 0; p < npad; ++p) {
        const size_t i0 = (size_t)p, i1 = (size_t)(npad + p), i2 = (size_t)(2 * npad + p);
        nrec[(size_t)(2 * p)] = make_float4(xh[i0], xh[i1], xh[i2], xl[i0]);
        nrec[(size_t)(2 * p + 1)] = make_float4(xl[i1], xl[i2], om[i0], om[i1]);
    }
    std::vector<float4> blk((size_t)std::max(nblk, tblk0 + tnblk));
    block_spheres(xh, npad, 0, n, blk.data());
    if (tn > 0) block_spheres(xh, npad, t0, tn, blk.data() + tblk0);
    std::vector<int32_t> tlist((size_t)tn + 1);
    for (int64_t k = 0; k < tn; ++k) tlist[(size_t)k] = (int32_t)(t0 + k);
    tlist[(size_t)tn] = (int32_t)tn;

    th_hbar.join();
    m->hbar = hbar;

    // ---- tets: centroids, bins
    std::vector<double> cen((size_t)(3 * T));
    std::vector<float> cen32((size_t)(3 * T));
    double clo[3] = {1e300, 1e300, 1e300}, chi[3] = {-1e300, -1e300, -1e300};
    double max_vc = 0.0;
    {
        // chunks in parallel, their extremes combined after (min and max are
        // exact, so the result does not depend on the split)
        const int64_t nch = std::max<int64_t>(1, std::min<int64_t>(64, T / 4096));
        std::vector<double> part((size_t)(7 * nch));
        parallel_items(nch, [&](int64_t c0) {
            double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300}, mv = 0.0;
            for (int64_t t = T * c0 / nch; t < T * (c0 + 1) / nch; ++t) {
                const int32_t *id = &m->tets[4 * t];
                double vc = 0.0;
                for (int c = 0; c < 3; ++c) {
                    const double v = (((X[3 * (int64_t)id[0] + c] + X[3 * (int64_t)id[1] + c]) +
                                       X[3 * (int64_t)id[2] + c]) + X[3 * (int64_t)id[3] + c]) * 0.25;
                    cen[(size_t)(3 * t + c)] = v;
                    cen32[(size_t)(3 * t + c)] = (float)v;
                    lo[c] = std::min(lo[c], v);
                    hi[c] = std::max(hi[c], v);
                }
                for (int j = 0; j < 4; ++j) {
                    double d2 = 0.0;
                    for (int c = 0; c < 3; ++c) {
                        const double d = X[3 * (int64_t)id[j] + c] - cen[(size_t)(3 * t + c)];
                        d2 += d * d;
                    }
                    vc = std::max(vc, d2);
                }
                mv = std::max(mv, std::sqrt(vc));
            }
            for (int c = 0; c < 3; ++c) {
                part[(size_t)(7 * c0 + c)] = lo[c];
                part[(size_t)(7 * c0 + 3 + c)] = hi[c];
            }
            part[(size_t)(7 * c0 + 6)] = mv;
        });
        for (int64_t c0 = 0; c0 < nch && T > 0; ++c0) {
            for (int c = 0; c < 3; ++c) {
                clo[c] = std::min(clo[c], part[(size_t)(7 * c0 + c)]);
                chi[c] = std::max(chi[c], part[(size_t)(7 * c0 + 3 + c)]);
            }
            max_vc = std::max(max_vc, part[(size_t)(7 * c0 + 6)]);
        }
    }
    m->max_vc = max_vc;
    m->max_abs = max_abs;
    bsk::Bins bins{};
    double cs = 2.0 * (m->hbar > 0 ? m->hbar : 1.0);
    if (T > 0) {
        // keep the bin count modest for very spread meshes
        for (;;) {
            int64_t tot = 1;
            for (int c = 0; c < 3; ++c) tot *= (int64_t)std::floor((chi[c] - clo[c]) / cs) + 1;
            if (tot <= std::max<int64_t>(64, 4 * T) && tot <= (1 << 26)) break;
            cs *= 1.5;
        }
    }
    for (int c = 0; c < 3; ++c) {
        bins.lo[c] = T > 0 ? (float)(clo[c] - 1e-3 * cs) : 0.f;
        bins.dim[c] = T > 0 ? (int)std::floor((chi[c] + 1e-3 * cs - (double)bins.lo[c]) / cs) + 1 : 1;
    }
    bins.cs = (float)cs;
    m->bins = bins;
    const int64_t ncell = (int64_t)bins.dim[0] * bins.dim[1] * bins.dim[2];
    std::vector<int32_t> cell_of((size_t)T), cell_start, order;
    parallel_for(T, [&](int64_t a, int64_t b) {
        for (int64_t t = a; t < b; ++t) {
            int ic[3];
            for (int c = 0; c < 3; ++c) {
                int k = (int)std::floor((cen32[(size_t)(3 * t + c)] - bins.lo[c]) / bins.cs);
                ic[c] = std::min(bins.dim[c] - 1, std::max(0, k));
            }
            cell_of[(size_t)t] = (ic[2] * bins.dim[1] + ic[1]) * bins.dim[0] + ic[0];
        }
    });
    // tets by bin, in input order within a bin
    stable_bucket(T, ncell, [&](int64_t t) { return cell_of[(size_t)t]; }, cell_start, order);

    m->h_rank = rank;
    m->h_order = order;
    m->h_cell_start = cell_start;
    m->h_cen32 = cen32;
    m->h_xh.resize((size_t)(3 * n));
    for (int64_t i = 0; i < 3 * n; ++i) m->h_xh[(size_t)i] = (float)X[i];

    // ---- per-tet records in bin order
    // host staging of the records, kept between builds (every element is
    // rewritten below): moving the nodes rebuilds them at each Lagrangian
    // stage, and fresh multi-GB vectors cost more to zero and fault in than
    // to fill
    if ((rc = pinned_reserve(m->h_g1, 4 * (size_t)T * 8)) || (rc = pinned_reserve(m->h_g4, 4 * (size_t)T * 32)) ||
        (rc = pinned_reserve(m->h_g11, 4 * (size_t)T * 88)))
        return rc;
    float *g1 = (float *)m->h_g1.p, *g4 = (float *)m->h_g4.p, *g11 = (float *)m->h_g11.p;
    std::vector<int4> &tid = m->h_tid;
    tid.resize((size_t)T);
    const TetRule R1 = tet_rule(1), R4 = tet_rule(4), R11 = tet_rule(11);
    parallel_for(T, [&](int64_t a, int64_t b) {
        for (int64_t k = a; k < b; ++k) {
            const int64_t t = order[(size_t)k];
            const int32_t *id = &m->tets[4 * t];
            double v[4][3], w[4][3];
            for (int j = 0; j < 4; ++j)
                for (int c = 0; c < 3; ++c) {
                    v[j][c] = X[3 * (int64_t)id[j] + c];
                    w[j][c] = W[3 * (int64_t)id[j] + c];
                }
            double e[3][3];
            for (int j = 0; j < 3; ++j)
                for (int c = 0; c < 3; ++c) e[j][c] = v[j + 1][c] - v[0][c];
            const double det = e[0][0] * (e[1][1] * e[2][2] - e[1][2] * e[2][1]) -
                               e[0][1] * (e[1][0] * e[2][2] - e[1][2] * e[2][0]) +
                               e[0][2] * (e[1][0] * e[2][1] - e[1][1] * e[2][0]);
            const double vol = std::fabs(det) / 6.0;
            auto put = [&](const TetRule &r, float *dst) {
                for (int q = 0; q < r.n; ++q) {
                    double p[3] = {0, 0, 0}, o[3] = {0, 0, 0};
                    for (int j = 0; j < 4; ++j)
                        for (int c = 0; c < 3; ++c) {
                            p[c] += r.lam[q][j] * v[j][c];
                            o[c] += r.lam[q][j] * w[j][c];
                        }
                    const double f = r.w[q] * vol / (4.0 * M_PI);
                    for (int c = 0; c < 3; ++c) {
                        dst[8 * q + c] = (float)p[c];
                        dst[8 * q + 3 + c] = (float)(f * o[c]);
                    }
                    dst[8 * q + 6] = 0.f;
                    dst[8 * q + 7] = 0.f;
                }
            };
            put(R1, &g1[(size_t)k * 8]);
            // the 1-point rule sits at the centroid used for the rule decision
            for (int c = 0; c < 3; ++c) g1[(size_t)k * 8 + c] = cen32[(size_t)(3 * t + c)];
            put(R4, &g4[(size_t)k * 32]);
            put(R11, &g11[(size_t)k * 88]);
            tid[(size_t)k] = make_int4(rank[(size_t)id[0]], rank[(size_t)id[1]], rank[(size_t)id[2]],
                                       rank[(size_t)id[3]]);
        }
    });
    // the records (most of the bytes uploaded) go to the device now, from
    // pinned memory, while the host builds the rest; every later return
    // first waits for these copies (the staging is rewritten by the next
    // build)
    if ((rc = dalloc(m->g1, 4 * (size_t)T * 8)) || (rc = dalloc(m->g4, 4 * (size_t)T * 32)) ||
        (rc = dalloc(m->g11, 4 * (size_t)T * 88)))
        return rc;
    {
        hipError_t e;
        if (T > 0 && ((e = hipMemcpyAsync(m->g1.p, g1, 4 * (size_t)T * 8, hipMemcpyHostToDevice, s)) ||
                      (e = hipMemcpyAsync(m->g4.p, g4, 4 * (size_t)T * 32, hipMemcpyHostToDevice, s)) ||
                      (e = hipMemcpyAsync(m->g11.p, g11, 4 * (size_t)T * 88, hipMemcpyHostToDevice, s)))) {
            (void)hipStreamSynchronize(s);
            return hip_fail(e, "upload Gauss records");
        }
    }
    auto wait_records = [&](int r) {
        (void)hipStreamSynchronize(s);
        return r;
    };

    // ---- bounding sphere of the binary32 centroids of every tile of 16
    // consecutive (sorted) tets, for the far kernel's band flags
    const int64_t ntile = (T + 15) / 16;
    std::vector<float4> tsph((size_t)std::max<int64_t>(ntile, 1));
    for (int64_t k = 0; k < ntile; ++k) {
        const int64_t a = 16 * k, b = std::min<int64_t>(T, a + 16);
        double lo[3] = {1e300, 1e300, 1e300}, hi[3] = {-1e300, -1e300, -1e300};
        for (int64_t t = a; t < b; ++t)
            for (int c = 0; c < 3; ++c) {
                lo[c] = std::min(lo[c], (double)g1[(size_t)t * 8 + c]);
                hi[c] = std::max(hi[c], (double)g1[(size_t)t * 8 + c]);
            }
        const float cc[3] = {(float)(0.5 * (lo[0] + hi[0])), (float)(0.5 * (lo[1] + hi[1])), (float)(0.5 * (lo[2] + hi[2]))};
        double r2 = 0.0;
        for (int64_t t = a; t < b; ++t) {
            double d2 = 0.0;
            for (int c = 0; c < 3; ++c) {
                const double d = (double)g1[(size_t)t * 8 + c] - (double)cc[c];
                d2 += d * d;
            }
            r2 = std::max(r2, d2);
        }
        tsph[(size_t)k] = make_float4(cc[0], cc[1], cc[2], (float)(std::sqrt(r2) * (1.0 + 1e-5) + 1e-6));
    }

    // ---- face neighbours (sorted numbering) and incident tets per node
    std::vector<int32_t> slot((size_t)T);
    parallel_for(T, [&](int64_t a, int64_t b) {
        for (int64_t k = a; k < b; ++k) slot[(size_t)order[(size_t)k]] = (int32_t)k;
    });
    std::vector<int4> nbr((size_t)T);
    parallel_for(T, [&](int64_t a, int64_t b) {
        for (int64_t k = a; k < b; ++k) {
            const int64_t t = order[(size_t)k];
            int32_t q[4];
            for (int f = 0; f < 4; ++f) {
                const int32_t u = m->nbr_in[(size_t)(4 * t + f)];
                q[f] = u >= 0 ? slot[(size_t)u] : -1;
            }
            nbr[(size_t)k] = make_int4(q[0], q[1], q[2], q[3]);
        }
    });
    // the tets incident to each node, in increasing sorted position: each
    // node's corners (input numbering, fixed with the connectivity: bucketed
    // once) renumbered and sorted, nodes in parallel
    if (m->inc_in_start.empty())
        stable_bucket(4 * T, n, [&](int64_t i) { return m->tets[(size_t)i]; }, m->inc_in_start, m->inc_in_list);
    std::vector<int32_t> inc_start((size_t)n + 1), inc_list((size_t)(4 * T));
    inc_start[0] = 0;
    for (int64_t r = 0; r < n; ++r) {
        const int32_t i = orig[(size_t)r];
        inc_start[(size_t)r + 1] = inc_start[(size_t)r] + (m->inc_in_start[(size_t)i + 1] - m->inc_in_start[(size_t)i]);
    }
    parallel_for(n, [&](int64_t a, int64_t b) {
        for (int64_t r = a; r < b; ++r) {
            const int32_t i = orig[(size_t)r], c0 = m->inc_in_start[(size_t)i], c1 = m->inc_in_start[(size_t)i + 1];
            int32_t *o = &inc_list[(size_t)inc_start[(size_t)r]];
            for (int32_t c = c0; c < c1; ++c) o[c - c0] = slot[(size_t)(m->inc_in_list[(size_t)c] >> 2)];
            std::sort(o, o + (c1 - c0));
        }
    });
    th_convex.join();
    m->convex = convex;

    // ---- upload
    const size_t nb = sizeof(float) * 3 * (size_t)npad;
    if ((rc = dalloc(m->xh, nb)) || (rc = dalloc(m->xl, nb)) || (rc = dalloc(m->om, nb)) ||
        (rc = dalloc(m->nrec, sizeof(float4) * nrec.size())) ||
        (rc = dalloc(m->blk, sizeof(float4) * blk.size())) || (rc = dalloc(m->node_orig, 4 * (size_t)n)) ||
        (rc = dalloc(m->torig, 4 * torig.size())) || (rc = dalloc(m->tlist, 4 * tlist.size())) ||
        (rc = dalloc(m->tvel, 8 * 3 * (size_t)tn)) || (rc = dalloc(m->tid, sizeof(int4) * (size_t)T)) ||
        (rc = dalloc(m->cell_start, 4 * cell_start.size())) || (rc = dalloc(m->band, 8 * 3 * (size_t)npad)) ||
        (rc = dalloc(m->rtv, 8 * 3 * (size_t)npad)) || (rc = dalloc(m->vel, 8 * 3 * (size_t)n)) ||
        (rc = dalloc(m->cnt, 8 * bsk::kCntWords)) || (rc = dalloc(m->nonfinite, 4)) ||
        (rc = dalloc(m->nbr, sizeof(int4) * (size_t)T)) ||
        (rc = dalloc(m->tsph, sizeof(float4) * tsph.size())) || (rc = dalloc(m->inc_start, 4 * inc_start.size())) ||
        (rc = dalloc(m->inc_list, 4 * inc_list.size())) || (rc = dalloc(m->om64, 8 * 3 * (size_t)std::max<int64_t>(n, 1))))
        return wait_records(rc);
    hipError_t e;
#define BS_UP(buf, vec)                                                                                            \
    if (!(vec).empty() &&                                                                                          \
        (e = hipMemcpyAsync(m->buf.p, (vec).data(), sizeof((vec)[0]) * (vec).size(), hipMemcpyHostToDevice, s)) != \
            hipSuccess)                                                                                            \
        return wait_records(hip_fail(e, "upload " #buf));
    BS_UP(xh, xh)
    BS_UP(xl, xl)
    BS_UP(om, om)
    BS_UP(nrec, nrec)
    BS_UP(blk, blk)
    BS_UP(node_orig, orig)
    BS_UP(torig, torig)
    BS_UP(tlist, tlist)
    BS_UP(tid, tid)
    BS_UP(cell_start, cell_start)
    BS_UP(nbr, nbr)
    BS_UP(tsph, tsph)
    BS_UP(inc_start, inc_start)
    BS_UP(inc_list, inc_list)
    BS_UP(om64, m->omega)
#undef BS_UP
    e = hipStreamSynchronize(s);
    if (e != hipSuccess) return hip_fail(e, "upload");
    if (uses_treecode(m->pol) && (rc = build_tree_plan(m, s))) return rc;
    return BS_OK;
}

int read_inputs(bs_mesh *m, const double *xyz, const double *omega, uint32_t flags, hipStream_t s)
{
    const size_t bytes = sizeof(double) * 3 * (size_t)m->n;
    if (flags & BS_PTR_DEVICE) {
        hipError_t e;
        if (xyz && (e = hipMemcpyAsync(m->xyz.data(), xyz, bytes, hipMemcpyDeviceToHost, s)) != hipSuccess)
            return hip_fail(e, "read xyz");
        if (omega && (e = hipMemcpyAsync(m->omega.data(), omega, bytes, hipMemcpyDeviceToHost, s)) != hipSuccess)
            return hip_fail(e, "read omega");
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "read inputs");
    } else {
        if (xyz) std::memcpy(m->xyz.data(), xyz, bytes);
        if (omega) std::memcpy(m->omega.data(), omega, bytes);
    }
    return BS_OK;
}

int install_angular(bs_mesh *m)
{
    const int N = m->pol.n_phi, M = m->pol.n_theta;
    if (N == m->ang_N && M == m->ang_M) return BS_OK;
    std::vector<double> tn, wn, tm, wm;
    gauss_legendre(N, tn, wn);
    gauss_legendre(M, tm, wm);
    const int M2 = 2 * M;
    std::vector<float4> dir((size_t)N * M2);
    std::vector<double> dir64((size_t)N * M2 * 3);
    std::vector<float> cphi((size_t)N), dia((size_t)M2);
    for (int n = 0; n < N; ++n) cphi[(size_t)n] = (float)std::cos((1.0 + tn[(size_t)n]) * M_PI / 2.0);
    for (int j = 0; j < M2; ++j) {
        const double th = (1.0 + tm[(size_t)(j % M)]) * M_PI / 2.0 + (j >= M ? M_PI : 0.0);
        const float c = (float)std::cos(th), s = (float)std::sin(th);
        float d;
        if (s >= 0.f) d = c >= 0.f ? s / (c + s) : 1.f - c / (-c + s);
        else d = c < 0.f ? 2.f - s / (-c - s) : 3.f + c / (c - s);
        dia[(size_t)j] = d;
    }
    for (int n = 0; n < N; ++n)
        for (int j = 0; j < M2; ++j) {
            // ray (n, j): line (n, j) for j < M; the reverse of line (N-1-n, j-M) otherwise
            const bool rev = j >= M;
            const int ln = rev ? N - 1 - n : n, lm = rev ? j - M : j;
            const double phi = (1.0 + tn[(size_t)ln]) * M_PI / 2.0;
            const double th = (1.0 + tm[(size_t)lm]) * M_PI / 2.0;
            const double sg = rev ? -1.0 : 1.0;
            const double d[3] = {sg * std::sin(phi) * std::cos(th), sg * std::sin(phi) * std::sin(th),
                                 sg * std::cos(phi)};
            const double k = M_PI / 16.0 * std::sin(phi) * wn[(size_t)ln] * wm[(size_t)lm];
            const size_t l = (size_t)n * M2 + j;
            dir[l] = make_float4((float)d[0], (float)d[1], (float)d[2], (float)k);
            for (int c = 0; c < 3; ++c) dir64[3 * l + c] = d[c];
        }
    int rc;
    if ((rc = dalloc(m->dir, sizeof(float4) * dir.size())) || (rc = dalloc(m->dir64, 8 * dir64.size())) ||
        (rc = dalloc(m->cphi, 4 * cphi.size())) || (rc = dalloc(m->dia, 4 * dia.size())))
        return rc;
    hipError_t e;
    if ((e = hipMemcpy(m->dir.p, dir.data(), sizeof(float4) * dir.size(), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(m->dir64.p, dir64.data(), 8 * dir64.size(), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(m->cphi.p, cphi.data(), 4 * cphi.size(), hipMemcpyHostToDevice)) ||
        (e = hipMemcpy(m->dia.p, dia.data(), 4 * dia.size(), hipMemcpyHostToDevice)))
        return hip_fail(e, "upload angular tables");
    m->ang_N = N;
    m->ang_M = M;
    return BS_OK;
}

bsk::DevMesh dev_view(const bs_mesh *m)
{
    bsk::DevMesh d{};
    d.n = (int)m->n;
    d.npad = m->npad;
    d.T = (int)m->T;
    d.nblk = m->nblk;
    d.xh = (const float *)m->xh.p;
    d.xl = (const float *)m->xl.p;
    d.om = (const float *)m->om.p;
    d.nrec = (const float4 *)m->nrec.p;
    d.blk = (const float4 *)m->blk.p;
    d.g1 = (const float *)m->g1.p;
    d.g4 = (const float *)m->g4.p;
    d.g11 = (const float *)m->g11.p;
    d.tid = (const int4 *)m->tid.p;
    d.cell_start = (const int *)m->cell_start.p;
    d.nbr = (const int4 *)m->nbr.p;
    d.tsph = (const float4 *)m->tsph.p;
    d.inc_start = (const int *)m->inc_start.p;
    d.inc_list = (const int *)m->inc_list.p;
    d.bins = m->bins;
    d.blk0 = 0;
    d.nv = (int)m->n;
    return d;
}

// The selector's BF16 blob (mu[16], inv_sigma[16], W1[16][64], b1[64],
// W2[64][64], b2[64], W3[64][4], b3[4]) in the operand order of the fused
// inference (the byte layout of bsk::PackedNet): A-operand vectors of the
// transposed layers, with the K index k = 8h + s of k-tile kt of layers 2
// and 3 reading unit U(kt, h, s) = 32(kt/2) + 8(2(kt%2) + s/4) + 4h + s%4,
// and the biases in output-register order.
std::vector<uint8_t> pack_network(const uint16_t *blob)
{
    const uint16_t *mu = blob, *isg = blob + 16, *W1 = blob + 32, *b1 = W1 + 16 * 64, *W2 = b1 + 64,
                   *b2 = W2 + 64 * 64, *W3 = b2 + 64, *b3 = W3 + 64 * 4;
    auto f32 = [](uint16_t b) {
        const uint32_t u = (uint32_t)b << 16;
        float x;
        std::memcpy(&x, &u, 4);
        return x;
    };
    auto U = [](int kt, int h, int s) { return 32 * (kt >> 1) + 8 * (2 * (kt & 1) + (s >> 2)) + 4 * h + (s & 3); };
    std::vector<uint8_t> out((size_t)bsk::kPackedNetBytes, 0);
    uint16_t *w1 = (uint16_t *)out.data(); // [2][64][8]
    uint16_t *w2 = w1 + 2 * 64 * 8;        // [2][4][64][8]
    uint16_t *w3 = w2 + 2 * 4 * 64 * 8;    // [4][64][8]
    float *fb = (float *)(w3 + 4 * 64 * 8);
    float *fb1 = fb, *fb2 = fb + 64, *fb3 = fb + 128, *fmu = fb + 132, *fisg = fb + 148;
    for (int l = 0; l < 64; ++l)
        for (int sidx = 0; sidx < 8; ++sidx) {
            const int h = l >> 5, col = l & 31;
            for (int rt = 0; rt < 2; ++rt) {
                w1[(rt * 64 + l) * 8 + sidx] = W1[(8 * h + sidx) * 64 + 32 * rt + col];
                for (int kt = 0; kt < 4; ++kt) w2[((rt * 4 + kt) * 64 + l) * 8 + sidx] = W2[U(kt, h, sidx) * 64 + 32 * rt + col];
            }
            for (int kt = 0; kt < 4; ++kt) w3[(kt * 64 + l) * 8 + sidx] = col < 4 ? W3[U(kt, h, sidx) * 4 + col] : 0;
        }
    for (int rt = 0; rt < 2; ++rt)
        for (int h = 0; h < 2; ++h)
            for (int r = 0; r < 16; ++r) {
                const int u = 32 * rt + 8 * (r >> 2) + 4 * h + (r & 3);
                fb1[(rt * 2 + h) * 16 + r] = f32(b1[u]);
                fb2[(rt * 2 + h) * 16 + r] = f32(b2[u]);
            }
    for (int c = 0; c < 4; ++c) fb3[c] = f32(b3[c]);
    for (int k = 0; k < 16; ++k) {
        fmu[k] = f32(mu[k]);
        fisg[k] = f32(isg[k]);
    }
    return out;
}

int check_policy(const bs_policy *p)
{
    if (p->kind < BS_POLICY_FIXED || p->kind > BS_POLICY_LEARNED)
        return fail(BS_E_POLICY, "unknown policy kind %d", p->kind);
    if (p->n_phi < 1 || p->n_phi > 256 || p->n_theta < 1 || p->n_theta > 256)
        return fail(BS_E_POLICY, "angular orders must lie in [1, 256] (got %d, %d)", p->n_phi, p->n_theta);
    if (!(p->near_cut > 0) || !(p->d_g11 >= p->near_cut) || !(p->d_g4 >= p->d_g11) || !std::isfinite(p->d_g4))
        return fail(BS_E_POLICY, "cut distances must satisfy 0 < near_cut <= d_g11 <= d_g4 < inf");
    if (p->kind == BS_POLICY_GAUSS_ONLY && (p->gauss_rule < BS_RULE_G1 || p->gauss_rule > BS_RULE_G11))
        return fail(BS_E_POLICY, "gauss_rule must be BS_RULE_G1, _G4 or _G11");
    if (p->precision < BS_PREC_FP32_NAIVE || p->precision > BS_PREC_FP64)
        return fail(BS_E_POLICY, "unknown precision %d", p->precision);
    if (p->kind == BS_POLICY_LEARNED) {
        if (!p->mlp_bf16 || p->mlp_len != bsk::kMlpBlobLen)
            return fail(BS_E_POLICY, "learned policy needs a weight blob of %d values (got %lld)", bsk::kMlpBlobLen,
                        (long long)p->mlp_len);
        if (!(p->conf_min >= 0.f && p->conf_min <= 1.f)) return fail(BS_E_POLICY, "conf_min must lie in [0, 1]");
    }
    if (p->far_field != BS_FAR_ALL_PAIRS && p->far_field != BS_FAR_TREECODE)
        return fail(BS_E_POLICY, "unknown far_field %d", p->far_field);
    if (p->far_field == BS_FAR_TREECODE) {
        if (p->kind != BS_POLICY_FIXED && p->kind != BS_POLICY_LEARNED)
            return fail(BS_E_POLICY, "the treecode far field needs the FIXED or LEARNED policy");
        if (!(p->tree_theta > 0.0 && p->tree_theta < 1.0)) return fail(BS_E_POLICY, "tree_theta must lie in (0, 1)");
        if (p->tree_order != 2 && p->tree_order != 4 && p->tree_order != 6)
            return fail(BS_E_POLICY, "tree_order must be 2, 4 or 6 (got %d)", p->tree_order);
    }
    return BS_OK;
}

} // namespace

// =============================================================== public ABI
extern "C" {

void bs_policy_default(bs_policy *p)
{
    if (!p) return;
    std::memset(p, 0, sizeof *p);
    p->kind = BS_POLICY_FIXED;
    p->n_phi = 16;
    p->n_theta = 16;
    p->near_cut = 2.0;
    p->d_g11 = 4.0;
    p->d_g4 = 8.0;
    p->gauss_rule = BS_RULE_G1;
    p->precision = BS_PREC_FP32_COMP;
    p->conf_min = 0.9f;
    p->far_field = BS_FAR_ALL_PAIRS;
    p->tree_theta = 0.3;
    p->tree_order = 4;
}

const char *bs_status_string(int s)
{
    switch (s) {
    case BS_OK: return "ok";
    case BS_E_ARG: return "invalid argument";
    case BS_E_INDEX: return "node index out of range or repeated within a tetrahedron";
    case BS_E_DEGENERATE: return "zero-volume tetrahedron";
    case BS_E_NONFINITE: return "non-finite input";
    case BS_E_STATE: return "call out of order";
    case BS_E_DEVICE: return "device or runtime failure";
    case BS_E_NOMEM: return "out of memory";
    case BS_E_POLICY: return "invalid policy";
    default: return "unknown status";
    }
}

const char *bs_last_error(void) { return g_err.c_str(); }

int bs_mesh_upload(const bs_mesh_desc *d, bs_mesh **out)
{
    g_err.clear();
    if (!d || !out) return fail(BS_E_ARG, "null descriptor or output pointer");
    *out = nullptr;
    if (d->n_nodes < 1 || d->n_tets < 0) return fail(BS_E_ARG, "n_nodes must be >= 1 and n_tets >= 0");
    if (!d->xyz || !d->omega || (d->n_tets > 0 && !d->tets)) return fail(BS_E_ARG, "null input array");
    if (d->flags & ~BS_PTR_DEVICE) return fail(BS_E_ARG, "unknown flags 0x%x", d->flags);
    if (round_up_1024(d->n_nodes) > kMaxNodeSlots || d->n_tets > kMaxTets)
        return fail(BS_E_ARG, "mesh too large for 32-bit indexing (n_nodes %lld, n_tets %lld; limits %lld, %lld)",
                    (long long)d->n_nodes, (long long)d->n_tets, (long long)kMaxNodeSlots,
                    (long long)kMaxTets);
    // device inputs need the device before anything can be validated
    int dev = -1, rc;
    if ((d->flags & BS_PTR_DEVICE) && (rc = check_device(&dev))) return rc;
    bs_mesh *m = new (std::nothrow) bs_mesh();
    if (!m) return fail(BS_E_NOMEM, "host allocation");
    m->n = d->n_nodes;
    m->T = d->n_tets;
    hipStream_t s = (hipStream_t)d->stream;
    try {
        m->tets.resize((size_t)(4 * m->T));
        m->xyz.resize((size_t)(3 * m->n));
        m->omega.resize((size_t)(3 * m->n));
    } catch (...) {
        delete m;
        return fail(BS_E_NOMEM, "host allocation");
    }
    if (d->flags & BS_PTR_DEVICE) {
        hipError_t e = m->T > 0 ? hipMemcpy(m->tets.data(), d->tets, 16 * (size_t)m->T, hipMemcpyDeviceToHost)
                                : hipSuccess;
        if (e != hipSuccess) {
            delete m;
            return hip_fail(e, "read tets");
        }
    } else if (m->T > 0) {
        std::memcpy(m->tets.data(), d->tets, 16 * (size_t)m->T);
    }
    for (int64_t t = 0; t < m->T; ++t) {
        const int32_t *id = &m->tets[(size_t)(4 * t)];
        for (int j = 0; j < 4; ++j) {
            if (id[j] < 0 || id[j] >= m->n) {
                delete m;
                return fail(BS_E_INDEX, "tetrahedron %lld: node index %d outside [0, %lld)", (long long)t, id[j],
                            (long long)m->n);
            }
            for (int k = 0; k < j; ++k)
                if (id[k] == id[j]) {
                    delete m;
                    return fail(BS_E_INDEX, "tetrahedron %lld repeats node %d", (long long)t, id[j]);
                }
        }
    }
    if ((rc = read_inputs(m, d->xyz, d->omega, d->flags, s)) || (rc = validate_geometry(m))) {
        delete m;
        return rc;
    }
    build_neighbours(m);
    if (dev < 0 && (rc = check_device(&dev))) {
        delete m;
        return rc;
    }
    m->device = dev;
    // set-up of the static scratch of bs_eval_velocity_noalloc, once per
    // device (with the device current): a failed lookup only disables that
    // entry point, which then reports it
    (void)bsk::scratch_setup(dev);
    if ((rc = build_device_mesh(m, s))) {
        bs_mesh_free(m);
        return rc;
    }
    bs_policy_default(&m->pol);
    for (auto &e : m->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            bs_mesh_free(m);
            return fail(BS_E_DEVICE, "hipEventCreate");
        }
    if (hipEventCreate(&m->ev_fork) != hipSuccess) {
        bs_mesh_free(m);
        return fail(BS_E_DEVICE, "hipEventCreate");
    }
    for (auto &a : m->aux)
        if (hipStreamCreateWithFlags(&a, hipStreamNonBlocking) != hipSuccess) {
            bs_mesh_free(m);
            return fail(BS_E_DEVICE, "hipStreamCreateWithFlags");
        }
    *out = m;
    return BS_OK;
}

int bs_mesh_update(bs_mesh *m, const double *xyz, const double *omega, uint32_t flags, void *stream)
{
    g_err.clear();
    if (!m) return fail(BS_E_STATE, "null mesh");
    if (flags & ~BS_PTR_DEVICE) return fail(BS_E_ARG, "unknown flags 0x%x", flags);
    hipStream_t s = (hipStream_t)stream;
    std::vector<double> keep_x = m->xyz, keep_w = m->omega;
    int rc;
    if ((rc = read_inputs(m, xyz, omega, flags, s)) || (rc = validate_geometry(m))) {
        m->xyz.swap(keep_x);
        m->omega.swap(keep_w);
        return rc;
    }
    return build_device_mesh(m, s);
}

void bs_mesh_free(bs_mesh *m)
{
    if (!m) return;
    DBuf *bufs[] = {&m->xh, &m->xl, &m->om, &m->nrec, &m->tsph, &m->blk, &m->node_orig, &m->g1, &m->g4, &m->g11, &m->tid,
                    &m->nbr, &m->inc_start, &m->inc_list, &m->fallback,
                    &m->cell_start, &m->part, &m->band, &m->rtv, &m->vel, &m->cnt, &m->nonfinite, &m->dir,
                    &m->dir64, &m->cphi, &m->dia, &m->mlp, &m->sel, &m->torig, &m->tlist, &m->tvel,
                    &m->gvel, &m->tgrad, &m->ngrad, &m->om64, &m->srate,
                    &m->tree.nrange, &m->tree.child, &m->tree.leaves, &m->tree.c64, &m->tree.crec,
                    &m->tree.src64, &m->tree.g1t, &m->tree.tidt, &m->tree.M, &m->tree.N, &m->tree.acc_start,
                    &m->tree.acc, &m->tree.dir_start, &m->tree.dir, &m->tree.torder, &m->tree.tin, &m->tree.x64,
                    &m->tree.rank};
    for (DBuf *b : bufs) dfree(*b);
    for (PinnedBuf *b : {&m->h_g1, &m->h_g4, &m->h_g11})
        if (b->p) (void)hipHostFree(b->p);
    for (auto &a : m->aux)
        if (a) (void)hipStreamSynchronize(a);
    for (auto &e : m->ev)
        if (e) (void)hipEventDestroy(e);
    if (m->ev_fork) (void)hipEventDestroy(m->ev_fork);
    for (auto &a : m->aux)
        if (a) (void)hipStreamDestroy(a);
    delete m;
}

int bs_set_policy(bs_mesh *m, const bs_policy *p)
{
    g_err.clear();
    if (!m) return fail(BS_E_STATE, "null mesh");
    if (!p) return fail(BS_E_ARG, "null policy");
    int rc = check_policy(p);
    if (rc) return rc;
    if (p->kind == BS_POLICY_LEARNED) {
        const std::vector<uint8_t> img = pack_network(p->mlp_bf16);
        if ((rc = dalloc(m->mlp, img.size()))) return rc;
        hipError_t e = hipMemcpy(m->mlp.p, img.data(), img.size(), hipMemcpyHostToDevice);
        if (e != hipSuccess) return hip_fail(e, "upload network");
    }
    m->pol = *p;
    m->pol.mlp_bf16 = nullptr;
    // the treecode's plan for the current positions (no evaluation builds it)
    const auto &tp = m->tree;
    if (uses_treecode(m->pol) &&
        !(tp.valid && tp.theta == p->tree_theta && tp.order == p->tree_order && tp.d_g4 == p->d_g4) &&
        (rc = build_tree_plan(m, nullptr)))
        return rc;
    // the angular tables of the policy's orders, so that an evaluation never
    // has to allocate them
    return install_angular(m);
}

} // extern "C"

namespace {

// The fixed-rule far field runs on the matrix cores except in FP64 mode or
// when the vector-ALU kernel is asked for.
bool far_on_matrix_cores(const bs_mesh *m)
{
    const bs_policy &P = m->pol;
    const bool fixed_like = P.kind == BS_POLICY_FIXED || P.kind == BS_POLICY_LEARNED;
    return fixed_like && P.precision != BS_PREC_FP64 && m->far_mode == 0 && P.far_field == BS_FAR_ALL_PAIRS;
}

// Tet splits of the all-pairs Gauss kernels (0: no far-field kernel).  The
// matrix-core kernel: eight (one eighth of the tets per XCD, see
// k_far_mfma), times the number of sub-splits that keeps each split's
// 32-byte records within 3 MiB of an XCD's 4 MiB L2.  The vector-ALU kernel:
// enough waves to fill 256 CUs.
int far_splits(const bs_mesh *m)
{
    const bs_policy &P = m->pol;
    const bool gauss_all =
        P.kind == BS_POLICY_FIXED || P.kind == BS_POLICY_LEARNED || P.kind == BS_POLICY_GAUSS_ONLY;
    if (!gauss_all || m->T <= 0) return 0;
    if (uses_treecode(P)) return 2 * tree_chunks(m); // expansions, direct leaves
    const int node_blocks = m->npad / 1024;
    if (far_on_matrix_cores(m)) {
        const int base = std::max(1, std::min<int>(8, (int)((m->T + 2047) / 2048)));
        if (base < 8) return base;
        const int64_t per_xcd = 32 * ((m->T + 7) / 8);
        return 8 * (int)std::max<int64_t>(1, (per_xcd + (3 << 20) - 1) / (3 << 20));
    }
    return std::max(1, std::min<int>((int)((4096 + 4 * node_blocks - 1) / (4 * node_blocks)), (int)((m->T + 255) / 256)));
}

// Device buffers of one evaluation that the caller provides instead of the
// mesh (the no-allocation entry point): partial sums, counters, the walk's
// fallback list and the learned policy's lists, and the output.
struct EvalBufs {
    double *part, *band, *rtv, *vel;
    unsigned long long *cnt;
    int *nonfinite, *fallback, *sel;
};

// One evaluation into m->vel (device, input node order), on stream s.
// targets: the evaluation points after the nodes (bs_eval_points) instead
// of the nodes; their velocities go to m->tvel.  With given buffers (nodes
// only) nothing is allocated: the buffers come from `given`, counters are
// cleared by a kernel, every kernel runs on s and no event is recorded.
int eval_device(bs_mesh *m, hipStream_t s, bool targets, const EvalBufs *given = nullptr)
{
    int rc;
    if (given) {
        if (m->ang_N != m->pol.n_phi || m->ang_M != m->pol.n_theta)
            return fail(BS_E_STATE, "angular tables of the policy not installed");
    } else if ((rc = install_angular(m))) {
        return rc;
    }
    const bs_policy &P = m->pol;
    bsk::DevMesh dm = dev_view(m);
    if (targets) {
        dm.n = (int)m->tn;
        dm.blk0 = m->tblk0;
        dm.nblk = m->tnblk;
        dm.nv = m->t0 + (int)m->tn;
    }
    m->last_targets = targets;

    const bool fixed_like = P.kind == BS_POLICY_FIXED || P.kind == BS_POLICY_LEARNED;
    const bool far_mfma = far_on_matrix_cores(m);
    const bool treecode = uses_treecode(P);
    if (treecode && !m->tree.valid) return fail(BS_E_STATE, "treecode plan missing (set the policy again)");
    const int splits = far_splits(m);
    if (splits > 0 && !given && (rc = dalloc(m->part, 8 * 3 * (size_t)m->npad * splits))) return rc;
    double *b_part = given ? given->part : (double *)m->part.p;
    double *b_band = given ? given->band : (double *)m->band.p;
    double *b_rtv = given ? given->rtv : (double *)m->rtv.p;
    unsigned long long *cnt = given ? given->cnt : (unsigned long long *)m->cnt.p;
    int *b_nonfinite = given ? given->nonfinite : (int *)m->nonfinite.p;
    bsk::Thresholds th{};
    const double hb = m->hbar;
    const double c_rt = P.near_cut * hb, c_11 = P.d_g11 * hb, c_4 = P.d_g4 * hb;
    th.rt2 = (float)(c_rt * c_rt);
    th.g11_2 = (float)(c_11 * c_11);
    th.g4_2 = (float)(c_4 * c_4);
    th.r_band = (float)(std::max(c_4, m->max_vc) * (1.0 + 1e-4) + 1e-6);
    th.r_rt = (float)(std::max(c_rt, m->max_vc) * (1.0 + 1e-4) + 1e-6);
    th.vc = (float)(m->max_vc * (1.0 + 1e-4) + 1e-6);
    th.inc_far = m->max_vc < c_4 * (1.0 - 1e-5) ? 0 : 1;
    // the rule's binary32 distance of an incident pair exceeds max_vc by at
    // most the rounding of the coordinates and the centroid
    th.inc_band = (m->max_vc + 16.0 * std::ldexp(1.0, -24) * m->max_abs) * (1.0 + 1e-5) < c_rt ? 0 : 1;
    // relative margin on d^2 around the G4 cut: the rule's binary32 d^2 and
    // the far kernel's block-relative matrix-core d^2 differ by a few units
    // in the last place of the coordinates' magnitude relative to the cut
    {
        const double eps = 2e-4 + 256.0 * std::ldexp(1.0, -24) * (m->max_abs / std::max(c_4, 1e-300));
        if (c_4 > 0.0 && eps < 0.5) {
            th.s_g1 = (float)std::pow(c_4 * c_4 * (1.0 + eps), -1.5);
            th.s_amb = (float)std::pow(c_4 * c_4 * (1.0 - eps), -1.5);
        } else { // every band pair takes the rule's test
            th.s_g1 = 0.f;
            th.s_amb = INFINITY;
        }
    }
    bsk::AngTab ang{};
    ang.dir = (const float4 *)m->dir.p;
    ang.dir64 = (const double *)m->dir64.p;
    ang.cphi = (const float *)m->cphi.p;
    ang.dia = (const float *)m->dia.p;
    ang.N = P.n_phi;
    ang.M2 = 2 * P.n_theta;

    hipError_t e;
    if (given) {
        if ((e = bsk::launch_fill_zero(cnt, 2 * bsk::kCntWords, s)) ||
            (e = bsk::launch_fill_zero(b_nonfinite, 1, s)))
            return hip_fail(e, "clear counters");
    } else if ((e = hipMemsetAsync(cnt, 0, 8 * bsk::kCntWords, s)) || (e = hipMemsetAsync(b_nonfinite, 0, 4, s))) {
        return hip_fail(e, "clear counters");
    }
    const double *part = nullptr, *band = nullptr, *rtv = nullptr;
    const bool one_stream = m->serial || given;
    auto record = [&](int k, hipStream_t st) {
        if (!given) (void)hipEventRecord(m->ev[k], st);
    };
    record(0, s);
    // the treecode's moments first, alone: a chain of small launches (one per
    // tree level) that would otherwise wait for slots behind the band and
    // ray-tracing kernels
    const bsk::TreeView tv = treecode ? tree_view(m) : bsk::TreeView{};
    if (treecode && m->T > 0 &&
        (e = bsk::launch_tree_moments(tv, m->tree.level_start.data(), (int)m->tree.level_start.size() - 1, s)))
        return hip_fail(e, "treecode moments");
    hipEvent_t fork = m->ev[0];
    if (!one_stream && treecode) {
        fork = m->ev_fork;
        if ((e = hipEventRecord(fork, s))) return hip_fail(e, "fork event");
    }
    if (!one_stream &&
        ((e = hipStreamWaitEvent(m->aux[0], fork, 0)) || (e = hipStreamWaitEvent(m->aux[1], fork, 0))))
        return hip_fail(e, "fork streams");
    if (m->T > 0) {
        if (P.kind == BS_POLICY_GAUSS_ONLY) {
            const int pts = P.gauss_rule == BS_RULE_G1 ? 1 : P.gauss_rule == BS_RULE_G4 ? 4 : 11;
            if ((e = bsk::launch_gauss_all(dm, pts, P.precision, splits, b_part, s)))
                return hip_fail(e, "gauss kernel");
            part = b_part;
        } else if (treecode) {
            if ((e = bsk::launch_tree_far(dm, tv, th.g4_2, th.inc_far, P.precision, tree_chunks(m), b_part, s)))
                return hip_fail(e, "treecode far field");
            part = b_part;
        } else if (far_mfma) {
            if ((e = bsk::launch_far_mfma(dm, th, P.precision, splits, b_part, s)))
                return hip_fail(e, "far-field kernel");
            part = b_part;
        } else if (fixed_like) {
            if ((e = bsk::launch_gauss_all(dm, 1, P.precision, splits, b_part, s)))
                return hip_fail(e, "far-field kernel");
            part = b_part;
        }
    }
    record(1, s);
    // band and ray tracing on their own streams, concurrent with the far field
    hipStream_t sb = one_stream ? s : m->aux[0], sr = one_stream ? s : m->aux[1];
    record(2, sb);
    if (m->T > 0 && fixed_like) {
        if ((e = bsk::launch_band(dm, th, P.precision, (far_mfma || treecode) ? 0 : 1, b_band, cnt, sb)))
            return hip_fail(e, "band kernel");
        band = b_band;
    }
    record(3, sb);
    record(4, sr);
    bsk::LearnParams lp{};
    lp.net = P.kind == BS_POLICY_LEARNED ? (const bsk::PackedNet *)m->mlp.p : nullptr;
    lp.conf_min = P.conf_min;
    lp.hbar = (float)m->hbar;
    m->last_rt = 0;
    if (m->T > 0 && (fixed_like || P.kind == BS_POLICY_PURE_RT)) {
        const int all = P.kind == BS_POLICY_PURE_RT;
        m->last_rt = 1;
        // the walk on face-manifold meshes; where the boundary is not
        // convex it leaves every node with a ray that exits the mesh early
        // to the candidate kernel (with every pair ray traced, rays run to
        // the boundary: there every node goes to the candidate kernel)
        if (m->manifold && (m->convex || !all) && m->rt_mode == 0 && !targets) {
            m->last_rt = 2;
            if (!given && (rc = dalloc(m->fallback, 4 * ((size_t)m->n + 1)))) return rc;
            int *fb = given ? given->fallback : (int *)m->fallback.p;
            int *nfb = fb + m->n;
            const float r_stop = all ? 3.0e38f : (float)((std::max(c_rt, m->max_vc) + m->max_vc) * (1.0 + 1e-4) + 1e-6);
            int *sel_list = nullptr, *sel_n = nullptr, *sel_cnt = nullptr;
            float *sel_dmax = nullptr;
            if (lp.net) {
                const size_t nn = (size_t)m->n;
                if (!given && (rc = dalloc(m->sel, 4 * (nn * bsk::kSelListCap + 5 * nn)))) return rc;
                sel_list = given ? given->sel : (int *)m->sel.p;
                sel_n = sel_list + nn * bsk::kSelListCap;
                sel_dmax = (float *)(sel_n + nn);
                sel_cnt = (int *)(sel_dmax + nn);
            }
            if ((e = given ? bsk::launch_fill_zero(nfb, 1, sr) : hipMemsetAsync(nfb, 0, 4, sr)) ||
                (lp.net && (e = bsk::launch_select(dm, th, lp, P.precision, b_rtv, sel_list, sel_n, sel_dmax,
                                                   sel_cnt, sr))) ||
                (e = bsk::launch_rt_walk(dm, th, ang, all, r_stop, m->convex ? 0 : 1, P.precision, b_rtv, cnt, fb,
                                         nfb, sel_list, sel_n, sel_dmax, sel_cnt, sr)) ||
                (e = bsk::launch_rt(dm, th, ang, lp, all, P.precision, b_rtv, cnt, fb, nfb, sr)))
                return hip_fail(e, "ray-tracing walk");
        } else if ((e = bsk::launch_rt(dm, th, ang, lp, all, P.precision, b_rtv, cnt,
                                       targets ? (const int *)m->tlist.p : nullptr,
                                       targets ? (const int *)m->tlist.p + m->tn : nullptr, sr))) {
            return hip_fail(e, "ray-tracing kernel");
        }
        rtv = b_rtv;
    }
    if (given) m->last_rt = 0; // (no statistics are read after a call that allocates nothing)
    record(5, sr);
    if (!one_stream && ((e = hipStreamWaitEvent(s, m->ev[3], 0)) || (e = hipStreamWaitEvent(s, m->ev[5], 0))))
        return hip_fail(e, "join streams");
    record(6, s);
    double *out = given ? given->vel : (double *)(targets ? m->tvel.p : m->vel.p);
    if ((e = bsk::launch_combine(dm, (const int *)(targets ? m->torig.p : m->node_orig.p), part, part ? splits : 0,
                                 band, rtv, out, b_nonfinite, s)))
        return hip_fail(e, "combine kernel");
    record(7, s);
    if (!targets) m->vel_valid = !given;
    return BS_OK;
}

// Bytes of scratch an evaluation of the nodes needs under the current
// policy and far-field mode, laid out (256-byte aligned) as part, band, rtv,
// counters, non-finite flag, fallback list, learned lists; offsets in off[7].
size_t eval_scratch_layout(const bs_mesh *m, size_t off[7])
{
    auto al = [](size_t v) { return (v + 255) / 256 * 256; };
    const size_t np = (size_t)m->npad, nn = (size_t)m->n;
    const size_t sz[7] = {8 * 3 * np * (size_t)far_splits(m), 8 * 3 * np, 8 * 3 * np, 8 * (size_t)bsk::kCntWords, 4,
                          4 * (nn + 1),
                          m->pol.kind == BS_POLICY_LEARNED ? 4 * (nn * bsk::kSelListCap + 5 * nn) : 0};
    size_t o = 0;
    for (int k = 0; k < 7; ++k) {
        off[k] = o;
        o += al(sz[k]);
    }
    return o;
}

int read_stats(bs_mesh *m, bs_stats *st)
{
    std::vector<unsigned long long> cc((size_t)bsk::kCntWords);
    int nf = 0;
    hipError_t e;
    if ((e = hipMemcpy(cc.data(), m->cnt.p, 8 * cc.size(), hipMemcpyDeviceToHost)) ||
        (e = hipMemcpy(&nf, m->nonfinite.p, 4, hipMemcpyDeviceToHost)))
        return hip_fail(e, "read counters");
    unsigned long long c[bsk::kNumCounters] = {};
    for (int k = 0; k < bsk::kCntStripes; ++k)
        for (int j = 0; j < bsk::kNumCounters; ++j) c[j] += cc[(size_t)(k * bsk::kCntStride + j)];
    const bs_policy &P = m->pol;
    std::memset(st, 0, sizeof *st);
    float ms = 0.f;
    (void)hipEventElapsedTime(&ms, m->ev[0], m->ev[7]);
    st->t_eval_s = ms * 1e-3;
    for (int k = 0; k < 4; ++k) {
        float mk = 0.f;
        (void)hipEventElapsedTime(&mk, m->ev[2 * k], m->ev[2 * k + 1]);
        st->t_kernel_s[k] = mk * 1e-3;
    }
    st->pairs = (m->last_targets ? m->tn : m->n) * m->T;
    if (P.kind == BS_POLICY_FIXED || P.kind == BS_POLICY_LEARNED) {
        // c[2] counts the pairs actually ray traced; the learned selector's
        // moves out of the ray-traced band are c[5..7]
        st->pairs_by_rule[BS_RULE_G4] = (int64_t)(c[0] + c[6]);
        st->pairs_by_rule[BS_RULE_G11] = (int64_t)(c[1] + c[7]);
        st->pairs_by_rule[BS_RULE_RT] = (int64_t)c[2];
        st->pairs_by_rule[BS_RULE_G1] = st->pairs - st->pairs_by_rule[BS_RULE_G4] - st->pairs_by_rule[BS_RULE_G11] -
                                        st->pairs_by_rule[BS_RULE_RT];
    } else if (P.kind == BS_POLICY_PURE_RT) {
        st->pairs_by_rule[BS_RULE_RT] = st->pairs;
    } else {
        st->pairs_by_rule[P.gauss_rule] = st->pairs;
    }
    st->rt_hit_lines = (int64_t)c[3];
    st->fp64_retests = (int64_t)c[4];
    st->reoriented = m->reoriented;
    st->nonfinite_out = nf;
    st->hbar = m->hbar;
    const int64_t nt = m->last_targets ? m->tn : m->n;
    if (m->last_rt == 2) {
        int nfb = 0;
        if ((e = hipMemcpy(&nfb, (const int *)m->fallback.p + m->n, 4, hipMemcpyDeviceToHost)))
            return hip_fail(e, "read counters");
        st->rt_candidate_nodes = nfb;
        st->rt_walk_nodes = nt - nfb;
    } else if (m->last_rt == 1) {
        st->rt_candidate_nodes = nt;
    }
    if (uses_treecode(P) && m->tree.valid) {
        st->tree_expansions = m->last_targets ? m->tree.exp_pts : m->tree.exp_nodes;
        st->tree_direct = m->last_targets ? m->tree.dir_pts : m->tree.dir_nodes;
        st->tree_covered = m->last_targets ? m->tree.cov_pts : m->tree.cov_nodes;
    }
    return BS_OK;
}

// Nodal velocity gradient into m->ngrad ([n][3][3] FP64, input order) from
// device velocities vel ([n][3], input order).
int velocity_gradient_device(bs_mesh *m, const double *vel, hipStream_t s)
{
    int rc;
    if ((rc = dalloc(m->tgrad, 8 * 10 * (size_t)std::max<int64_t>(m->T, 1))) ||
        (rc = dalloc(m->ngrad, 8 * 9 * (size_t)std::max<int64_t>(m->n, 1))))
        return rc;
    const bsk::DevMesh dm = dev_view(m);
    hipError_t e = bsk::launch_velocity_gradient(dm, (const int *)m->node_orig.p, vel, (double *)m->tgrad.p,
                                                 (double *)m->ngrad.p, s);
    if (e != hipSuccess) return hip_fail(e, "velocity gradient kernels");
    return BS_OK;
}

// Stretching rate G omega of every node into m->srate ([n][3] FP64, input
// order) from device velocities vel ([n][3], input order) and the mesh's
// current vorticity.
int stretching_device(bs_mesh *m, const double *vel, hipStream_t s)
{
    int rc = velocity_gradient_device(m, vel, s);
    if (rc || (rc = dalloc(m->srate, 8 * 3 * (size_t)std::max<int64_t>(m->n, 1)))) return rc;
    const hipError_t e = bsk::launch_stretching((int)m->n, (const double *)m->ngrad.p, (const double *)m->om64.p,
                                                (double *)m->srate.p, s);
    if (e != hipSuccess) return hip_fail(e, "stretching kernel");
    return BS_OK;
}

} // namespace

extern "C" {

int bs_velocity_gradient(bs_mesh *m, const double *vel, double *grad, uint32_t flags, void *stream)
{
    g_err.clear();
    if (!m) return fail(BS_E_STATE, "null mesh");
    if (!grad) return fail(BS_E_ARG, "null output");
    if (flags & ~BS_PTR_DEVICE) return fail(BS_E_ARG, "unknown flags 0x%x", flags);
    if (!vel && !m->vel_valid) return fail(BS_E_STATE, "no velocities: evaluate the nodes first or pass vel");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    const size_t n3 = 3 * (size_t)m->n;
    const double *dvel = (const double *)m->vel.p;
    if (vel) {
        if (flags & BS_PTR_DEVICE) {
            dvel = vel;
        } else {
            for (size_t i = 0; i < n3; ++i)
                if (!std::isfinite(vel[i])) return fail(BS_E_NONFINITE, "non-finite velocity");
            int rc = dalloc(m->gvel, 8 * std::max<size_t>(n3, 1));
            if (rc) return rc;
            if ((e = hipMemcpyAsync(m->gvel.p, vel, 8 * n3, hipMemcpyHostToDevice, s)) ||
                (e = hipStreamSynchronize(s)))
                return hip_fail(e, "upload velocities");
            dvel = (const double *)m->gvel.p;
        }
    }
    if (m->n == 0) return BS_OK;
    int rc = velocity_gradient_device(m, dvel, s);
    if (rc) return rc;
    if ((e = hipMemcpyAsync(grad, m->ngrad.p, 8 * 9 * (size_t)m->n,
                            (flags & BS_PTR_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s)) ||
        (e = hipStreamSynchronize(s)))
        return hip_fail(e, "velocity gradient");
    return BS_OK;
}

int bs_stretching_rate(bs_mesh *m, const double *vel, double *rate, uint32_t flags, void *stream)
{
    g_err.clear();
    if (!m) return fail(BS_E_STATE, "null mesh");
    if (!rate) return fail(BS_E_ARG, "null output");
    if (flags & ~BS_PTR_DEVICE) return fail(BS_E_ARG, "unknown flags 0x%x", flags);
    if (!vel && !m->vel_valid) return fail(BS_E_STATE, "no velocities: evaluate the nodes first or pass vel");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    const size_t n3 = 3 * (size_t)m->n;
    const double *dvel = (const double *)m->vel.p;
    if (vel) {
        if (flags & BS_PTR_DEVICE) {
            dvel = vel;
        } else {
            for (size_t i = 0; i < n3; ++i)
                if (!std::isfinite(vel[i])) return fail(BS_E_NONFINITE, "non-finite velocity");
            int rc = dalloc(m->gvel, 8 * std::max<size_t>(n3, 1));
            if (rc) return rc;
            if ((e = hipMemcpyAsync(m->gvel.p, vel, 8 * n3, hipMemcpyHostToDevice, s)) ||
                (e = hipStreamSynchronize(s)))
                return hip_fail(e, "upload velocities");
            dvel = (const double *)m->gvel.p;
        }
    }
    if (m->n == 0) return BS_OK;
    int rc = stretching_device(m, dvel, s);
    if (rc) return rc;
    if ((e = hipMemcpyAsync(rate, m->srate.p, 8 * n3,
                            (flags & BS_PTR_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s)) ||
        (e = hipStreamSynchronize(s)))
        return hip_fail(e, "stretching rate");
    return BS_OK;
}

int bs_mesh_read(bs_mesh *m, double *xyz, double *omega, uint32_t flags, void *stream)
{
    g_err.clear();
    if (!m) return fail(BS_E_STATE, "null mesh");
    if (flags & ~BS_PTR_DEVICE) return fail(BS_E_ARG, "unknown flags 0x%x", flags);
    const size_t bytes = 8 * 3 * (size_t)m->n;
    if (flags & BS_PTR_DEVICE) {
        hipStream_t s = (hipStream_t)stream;
        hipError_t e = hipSuccess;
        if (xyz && bytes) e = hipMemcpyAsync(xyz, m->xyz.data(), bytes, hipMemcpyHostToDevice, s);
        if (e == hipSuccess && omega && bytes)
            e = hipMemcpyAsync(omega, m->omega.data(), bytes, hipMemcpyHostToDevice, s);
        if (e == hipSuccess) e = hipStreamSynchronize(s);
        if (e != hipSuccess) return hip_fail(e, "copy mesh state");
    } else {
        if (xyz && bytes) std::memcpy(xyz, m->xyz.data(), bytes);
        if (omega && bytes) std::memcpy(omega, m->omega.data(), bytes);
    }
    return BS_OK;
}

int bs_eval_velocity(bs_mesh *m, double *vel, uint32_t vel_flags, void *stream, bs_stats *st)
{
    g_err.clear();
    if (!m) return fail(BS_E_STATE, "null mesh");
    if (!vel) return fail(BS_E_ARG, "null output");
    if (vel_flags & ~(BS_PTR_DEVICE | BS_EVAL_VALU_FAR | BS_EVAL_SERIAL))
        return fail(BS_E_ARG, "unknown flags 0x%x", vel_flags);
    hipStream_t s = (hipStream_t)stream;
    m->far_mode = (vel_flags & BS_EVAL_VALU_FAR) ? 1 : 0;
    m->serial = (vel_flags & BS_EVAL_SERIAL) ? 1 : 0;
    int rc = eval_device(m, s, false);
    m->far_mode = 0;
    m->serial = 0;
    if (rc) return rc;
    hipError_t e;
    const size_t vbytes = 8 * 3 * (size_t)m->n;
    e = hipMemcpyAsync(vel, m->vel.p, vbytes, (vel_flags & BS_PTR_DEVICE) ? hipMemcpyDeviceToDevice
                                                                          : hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "copy velocity");
    if (!(vel_flags & BS_PTR_DEVICE) || st) {
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "evaluation");
    }
    if (st && (rc = read_stats(m, st))) return rc;
    return BS_OK;
}

int bs_eval_velocity_noalloc(bs_mesh *m, double *vel, uint32_t flags, void *stream)
{
    g_err.clear();
    if (!m) return fail(BS_E_STATE, "null mesh");
    if (!vel) return fail(BS_E_ARG, "null output");
    if (flags & ~(BS_PTR_DEVICE | BS_EVAL_VALU_FAR)) return fail(BS_E_ARG, "unknown flags 0x%x", flags);
    if (!(flags & BS_PTR_DEVICE)) return fail(BS_E_ARG, "the output must be device memory (BS_PTR_DEVICE)");
    char *base = (char *)bsk::scratch_ptr(m->device);
    if (!base) return fail(BS_E_DEVICE, "the static scratch of device %d is not available", m->device);
    m->far_mode = (flags & BS_EVAL_VALU_FAR) ? 1 : 0;
    size_t off[7];
    const size_t need = eval_scratch_layout(m, off);
    if (need > bsk::kScratchBytes) {
        m->far_mode = 0;
        return fail(BS_E_ARG, "this mesh and policy need %zu bytes of scratch, above the static %zu", need,
                    bsk::kScratchBytes);
    }
    EvalBufs g{};
    g.part = (double *)(base + off[0]);
    g.band = (double *)(base + off[1]);
    g.rtv = (double *)(base + off[2]);
    g.cnt = (unsigned long long *)(base + off[3]);
    g.nonfinite = (int *)(base + off[4]);
    g.fallback = (int *)(base + off[5]);
    g.sel = m->pol.kind == BS_POLICY_LEARNED ? (int *)(base + off[6]) : nullptr;
    g.vel = vel;
    const int rc = eval_device(m, (hipStream_t)stream, false, &g);
    m->far_mode = 0;
    return rc;
}

int bs_eval_points(bs_mesh *m, int64_t n_pts, const double *pts, double *vel, uint32_t flags, void *stream,
                   bs_stats *st)
{
    g_err.clear();
    if (!m) return fail(BS_E_STATE, "null mesh");
    if (n_pts < 0 || (n_pts > 0 && (!pts || !vel))) return fail(BS_E_ARG, "n_pts < 0 or null pointer");
    if (n_pts > (int64_t)1 << 28 || round_up_1024(m->n) + n_pts > kMaxNodeSlots)
        return fail(BS_E_ARG, "too many points (%lld beside %lld nodes)", (long long)n_pts, (long long)m->n);
    if (flags & ~(BS_PTR_DEVICE | BS_EVAL_VALU_FAR | BS_EVAL_SERIAL)) return fail(BS_E_ARG, "unknown flags 0x%x", flags);
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    std::vector<double> p((size_t)3 * n_pts);
    if (n_pts > 0) {
        if (flags & BS_PTR_DEVICE) {
            if ((e = hipMemcpyAsync(p.data(), pts, 8 * p.size(), hipMemcpyDeviceToHost, s)) ||
                (e = hipStreamSynchronize(s)))
                return hip_fail(e, "read points");
        } else {
            std::memcpy(p.data(), pts, 8 * p.size());
        }
    }
    for (double v : p)
        if (!std::isfinite(v)) return fail(BS_E_NONFINITE, "non-finite point coordinate");
    int rc;
    if (p != m->tgt) {
        // the points join the node arrays after the nodes (one re-upload)
        m->tgt.swap(p);
        m->tn = n_pts;
        if ((rc = build_device_mesh(m, s))) return rc;
    }
    if (n_pts == 0) {
        if (st) std::memset(st, 0, sizeof *st);
        return BS_OK;
    }
    m->far_mode = (flags & BS_EVAL_VALU_FAR) ? 1 : 0;
    m->serial = (flags & BS_EVAL_SERIAL) ? 1 : 0;
    rc = eval_device(m, s, true);
    m->far_mode = 0;
    m->serial = 0;
    if (rc) return rc;
    e = hipMemcpyAsync(vel, m->tvel.p, 8 * 3 * (size_t)n_pts,
                       (flags & BS_PTR_DEVICE) ? hipMemcpyDeviceToDevice : hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return hip_fail(e, "copy velocity");
    if (!(flags & BS_PTR_DEVICE) || st) {
        if ((e = hipStreamSynchronize(s)) != hipSuccess) return hip_fail(e, "evaluation");
    }
    if (st && (rc = read_stats(m, st))) return rc;
    return BS_OK;
}

int bs_advect_heun(bs_mesh *m, double dt, int steps, double *xyz_out, uint32_t flags, void *stream,
                   double *step_seconds, bs_stats *st)
{
    g_err.clear();
    if (!m) return fail(BS_E_STATE, "null mesh");
    if (steps < 0 || !std::isfinite(dt)) return fail(BS_E_ARG, "steps must be >= 0 and dt finite");
    if (flags & ~(BS_PTR_DEVICE | BS_ADVECT_STRETCH)) return fail(BS_E_ARG, "unknown flags 0x%x", flags);
    const bool stretch = (flags & BS_ADVECT_STRETCH) != 0;
    hipStream_t s = (hipStream_t)stream;
    const size_t n3 = 3 * (size_t)m->n;
    std::vector<double> x = m->xyz, v1(n3), v2(n3), xs(n3);
    std::vector<double> w = m->omega, s1, s2, ws;
    if (stretch) {
        s1.resize(n3);
        s2.resize(n3);
        ws.resize(n3);
    }
    double t_dev = 0.0;
    int rc = BS_OK;
    hipError_t e;
    auto eval_to = [&](std::vector<double> &v) -> int {
        int r = eval_device(m, s, false);
        if (r) return r;
        if ((e = hipMemcpyAsync(v.data(), m->vel.p, 8 * n3, hipMemcpyDeviceToHost, s)) ||
            (e = hipStreamSynchronize(s)))
            return hip_fail(e, "read velocity");
        float ms = 0.f;
        (void)hipEventElapsedTime(&ms, m->ev[0], m->ev[7]);
        t_dev += ms * 1e-3;
        return BS_OK;
    };
    // vortex stretching (w . grad) v at every node, from the velocities just
    // evaluated (the gradient of their piecewise-linear interpolant)
    auto stretch_to = [&](std::vector<double> &out) -> int {
        int r = stretching_device(m, (const double *)m->vel.p, s);
        if (r) return r;
        if ((e = hipMemcpyAsync(out.data(), m->srate.p, 8 * n3, hipMemcpyDeviceToHost, s)) ||
            (e = hipStreamSynchronize(s)))
            return hip_fail(e, "read stretching rate");
        return BS_OK;
    };
    auto move_to = [&](const std::vector<double> &pos, const std::vector<double> &om) -> int {
        m->xyz = pos;
        m->omega = om;
        for (double o : om)
            if (!std::isfinite(o)) return fail(BS_E_NONFINITE, "non-finite vorticity");
        int r = validate_geometry(m);
        if (r) return r;
        return build_device_mesh(m, s);
    };
    for (int k = 0; k < steps && rc == BS_OK; ++k) {
        const auto t0 = std::chrono::steady_clock::now();
        const std::vector<double> x0 = x, w0 = w;
        if ((rc = eval_to(v1)) == BS_OK && (!stretch || (rc = stretch_to(s1)) == BS_OK)) {
            for (size_t i = 0; i < n3; ++i) xs[i] = x[i] + dt * v1[i];
            if (stretch)
                for (size_t i = 0; i < n3; ++i) ws[i] = w[i] + dt * s1[i];
            if ((rc = move_to(xs, stretch ? ws : w)) == BS_OK && (rc = eval_to(v2)) == BS_OK &&
                (!stretch || (rc = stretch_to(s2)) == BS_OK)) {
                for (size_t i = 0; i < n3; ++i) x[i] = x[i] + 0.5 * dt * (v1[i] + v2[i]);
                if (stretch)
                    for (size_t i = 0; i < n3; ++i) w[i] = w[i] + 0.5 * dt * (s1[i] + s2[i]);
                rc = move_to(x, w);
            }
        }
        if (rc) {
            // leave the mesh at the start of the failing step
            const std::string why = g_err;
            m->xyz = x0;
            m->omega = w0;
            if (validate_geometry(m) == BS_OK) build_device_mesh(m, s);
            g_err = why;
            return rc;
        }
        if (step_seconds)
            step_seconds[k] = std::chrono::duration<double>(std::chrono::steady_clock::now() - t0).count();
    }
    if (xyz_out) {
        if (flags & BS_PTR_DEVICE) {
            if ((e = hipMemcpyAsync(xyz_out, x.data(), 8 * n3, hipMemcpyHostToDevice, s)) ||
                (e = hipStreamSynchronize(s)))
                return hip_fail(e, "write positions");
        } else {
            std::memcpy(xyz_out, x.data(), 8 * n3);
        }
    }
    if (st) {
        if ((rc = read_stats(m, st))) return rc;
        st->t_eval_s = t_dev;
    }
    return BS_OK;
}

} // extern "C"

// =============================================================== rule selector
namespace {

// binary32 rule decision on the host, identical to the kernels' (no FMA:
// this file is built without contraction)
int host_rule(const float *x, const float *c, bool inc, float rt2, float g11_2, float g4_2)
{
    const float dx = x[0] - c[0], dy = x[1] - c[1], dz = x[2] - c[2];
    const float sx = dx * dx, sy = dy * dy, sz = dz * dz;
    const float d2 = (sx + sy) + sz;
    int rule = d2 < g4_2 ? BS_RULE_G4 : BS_RULE_G1;
    rule = d2 < g11_2 ? BS_RULE_G11 : rule;
    return (inc || d2 < rt2) ? BS_RULE_RT : rule;
}

void thresholds(const bs_mesh *m, float *rt2, float *g11_2, float *g4_2)
{
    const double hb = m->hbar;
    const double c_rt = m->pol.near_cut * hb, c_11 = m->pol.d_g11 * hb, c_4 = m->pol.d_g4 * hb;
    *rt2 = (float)(c_rt * c_rt);
    *g11_2 = (float)(c_11 * c_11);
    *g4_2 = (float)(c_4 * c_4);
}

uint64_t splitmix(uint64_t &s)
{
    uint64_t z = (s += 0x9e3779b97f4a7c15ull);
    z = (z ^ (z >> 30)) * 0xbf58476d1ce4e5b9ull;
    z = (z ^ (z >> 27)) * 0x94d049bb133111ebull;
    return z ^ (z >> 31);
}

double uniform01(uint64_t &s) { return (double)(splitmix(s) >> 11) * (1.0 / 9007199254740992.0); }

// collapsed Gauss rule on the reference triangle: (u, v, weight), q x q points
std::vector<double> triangle_rule(int q)
{
    std::vector<double> t, w;
    gauss_legendre(q, t, w);
    std::vector<double> out;
    for (int i = 0; i < q; ++i)
        for (int j = 0; j < q; ++j) {
            const double a = 0.5 * (t[(size_t)i] + 1.0), b = 0.5 * (t[(size_t)j] + 1.0);
            out.push_back(a * (1.0 - b));
            out.push_back(a * b);
            out.push_back(0.25 * w[(size_t)i] * w[(size_t)j] * a);
        }
    return out;
}

} // namespace

extern "C" {

int bs_learn_sample_pairs(bs_mesh *m, int64_t max_pairs, uint64_t seed, int32_t *pairs, int64_t *n_out)
{
    g_err.clear();
    if (!m) return fail(BS_E_STATE, "null mesh");
    if (!pairs || !n_out || max_pairs < 0) return fail(BS_E_ARG, "null output or negative count");
    float rt2, g11_2, g4_2;
    thresholds(m, &rt2, &g11_2, &g4_2);
    const double R = std::max(std::sqrt((double)rt2), m->max_vc) * (1.0 + 1e-4) + 1e-6;
    std::vector<int32_t> nodes((size_t)m->n);
    for (int64_t i = 0; i < m->n; ++i) nodes[(size_t)i] = (int32_t)i;
    uint64_t st = seed;
    int64_t k = 0;
    const bsk::Bins &b = m->bins;
    for (int64_t a = 0; a < m->n && k < max_pairs; ++a) {
        // draw the next node without replacement
        const int64_t j = a + (int64_t)(uniform01(st) * (double)(m->n - a));
        std::swap(nodes[(size_t)a], nodes[(size_t)std::min(j, m->n - 1)]);
        const int32_t i = nodes[(size_t)a];
        const float *x = &m->h_xh[3 * (size_t)i];
        int lo[3], hi[3];
        for (int c = 0; c < 3; ++c) {
            lo[c] = std::max(0, (int)std::floor((x[c] - R - b.lo[c]) / b.cs));
            hi[c] = std::min(b.dim[c] - 1, (int)std::floor((x[c] + R - b.lo[c]) / b.cs));
        }
        for (int iz = lo[2]; iz <= hi[2]; ++iz)
            for (int iy = lo[1]; iy <= hi[1]; ++iy) {
                const int row = (iz * b.dim[1] + iy) * b.dim[0];
                for (int32_t s = m->h_cell_start[(size_t)(row + lo[0])];
                     s < m->h_cell_start[(size_t)(row + hi[0] + 1)] && k < max_pairs; ++s) {
                    const int32_t t = m->h_order[(size_t)s];
                    const int32_t *id = &m->tets[4 * (size_t)t];
                    const bool inc = id[0] == i || id[1] == i || id[2] == i || id[3] == i;
                    if (inc) continue;
                    if (host_rule(x, &m->h_cen32[3 * (size_t)t], false, rt2, g11_2, g4_2) != BS_RULE_RT) continue;
                    pairs[2 * k] = i;
                    pairs[2 * k + 1] = t;
                    ++k;
                }
            }
    }
    *n_out = k;
    return BS_OK;
}

int bs_learn_pairs(bs_mesh *m, const int32_t *pairs, int64_t n, double tau, float *feats, int8_t *labels,
                   float *errs, void *stream)
{
    g_err.clear();
    if (!m) return fail(BS_E_STATE, "null mesh");
    if (n < 0 || (n > 0 && (!pairs || !feats || !labels || !errs))) return fail(BS_E_ARG, "null array");
    if (n > (int64_t)1 << 30) return fail(BS_E_ARG, "too many pairs");
    if (!(tau >= 0)) return fail(BS_E_ARG, "tau must be >= 0");
    hipStream_t s = (hipStream_t)stream;
    std::vector<int2> pr((size_t)n);
    // input numbering -> sorted node rank and sorted tet slot
    std::vector<int32_t> slot((size_t)m->T);
    for (int64_t k = 0; k < m->T; ++k) slot[(size_t)m->h_order[(size_t)k]] = (int32_t)k;
    for (int64_t k = 0; k < n; ++k) {
        const int32_t i = pairs[2 * k], t = pairs[2 * k + 1];
        if (i < 0 || i >= m->n || t < 0 || t >= m->T) return fail(BS_E_INDEX, "pair %lld out of range", (long long)k);
        pr[(size_t)k] = make_int2(m->h_rank[(size_t)i], slot[(size_t)t]);
    }
    const std::vector<double> tri = triangle_rule(24);
    std::vector<float> rules(80, 0.f);
    {
        int q = 0;
        for (int k : {1, 4, 11}) {
            const TetRule r = tet_rule(k);
            for (int p = 0; p < r.n; ++p, ++q) {
                for (int j = 0; j < 4; ++j) rules[(size_t)(4 * q + j)] = (float)r.lam[p][j];
                rules[(size_t)(64 + q)] = (float)r.w[p];
            }
        }
    }
    DBuf dpr, dtri, drules;
    int rc;
    if ((rc = dalloc(dpr, sizeof(int2) * (size_t)std::max<int64_t>(n, 1))) ||
        (rc = dalloc(dtri, 8 * tri.size())) || (rc = dalloc(drules, 4 * rules.size())))
        return rc;
    hipError_t e;
    if ((n > 0 && (e = hipMemcpyAsync(dpr.p, pr.data(), sizeof(int2) * (size_t)n, hipMemcpyHostToDevice, s))) ||
        (e = hipMemcpyAsync(dtri.p, tri.data(), 8 * tri.size(), hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(drules.p, rules.data(), 4 * rules.size(), hipMemcpyHostToDevice, s)) ||
        (e = bsk::launch_label(dev_view(m), (const int2 *)dpr.p, (int)n, (float)m->hbar, (const double *)dtri.p,
                               (int)(tri.size() / 3), (const float *)drules.p, tau, feats, labels, errs, s)) ||
        (e = hipStreamSynchronize(s))) {
        dfree(dpr);
        dfree(dtri);
        dfree(drules);
        return hip_fail(e, "label kernel");
    }
    dfree(dpr);
    dfree(dtri);
    dfree(drules);
    return BS_OK;
}

static uint16_t f32_to_bf16(float f)
{
    uint32_t u;
    std::memcpy(&u, &f, 4);
    const uint32_t lsb = (u >> 16) & 1u;
    u += 0x7fffu + lsb;
    return (uint16_t)(u >> 16);
}

static float bf16_to_f32(uint16_t h)
{
    const uint32_t u = (uint32_t)h << 16;
    float f;
    std::memcpy(&f, &u, 4);
    return f;
}

// shared scratch of the training entry points
struct TrainBufs {
    DBuf wb, master, m1, m2, gpart, wpart, lpart, cw, index, gout, lsum;
    ~TrainBufs()
    {
        for (DBuf *b : {&wb, &master, &m1, &m2, &gpart, &wpart, &lpart, &cw, &index, &gout, &lsum}) dfree(*b);
    }
};

int bs_mlp_grad(const uint16_t *blob, const float *feats, const int8_t *labels, int64_t n, const float *class_w,
                float *loss, float *grads, void *stream)
{
    g_err.clear();
    if (!blob || !feats || !labels || !class_w || !grads || n <= 0 || n > (1 << 26))
        return fail(BS_E_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    const int nb = (int)((n + 63) / 64);
    TrainBufs B;
    int rc;
    if ((rc = dalloc(B.wb, 2 * bsk::kMlpBlobLen)) || (rc = dalloc(B.gpart, 4 * (size_t)nb * bsk::kMlpGradLen)) ||
        (rc = dalloc(B.wpart, 4 * (size_t)nb)) || (rc = dalloc(B.lpart, 4 * (size_t)nb)) ||
        (rc = dalloc(B.cw, 16)) || (rc = dalloc(B.gout, 4 * bsk::kMlpGradLen)) || (rc = dalloc(B.lsum, 16)) ||
        (rc = dalloc(B.master, 4 * bsk::kMlpGradLen)) || (rc = dalloc(B.m1, 4 * bsk::kMlpGradLen)) ||
        (rc = dalloc(B.m2, 4 * bsk::kMlpGradLen)))
        return rc;
    hipError_t e;
    double sums[2] = {0, 0};
    if ((e = hipMemcpyAsync(B.wb.p, blob, 2 * bsk::kMlpBlobLen, hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(B.cw.p, class_w, 16, hipMemcpyHostToDevice, s)) ||
        (e = bsk::launch_mlp_grad_step(feats, labels, nullptr, (int)n, (__bf16 *)B.wb.p, (const float *)B.cw.p,
                                       (float *)B.gpart.p, (float *)B.wpart.p, (float *)B.lpart.p,
                                       (float *)B.master.p, (float *)B.m1.p, (float *)B.m2.p, 0.f, 0.9f, 0.999f,
                                       1e-8f, 1, (float *)B.gout.p, s)) ||
        (e = bsk::launch_sum_f((const float *)B.lpart.p, nb, (double *)B.lsum.p, s)) ||
        (e = bsk::launch_sum_f((const float *)B.wpart.p, nb, (double *)B.lsum.p + 1, s)) ||
        (e = hipMemcpyAsync(grads, B.gout.p, 4 * bsk::kMlpGradLen, hipMemcpyDeviceToHost, s)) ||
        (e = hipMemcpyAsync(sums, B.lsum.p, 16, hipMemcpyDeviceToHost, s)) || (e = hipStreamSynchronize(s)))
        return hip_fail(e, "gradient kernels");
    if (loss) *loss = (float)(sums[1] > 0 ? sums[0] / sums[1] : 0.0);
    return BS_OK;
}

int bs_mlp_train(const float *feats, const int8_t *labels, int64_t n, const bs_train_cfg *cfg, uint16_t *blob,
                 float *epoch_loss, void *stream)
{
    g_err.clear();
    if (!feats || !labels || !cfg || !blob || n <= 0 || n > (1 << 28) || cfg->epochs < 0 || cfg->batch < 64 ||
        cfg->batch % 64)
        return fail(BS_E_ARG, "bad arguments (batch must be a positive multiple of 64)");
    hipStream_t s = (hipStream_t)stream;
    hipError_t e;
    // feature standardisation from the training set (FP64 on the host)
    std::vector<float> hf((size_t)n * 16);
    if ((e = hipMemcpy(hf.data(), feats, 4 * hf.size(), hipMemcpyDeviceToHost)))
        return hip_fail(e, "read features");
    double mu[16] = {0}, var[16] = {0};
    for (int64_t i = 0; i < n; ++i)
        for (int q = 0; q < 16; ++q) mu[q] += hf[(size_t)i * 16 + q];
    for (int q = 0; q < 16; ++q) mu[q] /= (double)n;
    for (int64_t i = 0; i < n; ++i)
        for (int q = 0; q < 16; ++q) {
            const double d = hf[(size_t)i * 16 + q] - mu[q];
            var[q] += d * d;
        }
    std::vector<uint16_t> wb(bsk::kMlpBlobLen);
    for (int q = 0; q < 16; ++q) {
        const double sd = std::sqrt(var[q] / (double)n);
        wb[(size_t)q] = f32_to_bf16((float)mu[q]);
        wb[(size_t)(16 + q)] = f32_to_bf16(sd > 1e-6 ? (float)(1.0 / sd) : 0.f);
    }
    // He initialisation (Box-Muller on splitmix64), zero biases
    std::vector<float> master(bsk::kMlpGradLen, 0.f);
    uint64_t st = cfg->seed;
    auto gauss = [&]() {
        const double u1 = std::max(uniform01(st), 1e-300), u2 = uniform01(st);
        return std::sqrt(-2.0 * std::log(u1)) * std::cos(2.0 * M_PI * u2);
    };
    const int offs[3] = {0, 1024 + 64, 1024 + 64 + 4096 + 64};
    const int fan[3] = {16, 64, 64}, cnt[3] = {1024, 4096, 256};
    for (int L = 0; L < 3; ++L)
        for (int k = 0; k < cnt[L]; ++k) master[(size_t)(offs[L] + k)] = (float)(gauss() * std::sqrt(2.0 / fan[L]));
    for (int j = 0; j < bsk::kMlpGradLen; ++j) wb[(size_t)(32 + j)] = f32_to_bf16(master[(size_t)j]);
    const int bsz = cfg->batch, nb = bsz / 64;
    TrainBufs B;
    int rc;
    if ((rc = dalloc(B.wb, 2 * bsk::kMlpBlobLen)) || (rc = dalloc(B.master, 4 * bsk::kMlpGradLen)) ||
        (rc = dalloc(B.m1, 4 * bsk::kMlpGradLen)) || (rc = dalloc(B.m2, 4 * bsk::kMlpGradLen)) ||
        (rc = dalloc(B.gpart, 4 * (size_t)nb * bsk::kMlpGradLen)) || (rc = dalloc(B.wpart, 4 * (size_t)nb)) ||
        (rc = dalloc(B.lpart, 4 * (size_t)nb)) || (rc = dalloc(B.cw, 16)) || (rc = dalloc(B.index, 4 * (size_t)n)) ||
        (rc = dalloc(B.lsum, 16)))
        return rc;
    if ((e = hipMemcpyAsync(B.wb.p, wb.data(), 2 * wb.size(), hipMemcpyHostToDevice, s)) ||
        (e = hipMemcpyAsync(B.master.p, master.data(), 4 * master.size(), hipMemcpyHostToDevice, s)) ||
        (e = hipMemsetAsync(B.m1.p, 0, 4 * bsk::kMlpGradLen, s)) ||
        (e = hipMemsetAsync(B.m2.p, 0, 4 * bsk::kMlpGradLen, s)) ||
        (e = hipMemcpyAsync(B.cw.p, cfg->class_w, 16, hipMemcpyHostToDevice, s)))
        return hip_fail(e, "training setup");
    std::vector<int32_t> perm((size_t)n);
    for (int64_t i = 0; i < n; ++i) perm[(size_t)i] = (int32_t)i;
    int step = 0;
    for (int ep = 0; ep < cfg->epochs; ++ep) {
        for (int64_t i = n - 1; i > 0; --i) {
            const int64_t j = (int64_t)(uniform01(st) * (double)(i + 1));
            std::swap(perm[(size_t)i], perm[(size_t)std::min(j, i)]);
        }
        if ((e = hipMemcpyAsync(B.index.p, perm.data(), 4 * (size_t)n, hipMemcpyHostToDevice, s)))
            return hip_fail(e, "upload permutation");
        double lsum = 0.0, wsum = 0.0;
        for (int64_t b0 = 0; b0 + bsz <= n; b0 += bsz) {
            ++step;
            if ((e = bsk::launch_mlp_grad_step(feats, labels, (const int *)B.index.p + b0, bsz, (__bf16 *)B.wb.p,
                                               (const float *)B.cw.p, (float *)B.gpart.p, (float *)B.wpart.p,
                                               (float *)B.lpart.p, (float *)B.master.p, (float *)B.m1.p,
                                               (float *)B.m2.p, cfg->lr, cfg->beta1, cfg->beta2, cfg->eps, step,
                                               nullptr, s)))
                return hip_fail(e, "training step");
            if (epoch_loss && (b0 / bsz) % 64 == 0) {
                double sums[2];
                if ((e = bsk::launch_sum_f((const float *)B.lpart.p, nb, (double *)B.lsum.p, s)) ||
                    (e = bsk::launch_sum_f((const float *)B.wpart.p, nb, (double *)B.lsum.p + 1, s)) ||
                    (e = hipMemcpyAsync(sums, B.lsum.p, 16, hipMemcpyDeviceToHost, s)) ||
                    (e = hipStreamSynchronize(s)))
                    return hip_fail(e, "training loss");
                lsum += sums[0];
                wsum += sums[1];
            }
        }
        if (epoch_loss) epoch_loss[ep] = (float)(wsum > 0 ? lsum / wsum : 0.0);
    }
    if ((e = hipMemcpyAsync(wb.data(), B.wb.p, 2 * wb.size(), hipMemcpyDeviceToHost, s)) ||
        (e = hipStreamSynchronize(s)))
        return hip_fail(e, "read weights");
    std::memcpy(blob, wb.data(), 2 * wb.size());
    return BS_OK;
}

int bs_mlp_logits(const uint16_t *blob, const float *feats, int64_t n, float *logits, void *stream)
{
    g_err.clear();
    if (!blob || !feats || !logits || n < 0 || n > (1 << 28)) return fail(BS_E_ARG, "bad arguments");
    hipStream_t s = (hipStream_t)stream;
    DBuf wb;
    int rc = dalloc(wb, 2 * bsk::kMlpBlobLen);
    if (rc) return rc;
    hipError_t e;
    if ((e = hipMemcpyAsync(wb.p, blob, 2 * bsk::kMlpBlobLen, hipMemcpyHostToDevice, s)) ||
        (e = bsk::launch_mlp_logits(feats, (int)n, (const __bf16 *)wb.p, logits, s)) ||
        (e = hipStreamSynchronize(s))) {
        dfree(wb);
        return hip_fail(e, "logits kernel");
    }
    dfree(wb);
    return BS_OK;
}

} // extern "C"
