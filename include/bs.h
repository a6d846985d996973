/*
 * bs.h -- C ABI of the Biot-Savart node-velocity library for MI355X (gfx950).
 *
 * Problem (Carley, "Evaluation of Biot-Savart integrals on tetrahedral
 * meshes", Sections 1-2): given points x_i that carry vorticity omega_i and
 * form the vertices of a tetrahedral mesh over which omega varies linearly,
 * return the Biot-Savart velocity (eq. 1)
 *     v(x_i) = -(1/4pi) int_V (x_i - y) x omega(y) / |x_i - y|^3 dV(y)
 * at every node.  The method (Section 2.2): choose angular Gauss orders N
 * (polar) and M (azimuth), precompute the line directions s_nm and weights
 * k_nm, and sum over tetrahedra and lines the exact trapezoid of eq. 5 along
 * each chord; tetrahedra far from a node may instead be summed by a
 * volumetric Gauss rule (Introduction).
 *
 * Conventions shared by every entry point:
 *   - Every function returns an int status: BS_OK (0) or a negative BS_E_*
 *     code; none throws or aborts.  bs_last_error() gives a thread-local
 *     message for the last failure on the calling thread (offending index,
 *     HIP error string).
 *   - The caller owns every buffer it passes.  Uploads copy: inputs may be
 *     freed as soon as the call returns.  The library owns the device memory
 *     of a bs_mesh until bs_mesh_free.
 *   - Arrays are row-major, C-contiguous: xyz and omega are [n_nodes][3]
 *     doubles, tets is [n_tets][4] int32 node indices (0-based), vel is
 *     [n_nodes][3] doubles in input node order.
 *   - Pointers are host memory unless BS_PTR_DEVICE is set in the matching
 *     flags argument, in which case they are device pointers on the current
 *     HIP device.
 *   - `stream` is a hipStream_t cast to void* (NULL: the default stream).
 *     All device work is enqueued on it; calls that return host results
 *     synchronise it before returning.
 *   - A bs_mesh may be used by one thread at a time.
 */
#ifndef BS_H
#define BS_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------------ status */
#define BS_OK 0
#define BS_E_ARG (-1)        /* null pointer, negative size, bad flag         */
#define BS_E_INDEX (-2)      /* node index out of range or repeated in a tet  */
#define BS_E_DEGENERATE (-3) /* zero-volume tetrahedron                       */
#define BS_E_NONFINITE (-4)  /* NaN or Inf in coordinates or vorticity        */
#define BS_E_STATE (-5)      /* call out of order (e.g. eval without a mesh)  */
#define BS_E_DEVICE (-6)     /* no gfx950 device, or a HIP runtime failure    */
#define BS_E_NOMEM (-7)      /* device or host allocation failed              */
#define BS_E_POLICY (-8)     /* policy out of range                           */

#define BS_PTR_HOST 0u
#define BS_PTR_DEVICE 1u
/* bs_eval_velocity only: take the far field of the fixed-rule policies on
 * the vector ALUs (every pair by the 1-point rule, then the G1 term of the
 * other pairs removed) instead of the matrix cores (G1 pairs only, FP32
 * MFMA contractions).  Both compute the same sum; for comparison. */
#define BS_EVAL_VALU_FAR 0x10u
/* bs_eval_velocity only: run every kernel on the given stream, one after
 * another, instead of the band and ray-tracing kernels on two library
 * streams beside the far field (same results; per-kernel times then
 * measure each kernel alone). */
#define BS_EVAL_SERIAL 0x20u
/* bs_advect_heun only: advance the nodal vorticity too, by vortex
 * stretching dw/dt = (w . grad) v with the nodal velocity gradient of
 * bs_velocity_gradient (the paper's Lagrangian application, Sections 1 and
 * 3; the stretching model is this library's, the paper does not give one). */
#define BS_ADVECT_STRETCH 0x40u

/* Rules a (node, tetrahedron) pair can be evaluated with. */
#define BS_RULE_G1 0  /* 1-point Gauss rule (centroid), degree 1              */
#define BS_RULE_G4 1  /* 4-point symmetric Gauss rule, degree 2                */
#define BS_RULE_G11 2 /* 11-point symmetric Gauss rule, degree 4               */
#define BS_RULE_RT 3  /* ray tracing over the N x M lines (Section 2.1)        */

/* Pair-rule policies. */
#define BS_POLICY_FIXED 0      /* distance rule: RT / G11 / G4 / G1 (default)  */
#define BS_POLICY_PURE_RT 1    /* every pair ray traced (the paper's method)    */
#define BS_POLICY_GAUSS_ONLY 2 /* every pair by the Gauss rule `gauss_rule`     */
#define BS_POLICY_LEARNED 3    /* network-chosen rule, fixed rule as fallback   */

/* Accumulation precision of the pair sums (the final per-node sum is FP64). */
#define BS_PREC_FP32_NAIVE 0 /* one FP32 accumulator per component            */
#define BS_PREC_FP32_COMP 1  /* FP32 sums over short tiles, folded by TwoSum
                              * or in FP64 (default)                          */
#define BS_PREC_FP64 2       /* FP32 pair terms accumulated in FP64            */

typedef struct bs_mesh bs_mesh; /* opaque; owns all device memory */

/* Mesh description.  Nodes are both the vertices of the tetrahedra and the
 * points where the velocity is wanted (Section 2). */
typedef struct {
    int64_t n_nodes;      /* >= 1, at most 2^29                                */
    const double *xyz;    /* [n_nodes][3] coordinates                          */
    const double *omega;  /* [n_nodes][3] nodal vorticity                      */
    int64_t n_tets;       /* >= 0, at most 2^29                                */
    const int32_t *tets;  /* [n_tets][4] node indices                          */
    uint32_t flags;       /* BS_PTR_DEVICE: xyz, omega, tets are device memory */
    void *stream;         /* hipStream_t or NULL                               */
} bs_mesh_desc;

/* Validate and copy a mesh to the device, and run the O(n_tets) per-element
 * precompute (orientation, volume, centroid, rule points and strengths,
 * ray-tracing records, spatial bins).  Errors: BS_E_ARG (null pointers,
 * n_nodes outside [1, 2^29], n_tets outside [0, 2^29]: the kernels
 * index the node arrays in 32 bits), BS_E_INDEX (index outside [0, n_nodes) or
 * repeated within a tet; bs_last_error names the tet), BS_E_NONFINITE,
 * BS_E_DEGENERATE (|6 V| <= 1e-12 h_T^3, h_T its longest edge), BS_E_DEVICE,
 * BS_E_NOMEM.  On success *out holds a new mesh with the default policy. */
int bs_mesh_upload(const bs_mesh_desc *d, bs_mesh **out);

/* New coordinates and vorticity for the same connectivity (a Lagrangian
 * step, Section 3): re-runs the per-element precompute.  xyz and omega are
 * [n_nodes][3]; either may be NULL to keep the current values.  Errors as
 * bs_mesh_upload, plus BS_E_STATE for a NULL mesh. */
int bs_mesh_update(bs_mesh *m, const double *xyz, const double *omega, uint32_t flags, void *stream);

/* Release a mesh and all its device memory.  NULL is a no-op. */
void bs_mesh_free(bs_mesh *m);

/* Evaluation policy (Section 2.2 items 2-3 and the far-field rules of the
 * Introduction).  Distances are node-to-centroid, in units of the mesh's
 * mean edge length hbar (mean over unique edges):
 *   incident pair or d < near_cut      -> ray tracing,
 *   near_cut <= d < d_g11              -> 11-point rule,
 *   d_g11 <= d < d_g4                  -> 4-point rule,
 *   d >= d_g4                          -> 1-point rule.
 * The comparison is taken in binary32 on d^2.  LEARNED uses a 16-64-64-4
 * network (BF16 weights, layout documented at bs_mlp_* below) for the pairs
 * the fixed rule ray-traces whose tet does not contain the node: with p the
 * softmax of its logits over (G1, G4, G11, RT), the pair takes the cheapest
 * Gauss rule r with p_G1 + ... + p_r >= conf_min (the predicted probability
 * that r meets the error budget it was trained on), else keeps the fixed
 * rule. */
typedef struct {
    int kind;                 /* BS_POLICY_*                                    */
    int n_phi, n_theta;       /* N, M: each in [1, 256]                         */
    double near_cut;          /* > 0                                            */
    double d_g11, d_g4;       /* near_cut <= d_g11 <= d_g4                       */
    int gauss_rule;           /* GAUSS_ONLY: BS_RULE_G1, _G4 or _G11            */
    int precision;            /* BS_PREC_*                                      */
    const uint16_t *mlp_bf16; /* LEARNED: host pointer to the packed weights    */
    int64_t mlp_len;          /* LEARNED: number of uint16 in mlp_bf16          */
    float conf_min;           /* LEARNED: in [0, 1]                             */
    int far_field;            /* BS_FAR_*: how the 1-point-rule pairs are summed */
    double tree_theta;        /* BS_FAR_TREECODE: opening ratio, in (0, 1)      */
    int tree_order;           /* BS_FAR_TREECODE: expansion order, 2, 4 or 6    */
} bs_policy;

/* Far field of the FIXED and LEARNED policies (the pairs the distance rule
 * gives the 1-point rule).  ALL_PAIRS sums every such pair.  TREECODE is the
 * fast-multipole-like evaluation the paper leaves to future work (Section
 * 4), defined here as a batched Barnes-Hut treecode:
 *   - sources: the 1-point rule of each tet (centroid c_t, strength
 *     W_t = |T| omega(c_t) / 4pi);
 *   - clusters: the nodes of the recursive median split of the centroids
 *     (the node order's rule, leaves of at most 64 tets);
 *   - targets: the 64-node blocks of the node order;
 *   - each has the sphere (midpoint of the bounding box, largest distance
 *     to it) of its points in FP64.
 * Block B accepts cluster S iff
 *     |c_B - c_S|^2 >= (r_B + max(r_S / tree_theta, r_S + kappa))^2,
 *     kappa = max(d_g4 hbar, largest vertex-centroid distance) (1 + 1e-3),
 * so that every pair of (B, S) is a 1-point pair and every node sees the
 * cluster within ratio tree_theta.  Accepted clusters are evaluated by
 * their Cartesian multipole expansion of order tree_order.  Leaves that are
 * not accepted are summed pair by pair (the 1-point pairs only).  The error
 * against ALL_PAIRS is the expansions' truncation: at most
 *     |W| q^(P+1) ((P+2) - (P+1) q) / (R^2 (1 - q)^2)
 * per source at distance R from its cluster's centre, q = r_S / R <= theta.
 * TREECODE builds its plan (tree, spheres, interaction lists) on the host
 * when the policy is set and whenever the nodes move; it is refused for the
 * other policy kinds. */
#define BS_FAR_ALL_PAIRS 0
#define BS_FAR_TREECODE 1

/* Fill *p with the defaults: FIXED, N = M = 16, cuts 2 / 4 / 8, FP32_COMP,
 * ALL_PAIRS (tree_theta 0.3, tree_order 4 for TREECODE). */
void bs_policy_default(bs_policy *p);

/* Validate and install a policy on a mesh (copied; mlp weights copied to the
 * device; for BS_FAR_TREECODE the treecode's plan is built here and again
 * whenever the nodes move).  Errors: BS_E_STATE (NULL mesh), BS_E_POLICY (out
 * of range, bad weight blob size, the treecode for a policy without 1-point
 * pairs), BS_E_NOMEM (the treecode's interaction lists beyond 2^31 entries,
 * or no memory for them), BS_E_DEVICE. */
int bs_set_policy(bs_mesh *m, const bs_policy *p);

/* Counters of the last evaluation. */
typedef struct {
    double t_eval_s;          /* device time of the pair kernels and the sum   */
    double t_kernel_s[4];     /* far field, band corrections, ray tracing, sum */
    int64_t pairs;            /* n_nodes * n_tets                              */
    int64_t pairs_by_rule[4]; /* indexed by BS_RULE_*                          */
    int64_t rt_hit_lines;     /* (line, tet) hits of the ray-traced pairs      */
    int64_t fp64_retests;     /* near-edge orientation tests redone in FP64    */
    int64_t reoriented;       /* negatively oriented input tetrahedra          */
    int32_t nonfinite_out;    /* 1 if any output component is NaN or Inf       */
    double hbar;              /* mean edge length                              */
    int64_t tree_expansions;  /* TREECODE: (node, cluster) expansion terms     */
    int64_t tree_direct;      /* TREECODE: (node, tet) pairs of direct leaves  */
    int64_t tree_covered;     /* TREECODE: (node, tet) pairs the expansions sum */
    int64_t rt_walk_nodes;    /* nodes ray traced by walking face neighbours   */
    int64_t rt_candidate_nodes; /* nodes ray traced by candidate rays per pair:
                                 * off-node points, pure ray tracing on a
                                 * boundary that is not convex, nodes with no
                                 * or more than 48 incident tets, and, where the
                                 * boundary is not convex, nodes with a ray
                                 * that leaves the mesh before its last
                                 * ray-traced tet                              */
} bs_stats;

/* Velocity at every node, written to vel ([n_nodes][3] FP64, input node
 * order; host memory unless vel_flags has BS_PTR_DEVICE; BS_EVAL_VALU_FAR
 * selects the vector-ALU far field, BS_EVAL_SERIAL one stream).  The band
 * and ray-tracing kernels run on two streams owned by the mesh, joined back
 * to `stream` before the final sum, so the call is ordered on `stream` like
 * a single kernel.  Uses the policy last set (defaults if
 * none).  st may be NULL.  Errors: BS_E_STATE (NULL mesh), BS_E_ARG (NULL
 * vel, unknown flag), BS_E_DEVICE (launch or runtime failure). */
int bs_eval_velocity(bs_mesh *m, double *vel, uint32_t vel_flags, void *stream, bs_stats *st);

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops): bs_eval_velocity without any allocation.
 * The same kernels run on `stream` alone, with their partial sums, counters
 * and lists in a static device array of 64 MiB that the library holds on
 * every device it runs on until the process ends.  vel ([n_nodes][3] FP64,
 * input node order) must be device memory: flags must hold BS_PTR_DEVICE
 * (BS_EVAL_VALU_FAR allowed).  The policy's tables are installed by
 * bs_set_policy.  No statistics; the call does not synchronise.  The array
 * is shared by every call on a device, so calls that overlap on one device
 * (other streams or threads) race and must be ordered by the caller.
 * Errors: BS_E_STATE (NULL mesh), BS_E_ARG (NULL vel, host output, unknown
 * flag, or a mesh and policy whose buffers exceed 64 MiB: 24 bytes per
 * node slot for each tet split of the far field (8 splits on the matrix
 * cores), 48 more per node slot, and 532 per node for the learned policy),
 * BS_E_DEVICE. */
int bs_eval_velocity_noalloc(bs_mesh *m, double *vel, uint32_t flags, void *stream);

/* Velocity at n_pts arbitrary points pts ([n_pts][3] FP64; Section 3.1
 * evaluates the method at points that are not mesh nodes), written to vel
 * ([n_pts][3] FP64, the order of pts); pts and vel are device memory when
 * flags has BS_PTR_DEVICE, else host (BS_EVAL_VALU_FAR and BS_EVAL_SERIAL as
 * for bs_eval_velocity).  Every tet contributes by the current policy's
 * rule for its pair with the point; no tet has a point as a vertex, so a
 * point inside a tet is ray traced from inside it (its chords start at the
 * point, with the tet's linear vorticity there) and a point outside the
 * mesh sees only whole chords.  The points are kept with the mesh (a new
 * set re-runs the per-element precompute once; the nodes' own evaluation is
 * unaffected); n_pts = 0 clears them.  Errors: BS_E_STATE (NULL mesh),
 * BS_E_ARG (n_pts < 0 or above 2^28, or n_nodes rounded up to a multiple
 * of 1024 plus n_pts above 2^29; NULL pointer, unknown flag),
 * BS_E_NONFINITE (a coordinate), BS_E_DEVICE. */
int bs_eval_points(bs_mesh *m, int64_t n_pts, const double *pts, double *vel, uint32_t flags, void *stream,
                   bs_stats *st);

/* Lagrangian motion of the nodes (the paper's setting, Sections 1 and 3:
 * control points move with the flow and the velocity is re-evaluated every
 * step): `steps` Heun (RK2) steps of size dt,
 *     v1 = v(x); x* = x + dt v1; v2 = v(x*); x <- x + dt/2 (v1 + v2),
 * with the current policy and connectivity kept.  The nodal vorticity is
 * kept too, unless flags has BS_ADVECT_STRETCH: then it takes the same Heun
 * steps with dw/dt = G w, G the nodal velocity gradient (bs_velocity_gradient)
 * of each stage's velocities,
 *     s1 = G(v1) w; w* = w + dt s1; s2 = G(v2) w*; w <- w + dt/2 (s1 + s2),
 * and stage two is evaluated with w*.  The position and vorticity updates
 * are FP64 on the host; each stage re-runs the per-element precompute and
 * one evaluation.  The mesh ends at the new state (bs_mesh_read returns it);
 * xyz_out ([n_nodes][3], host or device per flags; may be NULL) receives
 * the positions; step_seconds (host, `steps` doubles; may be NULL) the wall
 * time of every step; st (may be NULL) the counters of the last evaluation,
 * with t_eval_s the summed device time of all evaluations.  Errors:
 * BS_E_STATE (NULL mesh), BS_E_ARG (steps < 0, non-finite dt, unknown
 * flag), BS_E_DEGENERATE (a tetrahedron flattens or inverts relative to its
 * uploaded orientation), BS_E_NONFINITE (the vorticity overflows); on an
 * error the mesh is left at the start of that step; BS_E_DEVICE. */
int bs_advect_heun(bs_mesh *m, double dt, int steps, double *xyz_out, uint32_t flags, void *stream,
                   double *step_seconds, bs_stats *st);

/* Nodal velocity gradient grad ([n_nodes][3][3] FP64, grad[i][a][b] =
 * dv_a/dx_b at node i, input order) of the piecewise-linear interpolant of
 * nodal velocities vel ([n_nodes][3] FP64), which the vortex-stretching
 * term (w . grad) v of a Lagrangian vortex method needs (the application of
 * Sections 1 and 3; the paper does not define a discretisation, this is the
 * library's): on each tetrahedron the interpolant's constant gradient
 * D E^-1 (E: edge vectors from vertex 0, D: the velocity differences along
 * them), at each node the mean of the gradients of its tetrahedra weighted
 * by their volumes (0 for a node of no tetrahedron).  vel = NULL takes the
 * velocities of the last bs_eval_velocity (at the current positions and
 * vorticity).  vel and grad are device memory when flags has BS_PTR_DEVICE,
 * else host.  FP64 throughout, deterministic.  Errors: BS_E_STATE (NULL mesh;
 * vel NULL with no current evaluation), BS_E_ARG (NULL grad, unknown flag),
 * BS_E_NONFINITE (a host velocity), BS_E_DEVICE. */
int bs_velocity_gradient(bs_mesh *m, const double *vel, double *grad, uint32_t flags, void *stream);

/* Vortex stretching rate (omega . grad) v at every node (Sections 1 and 3:
 * the Lagrangian vortex method moves vorticity-carrying nodes; the paper
 * gives no discretisation of the stretching term): rate[i] = G_i omega_i
 * with G_i the nodal velocity gradient of bs_velocity_gradient and omega_i
 * the mesh's current nodal vorticity, rate [n_nodes][3] FP64 in input node
 * order.  vel: nodal velocities as for bs_velocity_gradient (NULL: the last
 * bs_eval_velocity).  rate and vel are device memory with BS_PTR_DEVICE.
 * Errors as bs_velocity_gradient. */
int bs_stretching_rate(bs_mesh *m, const double *vel, double *rate, uint32_t flags, void *stream);

/* The mesh's current FP64 node positions and nodal vorticity ([n_nodes][3]
 * each, input order; either pointer may be NULL), e.g. after
 * bs_advect_heun; device memory when flags has BS_PTR_DEVICE, else host.
 * Errors: BS_E_STATE (NULL mesh), BS_E_ARG (unknown flag), BS_E_DEVICE. */
int bs_mesh_read(bs_mesh *m, double *xyz, double *omega, uint32_t flags, void *stream);

/* ------------------------------------------------------------ rule selector
 * A 16-64-64-4 network (ReLU, BF16 weights and activations, FP32
 * accumulation on the matrix cores) picks, for pairs the fixed rule sends
 * to ray tracing and whose tet does not contain the node, the cheapest
 * rule (BS_RULE_*) expected to meet an error budget; the fixed rule is the
 * fallback below a softmax confidence, and the method's own errors decide
 * the labels.  The
 * training pairs are labelled by the method itself (bs_learn_pairs).
 *
 * Packed blob (BS_MLP_BLOB_LEN uint16 BF16 values, in this order):
 *   mu[16], inv_sigma[16]   feature standardisation xs = (x - mu) * inv_sigma
 *   W1[16][64], b1[64], W2[64][64], b2[64], W3[64][4], b3[4]   (row = input)
 * Features of a pair (x, tet with vertices v_j): c = centroid - x, d = |c|,
 * h_T / h_min longest / shortest edge, lambda_j barycentric coordinates of
 * x, n_f outward unit face normals, 6V the volume triple product:
 *   d/h_T, d/hbar, h_T/h_min, hbar/d, sort_desc(lambda_j h_T/d) [4],
 *   sort_desc(n_f . (-c/d)) [4], incident (0/1), 6V/h_T^3,
 *   min_f dist(x, plane f)/h_T, 1. */
#define BS_MLP_BLOB_LEN 5540

/* Sample up to max_pairs (node, tet) pairs from the band the fixed rule
 * (current policy's cut distances) ray-traces, skipping tets that contain
 * the node: nodes are drawn without replacement (splitmix64 seeded by
 * `seed`) and all their band pairs taken.  pairs: host [max_pairs][2]
 * int32 (input node index, input tet index); *n_out: pairs written.
 * Errors: BS_E_STATE (NULL mesh), BS_E_ARG. */
int bs_learn_sample_pairs(bs_mesh *m, int64_t max_pairs, uint64_t seed, int32_t *pairs, int64_t *n_out);

/* Label given pairs (host [n][2] int32, input numbering): features
 * (device [n][16] float), relative errors of the 1-, 4- and 11-point rules
 * against a high-accuracy value of the pair's integral (device [n][3]
 * float; FP64 signed-cone integral with a 24 x 24 collapsed Gauss rule per
 * face), and label = the cheapest rule with error <= tau, else BS_RULE_RT
 * (device [n] int8).  Errors: BS_E_STATE, BS_E_ARG, BS_E_INDEX, BS_E_DEVICE. */
int bs_learn_pairs(bs_mesh *m, const int32_t *pairs, int64_t n, double tau, float *feats, int8_t *labels,
                   float *errs, void *stream);

typedef struct {
    int epochs;       /* passes over the data                                */
    int batch;        /* rows per Adam step, a positive multiple of 64       */
    float lr, beta1, beta2, eps; /* Adam                                     */
    float class_w[4]; /* cross-entropy weight of each true class             */
    uint64_t seed;    /* initialisation and shuffling                        */
} bs_train_cfg;

/* Train the network on n rows (feats device [n][16] float, labels device
 * [n] int8 in 0..3): standardisation from the data, He initialisation,
 * class-weighted softmax cross-entropy, forward and backward on the matrix
 * cores, Adam on FP32 master weights.  blob: host output (BS_MLP_BLOB_LEN);
 * epoch_loss: host [epochs] (may be NULL), mean weighted loss of sampled
 * steps.  Errors: BS_E_ARG, BS_E_NOMEM, BS_E_DEVICE. */
int bs_mlp_train(const float *feats, const int8_t *labels, int64_t n, const bs_train_cfg *cfg, uint16_t *blob,
                 float *epoch_loss, void *stream);

/* One forward and backward pass (gradient check): blob host BF16, feats /
 * labels device, class_w host [4]; loss (host, may be NULL) = weighted mean
 * cross-entropy; grads host [BS_MLP_BLOB_LEN - 32] FP32 gradients of
 * W1, b1, W2, b2, W3, b3 in blob order.  Errors: BS_E_ARG, BS_E_DEVICE. */
int bs_mlp_grad(const uint16_t *blob, const float *feats, const int8_t *labels, int64_t n, const float *class_w,
                float *loss, float *grads, void *stream);

/* Logits of the network for n rows: blob host, feats device [n][16],
 * logits device [n][4].  Errors: BS_E_ARG, BS_E_DEVICE. */
int bs_mlp_logits(const uint16_t *blob, const float *feats, int64_t n, float *logits, void *stream);

/* Static description of a status code. */
const char *bs_status_string(int status);

/* Thread-local detail of the last failure on this thread ("" if none). */
const char *bs_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* BS_H */
