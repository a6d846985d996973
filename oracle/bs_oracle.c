/*
 * bs_oracle.c -- plain, slow FP64 CPU oracle for the Biot-Savart velocity at
 * the nodes of a tetrahedral mesh carrying piecewise-linear vorticity
 * (M. Carley, "Evaluation of Biot-Savart integrals on tetrahedral meshes").
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may build, load or call this file.  It shares
 * no code, header, table or constant generator with the GPU library.
 *
 * What it computes, in the paper's order:
 *   - Gauss-Legendre nodes and weights (Section 2, eq. 3), by Newton's
 *     method on the Legendre polynomial;
 *   - the line directions s_nm and factors k_nm (Section 2.2, item 3), with
 *     the constant pi/16 (the printed 1/(16 pi^2) does not give the
 *     half-sphere measure; see the reading list in the design notes);
 *   - for each pair (node x, tetrahedron T) a rule from the policy; for ray
 *     tracing (Section 2.1): for every line the precheck (skip when
 *     (r.s)^2 < |r|^2 - 2 h^2, r = first vertex - x), then a Moller-Trumbore
 *     line/triangle test on each face in turn (eqs. 4-5), the vorticity at
 *     each hit by area coordinates, and the exact trapezoid of eq. 5 with
 *     the sign of R restored (the integrand of eq. 2 is sgn(R) s x omega on
 *     the full line);
 *   - far pairs by symmetric Gauss rules over the tetrahedron (1, 4 or 11
 *     points; the standard approach the introduction mentions);
 *   - the velocity at each node as the FP64 sum over tetrahedra, in input
 *     order (optionally Neumaier-compensated).
 *
 * Where a floating-point comparison picks the rule of a pair (the distance
 * from the node to the centroid against the thresholds) the decision is
 * taken in IEEE binary32, exactly as the GPU kernels take it, so both sides
 * agree on which rule each pair uses.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#ifdef _OPENMP
#include <omp.h>
#endif

#define BSO_RULE_G1 0
#define BSO_RULE_G4 1
#define BSO_RULE_G11 2
#define BSO_RULE_RT 3

#define BSO_POLICY_FIXED 0      /* distance rule: RT / G11 / G4 / G1 */
#define BSO_POLICY_PURE_RT 1    /* every pair ray traced (the paper's method) */
#define BSO_POLICY_GAUSS_ONLY 2 /* every pair by one Gauss rule (test policy) */
#define BSO_POLICY_EXPLICIT 3   /* rule per (target, tet) given by the caller */

typedef struct {
    int kind;
    int n_phi, n_theta;
    double near_cut, d_g11, d_g4; /* in mean-edge units */
    int gauss_rule;               /* BSO_RULE_G1/G4/G11 for GAUSS_ONLY */
    int precheck;                 /* apply the paper's precheck */
    int neumaier;                 /* compensated per-node sum */
    const int8_t *pair_rules;     /* EXPLICIT: [n_targets][n_tets] */
} bso_policy;

typedef struct {
    int64_t pairs_by_rule[4];
    int64_t rt_lines;      /* line tests reaching the face tests */
    int64_t rt_hit_lines;  /* lines that hit the tetrahedron */
    int64_t rt_face_hits;  /* accepted face intersections */
    double algo_flops;     /* algorithmic flop count (see the design notes) */
    double hbar;           /* mean edge length used by the distance rule */
} bso_counters;

/* ------------------------------------------------------------------------
 * Gauss-Legendre rule on [-1, 1]: Newton iteration on P_n from the
 * classical starting values cos(pi (i - 1/4) / (n + 1/2)).  Nodes returned
 * in ascending order. */
int bso_gauss_legendre(int n, double *t, double *w)
{
    if (n < 1 || n > 4096) return -1;
    for (int i = 0; i < n; ++i) {
        double x = cos(M_PI * (i + 0.75) / (n + 0.5));
        double dp = 0.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double pn = (n == 1) ? x : p1;
            double pm = (n == 1) ? 1.0 : p0;
            /* P_n'(x) = n (x P_n - P_{n-1}) / (x^2 - 1) */
            dp = n * (x * pn - pm) / (x * x - 1.0);
            double dx = pn / dp;
            x -= dx;
            if (fabs(dx) < 1e-16) break;
        }
        {
            double p0 = 1.0, p1 = x;
            for (int k = 2; k <= n; ++k) {
                double p2 = ((2.0 * k - 1.0) * x * p1 - (k - 1.0) * p0) / k;
                p0 = p1;
                p1 = p2;
            }
            double pn = (n == 1) ? x : p1;
            double pm = (n == 1) ? 1.0 : p0;
            dp = n * (x * pn - pm) / (x * x - 1.0);
        }
        /* cos of increasing angle decreases: store ascending */
        t[n - 1 - i] = x;
        w[n - 1 - i] = 2.0 / ((1.0 - x * x) * dp * dp);
    }
    return 0;
}

/* ------------------------------------------------------------------------
 * Symmetric Gauss rules on a tetrahedron, as barycentric points (k x 4) and
 * weights summing to one (the rule integrates f over T as |T| sum w f).
 *   k = 1:  centroid, degree 1;
 *   k = 4:  orbit (a, b, b, b), a = (5 + 3 sqrt5)/20, b = (5 - sqrt5)/20,
 *           weights 1/4, degree 2;
 *   k = 11: Keast's degree-4 rule: centroid (weight -148/1875), orbit
 *           (11/14, 1/14, 1/14, 1/14) (weight 343/7500) and orbit
 *           (c, c, d, d), c,d = (1 +- sqrt(5/14))/4 (weight 56/375). */
int bso_tet_rule(int k, double *lam, double *w)
{
    if (k == 1) {
        for (int j = 0; j < 4; ++j) lam[j] = 0.25;
        w[0] = 1.0;
        return 0;
    }
    if (k == 4) {
        double a = (5.0 + 3.0 * sqrt(5.0)) / 20.0, b = (5.0 - sqrt(5.0)) / 20.0;
        for (int q = 0; q < 4; ++q) {
            for (int j = 0; j < 4; ++j) lam[4 * q + j] = (j == q) ? a : b;
            w[q] = 0.25;
        }
        return 0;
    }
    if (k == 11) {
        int q = 0;
        for (int j = 0; j < 4; ++j) lam[4 * q + j] = 0.25;
        w[q++] = -148.0 / 1875.0;
        for (int v = 0; v < 4; ++v, ++q) {
            for (int j = 0; j < 4; ++j) lam[4 * q + j] = (j == v) ? 11.0 / 14.0 : 1.0 / 14.0;
            w[q] = 343.0 / 7500.0;
        }
        double c = (1.0 + sqrt(5.0 / 14.0)) / 4.0, d = (1.0 - sqrt(5.0 / 14.0)) / 4.0;
        for (int i = 0; i < 4; ++i)
            for (int j = i + 1; j < 4; ++j, ++q) {
                for (int l = 0; l < 4; ++l) lam[4 * q + l] = (l == i || l == j) ? c : d;
                w[q] = 56.0 / 375.0;
            }
        return 0;
    }
    return -1;
}

/* ------------------------------------------------------------------------
 * Mean edge length over the unique edges of the mesh.  Edges are keyed by
 * (min node, max node); the lengths are summed in increasing key order. */
typedef struct { int64_t key; } bso_edge;

static int cmp_i64(const void *a, const void *b)
{
    int64_t x = *(const int64_t *)a, y = *(const int64_t *)b;
    return (x > y) - (x < y);
}

double bso_mean_edge(int64_t n_nodes, const double *xyz, int64_t n_tets, const int32_t *tets)
{
    static const int ea[6] = {0, 0, 0, 1, 1, 2}, eb[6] = {1, 2, 3, 2, 3, 3};
    int64_t ne = 6 * n_tets;
    int64_t *keys = (int64_t *)malloc(sizeof(int64_t) * (size_t)(ne > 0 ? ne : 1));
    if (!keys) return -1.0;
    for (int64_t t = 0; t < n_tets; ++t)
        for (int e = 0; e < 6; ++e) {
            int64_t a = tets[4 * t + ea[e]], b = tets[4 * t + eb[e]];
            int64_t lo = a < b ? a : b, hi = a < b ? b : a;
            keys[6 * t + e] = lo * (n_nodes + 1) + hi;
        }
    qsort(keys, (size_t)ne, sizeof(int64_t), cmp_i64);
    double sum = 0.0;
    int64_t cnt = 0;
    for (int64_t i = 0; i < ne; ++i) {
        if (i > 0 && keys[i] == keys[i - 1]) continue;
        int64_t lo = keys[i] / (n_nodes + 1), hi = keys[i] % (n_nodes + 1);
        double dx = xyz[3 * hi] - xyz[3 * lo], dy = xyz[3 * hi + 1] - xyz[3 * lo + 1],
               dz = xyz[3 * hi + 2] - xyz[3 * lo + 2];
        sum += sqrt(dx * dx + dy * dy + dz * dz);
        ++cnt;
    }
    free(keys);
    return cnt ? sum / (double)cnt : 0.0;
}

/* ------------------------------------------------------------------------ */
static inline void cross3(const double *a, const double *b, double *c)
{
    c[0] = a[1] * b[2] - a[2] * b[1];
    c[1] = a[2] * b[0] - a[0] * b[2];
    c[2] = a[0] * b[1] - a[1] * b[0];
}
static inline double dot3(const double *a, const double *b) { return a[0] * b[0] + a[1] * b[1] + a[2] * b[2]; }

/* Per-tetrahedron data, computed once per evaluation. */
typedef struct {
    int32_t id[4];      /* node ids in input order */
    double v[4][3];     /* vertex coordinates */
    double om[4][3];    /* vertex vorticity */
    double vol;         /* |T| */
    double cen[3];      /* centroid (v0+v1+v2+v3)/4, summed in input order */
    float cen32[3];     /* centroid rounded to binary32 (rule decision) */
    double h2;          /* longest edge squared (precheck) */
} bso_tet;

static void tet_setup(const double *xyz, const double *omega, const int32_t *ids, bso_tet *T)
{
    for (int j = 0; j < 4; ++j) {
        T->id[j] = ids[j];
        for (int c = 0; c < 3; ++c) {
            T->v[j][c] = xyz[3 * (int64_t)ids[j] + c];
            T->om[j][c] = omega[3 * (int64_t)ids[j] + c];
        }
    }
    double e1[3], e2[3], e3[3], n[3];
    for (int c = 0; c < 3; ++c) {
        e1[c] = T->v[1][c] - T->v[0][c];
        e2[c] = T->v[2][c] - T->v[0][c];
        e3[c] = T->v[3][c] - T->v[0][c];
    }
    cross3(e2, e3, n);
    T->vol = fabs(dot3(e1, n)) / 6.0;
    for (int c = 0; c < 3; ++c) {
        T->cen[c] = (((T->v[0][c] + T->v[1][c]) + T->v[2][c]) + T->v[3][c]) * 0.25;
        T->cen32[c] = (float)T->cen[c];
    }
    double h2 = 0.0;
    for (int a = 0; a < 4; ++a)
        for (int b = a + 1; b < 4; ++b) {
            double d[3] = {T->v[b][0] - T->v[a][0], T->v[b][1] - T->v[a][1], T->v[b][2] - T->v[a][2]};
            double l2 = dot3(d, d);
            if (l2 > h2) h2 = l2;
        }
    T->h2 = h2;
}

/* Rule of a pair under the fixed distance policy, decided in binary32:
 * d2 = ((dx*dx + dy*dy) + dz*dz) with dx = fl32(x) - fl32(centroid), each
 * operation rounded separately (no fused multiply-add). */
static int fixed_rule(const float x32[3], const bso_tet *T, int incident, const float thr2[3])
{
    if (incident) return BSO_RULE_RT;
    volatile float dx = x32[0] - T->cen32[0];
    volatile float dy = x32[1] - T->cen32[1];
    volatile float dz = x32[2] - T->cen32[2];
    volatile float sx = dx * dx;
    volatile float sy = dy * dy;
    volatile float sz = dz * dz;
    volatile float sxy = sx + sy;
    float d2 = sxy + sz;
    if (d2 < thr2[0]) return BSO_RULE_RT;
    if (d2 < thr2[1]) return BSO_RULE_G11;
    if (d2 < thr2[2]) return BSO_RULE_G4;
    return BSO_RULE_G1;
}

/* Far-field Gauss rule: -(1/4 pi) sum_q w_q |T| (x - p_q) x omega(p_q) / |x - p_q|^3. */
static void gauss_rule(const double *x, const bso_tet *T, int npts, const double *lam, const double *wq,
                       double *out)
{
    out[0] = out[1] = out[2] = 0.0;
    for (int q = 0; q < npts; ++q) {
        double p[3] = {0, 0, 0}, om[3] = {0, 0, 0};
        for (int j = 0; j < 4; ++j)
            for (int c = 0; c < 3; ++c) {
                p[c] += lam[4 * q + j] * T->v[j][c];
                om[c] += lam[4 * q + j] * T->om[j][c];
            }
        double r[3] = {x[0] - p[0], x[1] - p[1], x[2] - p[2]};
        double R2 = dot3(r, r);
        double R3 = R2 * sqrt(R2);
        double rxw[3];
        cross3(r, om, rxw);
        double f = -wq[q] * T->vol / (4.0 * M_PI * R3);
        for (int c = 0; c < 3; ++c) out[c] += f * rxw[c];
    }
}

/* Moller-Trumbore test of the full line x + t s against triangle (a, b, c):
 * two-sided, t of either sign, closed inclusion tests; a (near-)parallel
 * triangle (|det| <= 1e-14 |e1| |e2|) gives no hit.  Returns 1 and (t,u,v)
 * on a hit. */
static int mt_line(const double *x, const double *s, const double *a, const double *b, const double *c,
                   double *t, double *u, double *v)
{
    double e1[3] = {b[0] - a[0], b[1] - a[1], b[2] - a[2]};
    double e2[3] = {c[0] - a[0], c[1] - a[1], c[2] - a[2]};
    double P[3];
    cross3(s, e2, P);
    double det = dot3(e1, P);
    if (fabs(det) <= 1e-14 * sqrt(dot3(e1, e1) * dot3(e2, e2))) return 0;
    double inv = 1.0 / det;
    double Tv[3] = {x[0] - a[0], x[1] - a[1], x[2] - a[2]};
    double uu = dot3(Tv, P) * inv;
    if (uu < 0.0 || uu > 1.0) return 0;
    double Q[3];
    cross3(Tv, e1, Q);
    double vv = dot3(s, Q) * inv;
    if (vv < 0.0 || uu + vv > 1.0) return 0;
    *t = dot3(e2, Q) * inv;
    *u = uu;
    *v = vv;
    return 1;
}

/* Ray-traced contribution of one tetrahedron to the velocity at node x
 * (node index `self`, nodal vorticity om_x), summed over all N x M lines. */
static void ray_trace(const double *x, int64_t self, const double *om_x, const bso_tet *T, int nl,
                      const double *s_tab, const double *k_tab, int precheck, double *out, int64_t *lines,
                      int64_t *hit_lines, int64_t *face_hits)
{
    /* faces: the face opposite vertex f has vertices in ascending local order */
    static const int fv[4][3] = {{1, 2, 3}, {0, 2, 3}, {0, 1, 3}, {0, 1, 2}};
    int inc = -1;
    for (int j = 0; j < 4; ++j)
        if ((int64_t)T->id[j] == self) inc = j;
    double acc[3] = {0, 0, 0};
    double r[3] = {T->v[0][0] - x[0], T->v[0][1] - x[1], T->v[0][2] - x[2]};
    double rr = dot3(r, r);
    for (int l = 0; l < nl; ++l) {
        const double *s = s_tab + 3 * l;
        if (precheck) {
            double rs = dot3(r, s);
            if (rs * rs < rr - 2.0 * T->h2) continue;
        }
        ++*lines;
        double th[4], wh[4][3];
        int nh = 0;
        for (int f = 0; f < 4; ++f) {
            if (inc >= 0 && f != inc) continue; /* faces containing x are skipped */
            const int *q = fv[f];
            double t, u, v;
            if (!mt_line(x, s, T->v[q[0]], T->v[q[1]], T->v[q[2]], &t, &u, &v)) continue;
            th[nh] = t;
            for (int c = 0; c < 3; ++c)
                wh[nh][c] = (1.0 - u - v) * T->om[q[0]][c] + u * T->om[q[1]][c] + v * T->om[q[2]][c];
            ++nh;
        }
        *face_hits += nh;
        double I[3] = {0, 0, 0};
        if (inc >= 0) {
            if (nh < 1) continue;
            /* chord from x (R = 0, omega_x) to the opposite face (R = t):
             * the integral of sgn(R) s x omega over it is t/2 s x (om_x + om_t) */
            double ws[3] = {om_x[0] + wh[0][0], om_x[1] + wh[0][1], om_x[2] + wh[0][2]};
            double sx[3];
            cross3(s, ws, sx);
            for (int c = 0; c < 3; ++c) I[c] = 0.5 * th[0] * sx[c];
        } else {
            if (nh < 2) continue;
            int i0 = 0, i1 = 0;
            for (int h = 1; h < nh; ++h) {
                if (th[h] < th[i0]) i0 = h;
                if (th[h] > th[i1]) i1 = h;
            }
            double R0 = th[i0], R1 = th[i1];
            const double *w0 = wh[i0], *w1 = wh[i1];
            if (R0 >= 0.0 || R1 <= 0.0) {
                double sg = (R0 >= 0.0) ? 1.0 : -1.0;
                double ws[3] = {w0[0] + w1[0], w0[1] + w1[1], w0[2] + w1[2]};
                double sx[3];
                cross3(s, ws, sx);
                for (int c = 0; c < 3; ++c) I[c] = sg * 0.5 * (R1 - R0) * sx[c];
            } else {
                /* the line passes through x inside T: split at R = 0 */
                double wz[3], a1[3], a0[3], s1[3], s0[3];
                double f = -R0 / (R1 - R0);
                for (int c = 0; c < 3; ++c) {
                    wz[c] = w0[c] + f * (w1[c] - w0[c]);
                    a1[c] = wz[c] + w1[c];
                    a0[c] = w0[c] + wz[c];
                }
                cross3(s, a1, s1);
                cross3(s, a0, s0);
                for (int c = 0; c < 3; ++c) I[c] = 0.5 * R1 * s1[c] - 0.5 * (-R0) * s0[c];
            }
        }
        ++*hit_lines;
        for (int c = 0; c < 3; ++c) acc[c] += k_tab[l] * I[c];
    }
    for (int c = 0; c < 3; ++c) out[c] = acc[c];
}

/* ------------------------------------------------------------------------
 * Angular tables: line directions s_nm and factors k_nm = (pi/16) sin(phi_n)
 * w_n w_m with phi_n = (1 + t_n) pi/2, theta_m = (1 + t_m) pi/2.  Line index
 * l = n * M + m. */
int bso_angular_tables(int N, int M, double *s_tab, double *k_tab)
{
    double *tn = (double *)malloc(sizeof(double) * (size_t)(2 * N + 2 * M));
    if (!tn) return -1;
    double *wn = tn + N, *tm = wn + N, *wm = tm + M;
    if (bso_gauss_legendre(N, tn, wn) || bso_gauss_legendre(M, tm, wm)) {
        free(tn);
        return -1;
    }
    for (int n = 0; n < N; ++n) {
        double phi = (1.0 + tn[n]) * M_PI / 2.0;
        for (int m = 0; m < M; ++m) {
            double th = (1.0 + tm[m]) * M_PI / 2.0;
            int l = n * M + m;
            s_tab[3 * l + 0] = sin(phi) * cos(th);
            s_tab[3 * l + 1] = sin(phi) * sin(th);
            s_tab[3 * l + 2] = cos(phi);
            k_tab[l] = M_PI / 16.0 * sin(phi) * wn[n] * wm[m];
        }
    }
    free(tn);
    return 0;
}

/* ------------------------------------------------------------------------
 * Velocity at the target nodes.  targets == NULL means every node, in node
 * order.  vel: [n_targets][3].  rules_out (optional): [n_targets][n_tets]
 * rule ids actually used.  Returns 0, or -1 on bad arguments / memory. */
int bso_eval(int64_t n_nodes, const double *xyz, const double *omega, int64_t n_tets, const int32_t *tets,
             const bso_policy *pol, int64_t n_targets, const int64_t *targets, double *vel, int8_t *rules_out,
             bso_counters *cnt)
{
    if (!xyz || !omega || !tets || !pol || !vel || n_nodes <= 0 || n_tets < 0) return -1;
    if (!targets) n_targets = n_nodes;
    if (pol->n_phi < 1 || pol->n_theta < 1) return -1;
    int nl = pol->n_phi * pol->n_theta;
    double *s_tab = (double *)malloc(sizeof(double) * 4 * (size_t)nl);
    bso_tet *TT = (bso_tet *)malloc(sizeof(bso_tet) * (size_t)(n_tets > 0 ? n_tets : 1));
    if (!s_tab || !TT) {
        free(s_tab);
        free(TT);
        return -1;
    }
    double *k_tab = s_tab + 3 * nl;
    if (bso_angular_tables(pol->n_phi, pol->n_theta, s_tab, k_tab)) {
        free(s_tab);
        free(TT);
        return -1;
    }
    double lam1[4], w1[1], lam4[16], w4[4], lam11[44], w11[11];
    bso_tet_rule(1, lam1, w1);
    bso_tet_rule(4, lam4, w4);
    bso_tet_rule(11, lam11, w11);

    for (int64_t t = 0; t < n_tets; ++t) tet_setup(xyz, omega, tets + 4 * t, &TT[t]);

    double hbar = (n_tets > 0) ? bso_mean_edge(n_nodes, xyz, n_tets, tets) : 0.0;
    float thr2[3];
    {
        double c[3] = {pol->near_cut * hbar, pol->d_g11 * hbar, pol->d_g4 * hbar};
        for (int i = 0; i < 3; ++i) thr2[i] = (float)(c[i] * c[i]);
    }

    int64_t pr[4] = {0, 0, 0, 0}, lines = 0, hitl = 0, fh = 0;
    int64_t ti;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : lines, hitl, fh)
    for (ti = 0; ti < n_targets; ++ti) {
        int64_t i = targets ? targets[ti] : ti;
        const double *x = xyz + 3 * i;
        const double *om_x = omega + 3 * i;
        float x32[3] = {(float)x[0], (float)x[1], (float)x[2]};
        double sum[3] = {0, 0, 0}, comp[3] = {0, 0, 0};
        int64_t lpr[4] = {0, 0, 0, 0};
        for (int64_t t = 0; t < n_tets; ++t) {
            const bso_tet *T = &TT[t];
            int incident = (T->id[0] == i || T->id[1] == i || T->id[2] == i || T->id[3] == i);
            int rule;
            switch (pol->kind) {
            case BSO_POLICY_PURE_RT: rule = BSO_RULE_RT; break;
            case BSO_POLICY_GAUSS_ONLY: rule = pol->gauss_rule; break;
            case BSO_POLICY_EXPLICIT: rule = pol->pair_rules[ti * n_tets + t]; break;
            default: rule = fixed_rule(x32, T, incident, thr2);
            }
            if (rules_out) rules_out[ti * n_tets + t] = (int8_t)rule;
            lpr[rule & 3]++;
            double c[3];
            if (rule == BSO_RULE_RT)
                ray_trace(x, i, om_x, T, nl, s_tab, k_tab, pol->precheck, c, &lines, &hitl, &fh);
            else if (rule == BSO_RULE_G11)
                gauss_rule(x, T, 11, lam11, w11, c);
            else if (rule == BSO_RULE_G4)
                gauss_rule(x, T, 4, lam4, w4, c);
            else
                gauss_rule(x, T, 1, lam1, w1, c);
            for (int k = 0; k < 3; ++k) {
                if (pol->neumaier) {
                    double s2 = sum[k] + c[k];
                    if (fabs(sum[k]) >= fabs(c[k]))
                        comp[k] += (sum[k] - s2) + c[k];
                    else
                        comp[k] += (c[k] - s2) + sum[k];
                    sum[k] = s2;
                } else {
                    sum[k] += c[k];
                }
            }
        }
        for (int k = 0; k < 3; ++k) vel[3 * ti + k] = sum[k] + comp[k];
#pragma omp critical
        {
            for (int k = 0; k < 4; ++k) pr[k] += lpr[k];
        }
    }
    if (cnt) {
        for (int k = 0; k < 4; ++k) cnt->pairs_by_rule[k] = pr[k];
        cnt->rt_lines = lines;
        cnt->rt_hit_lines = hitl;
        cnt->rt_face_hits = fh;
        cnt->hbar = hbar;
        /* algorithmic flops: 26 per Gauss point; ray tracing 9 per pair +
         * 7 per line precheck + 156 per line that hits */
        cnt->algo_flops = 26.0 * pr[0] + 104.0 * pr[1] + 286.0 * pr[2] + 9.0 * pr[3] +
                          7.0 * (double)nl * pr[3] + 156.0 * (double)hitl;
    }
    free(s_tab);
    free(TT);
    return 0;
}

/* Per-pair contribution of one rule (for brute-force and per-rule tests):
 * target x (a point), node index self (-1: not a node of T), om_x the
 * vorticity at x (used only when x is a vertex of T). */
int bso_pair(const double *x, int64_t self, const double *om_x, const double *tv, const double *tw,
             const int32_t *ids, int rule, int N, int M, int precheck, double *out)
{
    bso_tet T;
    double xyz[12], om[12];
    int32_t loc[4] = {0, 1, 2, 3};
    memcpy(xyz, tv, sizeof(xyz));
    memcpy(om, tw, sizeof(om));
    tet_setup(xyz, om, loc, &T);
    for (int j = 0; j < 4; ++j) T.id[j] = ids ? ids[j] : -2 - j;
    if (rule == BSO_RULE_RT) {
        int nl = N * M;
        double *s_tab = (double *)malloc(sizeof(double) * 4 * (size_t)nl);
        if (!s_tab) return -1;
        if (bso_angular_tables(N, M, s_tab, s_tab + 3 * nl)) {
            free(s_tab);
            return -1;
        }
        int64_t a = 0, b = 0, c = 0;
        ray_trace(x, self, om_x, &T, nl, s_tab, s_tab + 3 * nl, precheck, out, &a, &b, &c);
        free(s_tab);
        return 0;
    }
    double lam[44], w[11];
    int k = rule == BSO_RULE_G1 ? 1 : rule == BSO_RULE_G4 ? 4 : 11;
    bso_tet_rule(k, lam, w);
    gauss_rule(x, &T, k, lam, w, out);
    return 0;
}

int bso_num_threads(void)
{
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}
