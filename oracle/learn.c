/*
 * CPU oracle for the learned branching rule.  TEST INFRASTRUCTURE ONLY (see
 * oracle.h): it produces the training traces and is the FP64 reference the
 * GPU feature, inference and training kernels are checked against.  It
 * shares no code with the product.
 *
 * The paper leaves the search strategy open (§5, Evaluation).  The learned
 * rule scores every unfixed decision variable with a small network over six
 * features of its interval and its constraints, and branches on the best
 * score; first-fail is its fallback.  Definitions (decision variable x with
 * initial interval [lo, hi], H = max(1, hi - lo)):
 *   f0 = (lb(x) - lo) / H
 *   f1 = (ub(x) - lo) / H
 *   f2 = (ub(x) - lb(x)) / H
 *   f3 = deg(x) / max(1, max_v deg(v)); deg(v) = number of linear rows plus
 *        reified items (as b, si or sj) that contain v
 *   f4 = min(1, min over rows x - y <= c (two terms, +1 on x, -1 on y) of
 *        (c + ub(y) - lb(x)) / H), or 1 without such a row: the slack of
 *        the tightest precedence leaving x
 *   f5 = sl(x) + cnt(x) / max(1, N(x)), N(x) = number of reified items with
 *        si = x, cnt(x) = those with lb(b) >= 1, and sl(x) =
 *        (1 / max(1, N(x))) * sum over those items of d * w(b) / H, with
 *        w(b) = sum over rows containing b with coefficient a > 0 and
 *        rhs c > 0 of a / c (the task's demand/capacity energy when b is a
 *        resource-usage term)
 * Network: z = W1 x + b1 (64 hidden units), h = max(0, z), s = w2 . h + b2.
 * Parameter vector (513 values): W1[k][f] at k*6+f, b1 at 384+k, w2 at
 * 448+k, b2 at 512.
 * Expert label of a node: for each candidate, propagate both children
 * (x = lb(x) and x >= lb(x) + 1); score = sum over the two children of
 * (1e6 if the child fails, else log(1 + total width removed over all
 * variables)); the label is the candidate with the largest score (ties to
 * the earliest).  The training loss is the mean over nodes of the
 * cross-entropy between a target distribution over the node's candidates
 * and the softmax of their scores (a one-hot target on the label, or a
 * softmax of the expert scores).
 */
#include "oracle.h"

#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

int32_t orc_propagate_validated(const orc_model *m, int32_t *lb, int32_t *ub,
                                int32_t sched, uint64_t seed, int64_t *sweeps);

#define NF 6
#define NH 64
#define NP (NH * NF + NH + NH + 1)

/* ------------------------------------------------------------- features */
typedef struct {
    int32_t D;
    double *H, *lo, *degn, *sl, *invN;
    int32_t *pr;            /* CSR per decision var: rows x - y <= c       */
    int32_t *ry, *rc;
    int32_t *pb;            /* CSR per decision var: b of items with si = x */
    int32_t *rb;
} fstatic;

static void fstatic_free(fstatic *S)
{
    free(S->H); free(S->lo); free(S->degn); free(S->sl); free(S->invN);
    free(S->pr); free(S->ry); free(S->rc); free(S->pb); free(S->rb);
}

/* is row r of the form x - y <= c?  returns x (and y, c) or -1 */
static int32_t diff_row(const orc_model *m, int32_t r, int32_t *y, int32_t *c)
{
    int32_t a0 = m->row_ptr[r];
    if (m->row_ptr[r + 1] - a0 != 2) return -1;
    *c = m->rhs[r];
    if (m->coef[a0] == 1 && m->coef[a0 + 1] == -1) { *y = m->var[a0 + 1]; return m->var[a0]; }
    if (m->coef[a0] == -1 && m->coef[a0 + 1] == 1) { *y = m->var[a0]; return m->var[a0 + 1]; }
    return -1;
}

static void fstatic_build(const orc_model *m, fstatic *S)
{
    const int32_t V = m->nvars, D = m->ndec;
    S->D = D;
    double *deg = (double *)calloc((size_t)V + 1, sizeof(double));
    double *w = (double *)calloc((size_t)V + 1, sizeof(double));
    for (int32_t r = 0; r < m->nrows; ++r)
        for (int32_t t = m->row_ptr[r]; t < m->row_ptr[r + 1]; ++t) {
            deg[m->var[t]] += 1.0;
            if (m->coef[t] > 0 && m->rhs[r] > 0)
                w[m->var[t]] += (double)m->coef[t] / (double)m->rhs[r];
        }
    for (int32_t q = 0; q < m->nreif; ++q)
        for (int k = 0; k < 3; ++k)
            deg[m->reif[4 * (int64_t)q + k]] += 1.0;
    double maxdeg = 1.0;
    for (int32_t v = 0; v < V; ++v)
        if (deg[v] > maxdeg) maxdeg = deg[v];

    int32_t *pos = (int32_t *)malloc(sizeof(int32_t) * ((size_t)V + 1));
    for (int32_t v = 0; v < V; ++v) pos[v] = -1;
    for (int32_t q = 0; q < D; ++q) pos[m->dec[q]] = q;

    S->H = (double *)calloc((size_t)D + 1, sizeof(double));
    S->lo = (double *)calloc((size_t)D + 1, sizeof(double));
    S->degn = (double *)calloc((size_t)D + 1, sizeof(double));
    S->sl = (double *)calloc((size_t)D + 1, sizeof(double));
    S->invN = (double *)calloc((size_t)D + 1, sizeof(double));
    S->pr = (int32_t *)calloc((size_t)D + 1, sizeof(int32_t));
    S->pb = (int32_t *)calloc((size_t)D + 1, sizeof(int32_t));
    int32_t y, c;
    for (int32_t r = 0; r < m->nrows; ++r) {
        int32_t x = diff_row(m, r, &y, &c);
        if (x >= 0 && pos[x] >= 0) S->pr[pos[x] + 1]++;
    }
    for (int32_t q = 0; q < m->nreif; ++q) {
        int32_t si = m->reif[4 * (int64_t)q + 1];
        if (pos[si] >= 0) S->pb[pos[si] + 1]++;
    }
    for (int32_t q = 0; q < D; ++q) {
        S->pr[q + 1] += S->pr[q];
        S->pb[q + 1] += S->pb[q];
    }
    S->ry = (int32_t *)malloc(sizeof(int32_t) * ((size_t)S->pr[D] + 1));
    S->rc = (int32_t *)malloc(sizeof(int32_t) * ((size_t)S->pr[D] + 1));
    S->rb = (int32_t *)malloc(sizeof(int32_t) * ((size_t)S->pb[D] + 1));
    int32_t *fill = (int32_t *)calloc((size_t)D + 1, sizeof(int32_t));
    for (int32_t r = 0; r < m->nrows; ++r) {
        int32_t x = diff_row(m, r, &y, &c);
        if (x >= 0 && pos[x] >= 0) {
            int32_t q = pos[x], k = S->pr[q] + fill[q]++;
            S->ry[k] = y;
            S->rc[k] = c;
        }
    }
    memset(fill, 0, sizeof(int32_t) * ((size_t)D + 1));
    for (int32_t q = 0; q < D; ++q) S->sl[q] = 0.0;
    for (int32_t it = 0; it < m->nreif; ++it) {
        const int32_t *e = m->reif + 4 * (int64_t)it;
        if (pos[e[1]] >= 0) {
            int32_t q = pos[e[1]], k = S->pb[q] + fill[q]++;
            S->rb[k] = e[0];
            S->sl[q] += (double)e[3] * w[e[0]];
        }
    }
    for (int32_t q = 0; q < D; ++q) {
        int32_t x = m->dec[q];
        double H = (double)m->ub0[x] - (double)m->lb0[x];
        if (H < 1.0) H = 1.0;
        int32_t N = S->pb[q + 1] - S->pb[q];
        S->H[q] = H;
        S->lo[q] = (double)m->lb0[x];
        S->degn[q] = deg[x] / maxdeg;
        S->invN[q] = 1.0 / (N > 1 ? (double)N : 1.0);
        S->sl[q] = S->sl[q] * S->invN[q] / H;
    }
    free(fill);
    free(pos);
    free(deg);
    free(w);
}

static void features_of(const fstatic *S, const orc_model *m, const int32_t *lb,
                        const int32_t *ub, int32_t q, double *f)
{
    const int32_t x = m->dec[q];
    const double H = S->H[q];
    f[0] = ((double)lb[x] - S->lo[q]) / H;
    f[1] = ((double)ub[x] - S->lo[q]) / H;
    f[2] = ((double)ub[x] - (double)lb[x]) / H;
    f[3] = S->degn[q];
    double slack = 1.0;
    for (int32_t k = S->pr[q]; k < S->pr[q + 1]; ++k) {
        double s = ((double)S->rc[k] + (double)ub[S->ry[k]] - (double)lb[x]) / H;
        if (s < slack) slack = s;
    }
    f[4] = slack;
    int32_t cnt = 0;
    for (int32_t k = S->pb[q]; k < S->pb[q + 1]; ++k)
        cnt += lb[S->rb[k]] >= 1;
    f[5] = S->sl[q] + (double)cnt * S->invN[q];
}

int32_t orc_features(const orc_model *m, const int32_t *lb, const int32_t *ub, double *out)
{
    int32_t rc = orc_validate(m);
    if (rc) return rc;
    fstatic S;
    fstatic_build(m, &S);
    for (int32_t q = 0; q < m->ndec; ++q)
        features_of(&S, m, lb, ub, q, out + (int64_t)q * NF);
    fstatic_free(&S);
    return 0;
}

/* ------------------------------------------------------------- network */
static double mlp_score(const double *p, const double *x, double *z)
{
    double s = p[NH * NF + 2 * NH];
    for (int k = 0; k < NH; ++k) {
        double a = p[NH * NF + k];
        for (int f = 0; f < NF; ++f) a += p[k * NF + f] * x[f];
        if (z) z[k] = a;
        s += p[NH * NF + NH + k] * (a > 0.0 ? a : 0.0);
    }
    return s;
}

int32_t orc_mlp_forward(const double *p, const double *x, int64_t ncand, double *scores)
{
    for (int64_t c = 0; c < ncand; ++c)
        scores[c] = mlp_score(p, x + c * NF, NULL);
    return 0;
}

/* mean over nodes of the cross-entropy between the target distribution t
 * (per candidate, summing to 1 over each node) and the softmax of the
 * node's scores: logsumexp(s) - sum_c t_c s_c; gradient into g (NP) */
int32_t orc_mlp_loss_grad(const double *p, const double *x, const int32_t *node_off,
                          const double *t, int32_t nnodes, double *loss, double *g)
{
    memset(g, 0, sizeof(double) * NP);
    double L = 0.0;
    int32_t maxc = 0;
    for (int32_t i = 0; i < nnodes; ++i)
        if (node_off[i + 1] - node_off[i] > maxc) maxc = node_off[i + 1] - node_off[i];
    double *s = (double *)malloc(sizeof(double) * ((size_t)maxc + 1));
    double *z = (double *)malloc(sizeof(double) * (size_t)NH * ((size_t)maxc + 1));
    for (int32_t i = 0; i < nnodes; ++i) {
        const int32_t c0 = node_off[i], nc = node_off[i + 1] - c0;
        if (nc <= 0) continue;
        double mx = -INFINITY;
        for (int32_t c = 0; c < nc; ++c) {
            s[c] = mlp_score(p, x + (int64_t)(c0 + c) * NF, z + (int64_t)c * NH);
            if (s[c] > mx) mx = s[c];
        }
        double se = 0.0, ts = 0.0;
        for (int32_t c = 0; c < nc; ++c) {
            se += exp(s[c] - mx);
            ts += t[c0 + c] * s[c];
        }
        L += (mx + log(se)) - ts;
        for (int32_t c = 0; c < nc; ++c) {
            /* dL_i/ds_c = softmax_c - t_c, averaged over nodes */
            double gs = (exp(s[c] - mx) / se - t[c0 + c]) / (double)nnodes;
            const double *xc = x + (int64_t)(c0 + c) * NF;
            const double *zc = z + (int64_t)c * NH;
            g[NH * NF + 2 * NH] += gs;
            for (int k = 0; k < NH; ++k) {
                double h = zc[k] > 0.0 ? zc[k] : 0.0;
                g[NH * NF + NH + k] += gs * h;
                if (zc[k] > 0.0) {
                    double dz = gs * p[NH * NF + NH + k];
                    g[NH * NF + k] += dz;
                    for (int f = 0; f < NF; ++f) g[k * NF + f] += dz * xc[f];
                }
            }
        }
    }
    *loss = L / (double)(nnodes > 0 ? nnodes : 1);
    free(s);
    free(z);
    return 0;
}

/* ------------------------------------------------------------- traces */
typedef struct {
    const orc_model *m;
    fstatic S;
    int64_t node_limit, nodes;
    int32_t mode;
    int32_t best;
    /* output */
    float *feat;
    double *score;
    int32_t *cand, *off, *label;
    int64_t cap_nodes, cap_cand, nrec, ncand_tot;
    int full;
} tctx;

static int64_t total_width(const orc_model *m, const int32_t *lb, const int32_t *ub)
{
    int64_t w = 0;
    for (int32_t v = 0; v < m->nvars; ++v) w += (int64_t)ub[v] - lb[v];
    return w;
}

static void record_node(tctx *T, const int32_t *lb, const int32_t *ub)
{
    const orc_model *m = T->m;
    int32_t nc = 0;
    for (int32_t q = 0; q < m->ndec; ++q)
        nc += ub[m->dec[q]] > lb[m->dec[q]];
    if (nc < 2) return;                              /* no choice to learn */
    if (T->nrec >= T->cap_nodes || T->ncand_tot + nc > T->cap_cand) { T->full = 1; return; }
    const size_t bytes = sizeof(int32_t) * (size_t)m->nvars;
    int32_t *clb = (int32_t *)malloc(bytes), *cub = (int32_t *)malloc(bytes);
    const int64_t w0 = total_width(m, lb, ub);
    double best = -1.0;
    int32_t best_i = 0, i = 0;
    double f[NF];
    for (int32_t q = 0; q < m->ndec; ++q) {
        const int32_t x = m->dec[q];
        if (ub[x] <= lb[x]) continue;
        features_of(&T->S, m, lb, ub, q, f);
        for (int k = 0; k < NF; ++k)
            T->feat[(T->ncand_tot + i) * NF + k] = (float)f[k];
        T->cand[T->ncand_tot + i] = q;
        double score = 0.0;
        for (int side = 0; side < 2; ++side) {
            memcpy(clb, lb, bytes);
            memcpy(cub, ub, bytes);
            if (side == 0) cub[x] = lb[x]; else clb[x] = lb[x] + 1;
            int32_t st = orc_propagate_validated(m, clb, cub, ORC_SCHED_GS, 0, NULL);
            if (st != ORC_FIXPOINT) score += 1e6;
            else score += log(1.0 + (double)(w0 - total_width(m, clb, cub)));
        }
        if (T->score) T->score[T->ncand_tot + i] = score;
        if (score > best) { best = score; best_i = i; }
        ++i;
    }
    T->label[T->nrec] = best_i;
    T->off[T->nrec] = (int32_t)T->ncand_tot;
    T->ncand_tot += nc;
    T->off[T->nrec + 1] = (int32_t)T->ncand_tot;
    T->nrec += 1;
    free(clb);
    free(cub);
}

/* The expert's choice at a propagated node: the decision-list position of
 * the candidate with the largest strong-branching score (see above), or -1
 * if every decision variable is fixed. */
int32_t orc_expert_choice(const orc_model *m, const int32_t *lb, const int32_t *ub)
{
    const size_t bytes = sizeof(int32_t) * (size_t)(m->nvars > 0 ? m->nvars : 1);
    int32_t *clb = (int32_t *)malloc(bytes), *cub = (int32_t *)malloc(bytes);
    const int64_t w0 = total_width(m, lb, ub);
    double best = -1.0;
    int32_t pick = -1;
    for (int32_t q = 0; q < m->ndec; ++q) {
        const int32_t x = m->dec[q];
        if (ub[x] <= lb[x]) continue;
        double score = 0.0;
        for (int side = 0; side < 2; ++side) {
            memcpy(clb, lb, sizeof(int32_t) * (size_t)m->nvars);
            memcpy(cub, ub, sizeof(int32_t) * (size_t)m->nvars);
            if (side == 0) cub[x] = lb[x]; else clb[x] = lb[x] + 1;
            int32_t st = orc_propagate_validated(m, clb, cub, ORC_SCHED_GS, 0, NULL);
            if (st != ORC_FIXPOINT) score += 1e6;
            else score += log(1.0 + (double)(w0 - total_width(m, clb, cub)));
        }
        if (score > best) { best = score; pick = q; }
    }
    free(clb);
    free(cub);
    return pick;
}

/* The network's choice at a propagated node: the decision-list position of
 * the unfixed candidate with the largest score under parameters p (ties to
 * the earliest), or -1 if every decision variable is fixed. */
int32_t orc_mlp_choice(const orc_model *m, const double *p, const int32_t *lb, const int32_t *ub)
{
    fstatic S;
    fstatic_build(m, &S);
    double f[NF], best = -INFINITY;
    int32_t pick = -1;
    for (int32_t q = 0; q < m->ndec; ++q) {
        const int32_t x = m->dec[q];
        if (ub[x] <= lb[x]) continue;
        features_of(&S, m, lb, ub, q, f);
        const double sc = mlp_score(p, f, NULL);
        if (pick < 0 || sc > best) { best = sc; pick = q; }
    }
    fstatic_free(&S);
    return pick;
}

static void trace_dfs(tctx *T, const int32_t *plb, const int32_t *pub)
{
    const orc_model *m = T->m;
    if (T->nodes >= T->node_limit || T->full) return;
    const size_t bytes = sizeof(int32_t) * (size_t)(m->nvars > 0 ? m->nvars : 1);
    int32_t *lb = (int32_t *)malloc(bytes), *ub = (int32_t *)malloc(bytes);
    memcpy(lb, plb, sizeof(int32_t) * (size_t)m->nvars);
    memcpy(ub, pub, sizeof(int32_t) * (size_t)m->nvars);
    T->nodes += 1;
    if (T->mode == ORC_MINIMIZE && T->best != INT32_MAX && T->best - 1 < ub[m->objective])
        ub[m->objective] = T->best - 1;
    if (orc_propagate_validated(m, lb, ub, ORC_SCHED_GS, 0, NULL) == ORC_FIXPOINT) {
        int32_t pick = -1;
        int64_t wbest = 0;
        for (int32_t q = 0; q < m->ndec; ++q) {     /* first-fail drives the search */
            int64_t w = (int64_t)ub[m->dec[q]] - lb[m->dec[q]];
            if (w > 0 && (pick < 0 || w < wbest)) { pick = q; wbest = w; }
        }
        if (pick < 0) {
            if (T->mode == ORC_MINIMIZE && lb[m->objective] < T->best)
                T->best = lb[m->objective];
        } else {
            record_node(T, lb, ub);
            const int32_t x = m->dec[pick], val = lb[x], keep = ub[x];
            ub[x] = val;
            trace_dfs(T, lb, ub);
            ub[x] = keep;
            lb[x] = val + 1;
            trace_dfs(T, lb, ub);
        }
    }
    free(lb);
    free(ub);
}

/* Search traces: depth-first with first-fail (and branch-and-bound when
 * mode is ORC_MINIMIZE) for at most node_limit nodes; every propagated,
 * non-failed node with at least two unfixed decision variables is
 * recorded: its candidates' features (feat: NF floats each), their
 * expert scores (score, may be NULL), their decision-list positions (cand),
 * the node's candidate range
 * [off[i], off[i+1]) and the expert label (an index within the range).
 * Returns the number of recorded nodes (*ncand receives the number of
 * candidates), or a negative error. */
int64_t orc_trace(const orc_model *m, int32_t mode, int64_t node_limit, float *feat,
                  double *score, int32_t *cand, int32_t *off, int32_t *label, int64_t cap_nodes,
                  int64_t cap_cand, int64_t *ncand)
{
    int32_t rc = orc_validate(m);
    if (rc) return rc;
    if (mode == ORC_MINIMIZE && m->objective < 0) return -1;
    tctx T;
    memset(&T, 0, sizeof(T));
    T.m = m;
    T.node_limit = node_limit;
    T.mode = mode;
    T.best = INT32_MAX;
    T.feat = feat;
    T.score = score;
    T.cand = cand;
    T.off = off;
    T.label = label;
    T.cap_nodes = cap_nodes;
    T.cap_cand = cap_cand;
    fstatic_build(m, &T.S);
    off[0] = 0;
    trace_dfs(&T, m->lb0, m->ub0);
    fstatic_free(&T.S);
    if (ncand) *ncand = T.ncand_tot;
    return T.nrec;
}

/* One step of Adam (Kingma and Ba 2015), the optimiser of the training
 * loop, in double precision: with beta1 = 0.9, beta2 = 0.999, eps = 1e-8,
 *   m <- beta1 m + (1 - beta1) g,   v <- beta2 v + (1 - beta2) g^2,
 *   p <- p - lr * (m / (1 - beta1^t)) / (sqrt(v / (1 - beta2^t)) + eps)
 * for step t >= 1 (m and v start at 0). */
int32_t orc_adam_step(double *p, const double *g, double *m, double *v, int32_t n, double lr,
                      int32_t step)
{
    if (!p || !g || !m || !v || n < 0 || step < 1) return -1;
    const double b1 = 0.9, b2 = 0.999, eps = 1e-8;
    const double c1 = 1.0 - pow(b1, (double)step), c2 = 1.0 - pow(b2, (double)step);
    for (int32_t i = 0; i < n; ++i) {
        m[i] = b1 * m[i] + (1.0 - b1) * g[i];
        v[i] = b2 * v[i] + (1.0 - b2) * g[i] * g[i];
        p[i] -= lr * (m[i] / c1) / (sqrt(v[i] / c2) + eps);
    }
    return 0;
}
