/*
 * Oracle sparse Cholesky (test infrastructure only; never part of the product
 * path). Plain C, FP64, single-threaded, written for readability.
 *
 * The method factors one symmetric positive-definite matrix once and then
 * applies its inverse by a forward/backward substitution pair (Alg. 1, the
 * substitution pair; Alg. 2, LU_Decompose once before the time loop). For the
 * R-MATEX variant the factored matrix is C + gamma*G (Sec. 3.3.2); the DC and
 * F/P terms of Eq. 6 need G itself. Both are symmetric positive definite for
 * an RC grid with supply pads, so a Cholesky factor L L^T stands in for the
 * paper's LU.
 *
 * Ordering: recursive bisection by breadth-first level structures (a level
 * set of a BFS is a vertex separator), separators ordered last. It only
 * reduces fill; any ordering gives the same solution up to rounding.
 * Symbolic: elimination tree, then the row patterns of L from tree reaches.
 * Numeric: row-by-row ("up-looking") Cholesky, L stored by columns.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef struct {
    int64_t n;
    int64_t *colptr;   /* n+1 */
    int32_t *rowidx;   /* nnz; first entry of each column is the diagonal */
    double *val;       /* nnz */
    int32_t *perm;     /* new -> old */
    int32_t *iperm;    /* old -> new */
    int64_t nnz;
} orc_chol;

/* ---------------------------------------------------------------- ordering */

typedef struct {
    int64_t n;
    const int64_t *rp;
    const int32_t *ci;
    int32_t *mark;      /* region id per vertex; -1 = already ordered */
    int32_t *level;
    int32_t *queue;
    int32_t *out;       /* ordering being built (new -> old) */
    int64_t nout;
    int32_t next_region;
} nd_ctx;

/* BFS from s over vertices with mark == region; returns number reached,
 * fills queue in BFS order and level[]. */
static int64_t bfs(nd_ctx *c, int32_t s, int32_t region, int32_t *nlev)
{
    int64_t head = 0, tail = 0;
    c->queue[tail++] = s;
    c->level[s] = 0;
    int32_t maxl = 0;
    /* temporarily flip marks to region+1<<30 to mean "visited" */
    const int32_t vis = region | (1 << 30);
    c->mark[s] = vis;
    while (head < tail) {
        int32_t u = c->queue[head++];
        for (int64_t p = c->rp[u]; p < c->rp[u + 1]; ++p) {
            int32_t w = c->ci[p];
            if (c->mark[w] == region) {
                c->mark[w] = vis;
                c->level[w] = c->level[u] + 1;
                if (c->level[w] > maxl) maxl = c->level[w];
                c->queue[tail++] = w;
            }
        }
    }
    for (int64_t k = 0; k < tail; ++k) c->mark[c->queue[k]] = region;
    *nlev = maxl + 1;
    return tail;
}

static void emit(nd_ctx *c, const int32_t *v, int64_t cnt)
{
    for (int64_t k = 0; k < cnt; ++k) {
        c->out[c->nout++] = v[k];
        c->mark[v[k]] = -1;
    }
}

/* Order the connected set reachable from seed inside `region`. */
static void nd_component(nd_ctx *c, int32_t seed, int32_t region, int depth)
{
    int32_t nlev;
    int64_t cnt = bfs(c, seed, region, &nlev);
    if (cnt <= 48 || depth > 200) {
        int32_t *tmp = (int32_t *)malloc(sizeof(int32_t) * cnt);
        memcpy(tmp, c->queue, sizeof(int32_t) * cnt);
        emit(c, tmp, cnt);
        free(tmp);
        return;
    }
    /* pseudo-peripheral start: restart from the last vertex reached, twice */
    int32_t far = c->queue[cnt - 1];
    cnt = bfs(c, far, region, &nlev);
    far = c->queue[cnt - 1];
    cnt = bfs(c, far, region, &nlev);
    int32_t *verts = (int32_t *)malloc(sizeof(int32_t) * cnt);
    memcpy(verts, c->queue, sizeof(int32_t) * cnt);
    if (nlev < 3) {
        emit(c, verts, cnt);
        free(verts);
        return;
    }
    /* separator level: the first level at which half the vertices are reached */
    int64_t *lc = (int64_t *)calloc((size_t)nlev, sizeof(int64_t));
    for (int64_t k = 0; k < cnt; ++k) lc[c->level[verts[k]]]++;
    int64_t acc = 0;
    int32_t sep = 1;
    for (int32_t l = 0; l < nlev; ++l) {
        acc += lc[l];
        if (2 * acc >= cnt) { sep = l; break; }
    }
    if (sep == 0) sep = 1;
    if (sep == nlev - 1) sep = nlev - 2;
    free(lc);
    int32_t ra = c->next_region++, rb = c->next_region++;
    int64_t ns = 0;
    for (int64_t k = 0; k < cnt; ++k) {
        int32_t v = verts[k];
        int32_t l = c->level[v];
        if (l < sep) c->mark[v] = ra;
        else if (l > sep) c->mark[v] = rb;
        else verts[ns++] = v;     /* compact separator vertices in place */
    }
    /* each side may be disconnected: relabel and order every connected
     * piece of each side separately */
    {
        /* c->queue still holds the last BFS order of the whole component */
        int32_t *comp = (int32_t *)malloc(sizeof(int32_t) * cnt);
        memcpy(comp, c->queue, sizeof(int32_t) * cnt);
        for (int side = 0; side < 2; ++side) {
            int32_t r = side ? rb : ra;
            for (int64_t k = 0; k < cnt; ++k) {
                int32_t v = comp[k];
                if (c->mark[v] == r) {
                    int32_t sub = c->next_region++;
                    /* relabel the connected piece of region r containing v */
                    int64_t h = 0, t = 0;
                    int32_t *q = (int32_t *)malloc(sizeof(int32_t) * cnt);
                    q[t++] = v;
                    c->mark[v] = sub;
                    while (h < t) {
                        int32_t u = q[h++];
                        for (int64_t p = c->rp[u]; p < c->rp[u + 1]; ++p) {
                            int32_t w = c->ci[p];
                            if (c->mark[w] == r) { c->mark[w] = sub; q[t++] = w; }
                        }
                    }
                    free(q);
                    nd_component(c, v, sub, depth + 1);
                }
            }
        }
        free(comp);
    }
    emit(c, verts, ns);
    free(verts);
}

static void nd_order(int64_t n, const int64_t *rp, const int32_t *ci, int32_t *perm)
{
    nd_ctx c;
    c.n = n; c.rp = rp; c.ci = ci;
    c.mark = (int32_t *)malloc(sizeof(int32_t) * n);
    c.level = (int32_t *)malloc(sizeof(int32_t) * n);
    c.queue = (int32_t *)malloc(sizeof(int32_t) * n);
    c.out = perm;
    c.nout = 0;
    for (int64_t i = 0; i < n; ++i) c.mark[i] = 0;
    c.next_region = 1;
    for (int64_t i = 0; i < n; ++i) {
        if (c.mark[i] == 0) {
            int32_t r = c.next_region++;
            /* label the component of i as region r */
            int64_t h = 0, t = 0;
            c.queue[t++] = (int32_t)i;
            c.mark[i] = r;
            while (h < t) {
                int32_t u = c.queue[h++];
                for (int64_t p = rp[u]; p < rp[u + 1]; ++p) {
                    int32_t w = ci[p];
                    if (c.mark[w] == 0) { c.mark[w] = r; c.queue[t++] = w; }
                }
            }
            nd_component(&c, (int32_t)i, r, 0);
        }
    }
    free(c.mark); free(c.level); free(c.queue);
}

/* --------------------------------------------------------------- factor */

static int cmp_i32(const void *a, const void *b)
{
    int32_t x = *(const int32_t *)a, y = *(const int32_t *)b;
    return (x > y) - (x < y);
}

/*
 * A is given as full symmetric CSR (both triangles), rows/cols 0..n-1.
 * use_nd = 0 keeps the natural order (used by tests on tiny systems).
 * Returns 0 on success, -1 on allocation failure, k+1 if the pivot of
 * (permuted) column k is not positive.
 */
int orc_chol_factor(int64_t n, const int64_t *rp, const int32_t *ci, const double *av,
                    int use_nd, orc_chol **out)
{
    orc_chol *F = (orc_chol *)calloc(1, sizeof(orc_chol));
    if (!F) return -1;
    F->n = n;
    F->perm = (int32_t *)malloc(sizeof(int32_t) * n);
    F->iperm = (int32_t *)malloc(sizeof(int32_t) * n);
    if (use_nd) nd_order(n, rp, ci, F->perm);
    else for (int64_t i = 0; i < n; ++i) F->perm[i] = (int32_t)i;
    for (int64_t k = 0; k < n; ++k) F->iperm[F->perm[k]] = (int32_t)k;

    /* permuted matrix B = P A P^T, keep the upper part of each column:
     * B(i,k) with i <= k, i.e. for new column k, old row perm[k]'s entries. */
    int64_t *bp = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
    bp[0] = 0;
    for (int64_t k = 0; k < n; ++k) {
        int32_t o = F->perm[k];
        int64_t cnt = 0;
        for (int64_t p = rp[o]; p < rp[o + 1]; ++p)
            if (F->iperm[ci[p]] <= k) cnt++;
        bp[k + 1] = bp[k] + cnt;
    }
    int32_t *bi = (int32_t *)malloc(sizeof(int32_t) * bp[n]);
    double *bv = (double *)malloc(sizeof(double) * bp[n]);
    for (int64_t k = 0; k < n; ++k) {
        int32_t o = F->perm[k];
        int64_t q = bp[k];
        for (int64_t p = rp[o]; p < rp[o + 1]; ++p) {
            int32_t i = F->iperm[ci[p]];
            if (i <= k) { bi[q] = i; bv[q] = av[p]; q++; }
        }
    }

    /* elimination tree: parent[i] = min{ k > i : L(k,i) != 0 } */
    int32_t *parent = (int32_t *)malloc(sizeof(int32_t) * n);
    int32_t *anc = (int32_t *)malloc(sizeof(int32_t) * n);
    for (int64_t k = 0; k < n; ++k) {
        parent[k] = -1;
        anc[k] = -1;
        for (int64_t p = bp[k]; p < bp[k + 1]; ++p) {
            int32_t i = bi[p];
            /* climb from i to its current root, compressing to k */
            while (i != -1 && i < k) {
                int32_t next = anc[i];
                anc[i] = (int32_t)k;
                if (next == -1) { parent[i] = (int32_t)k; break; }
                i = next;
            }
        }
    }
    free(anc);

    /* column counts from the row patterns (reach of each row in the tree) */
    int32_t *flag = (int32_t *)malloc(sizeof(int32_t) * n);
    int64_t *cc = (int64_t *)calloc((size_t)n, sizeof(int64_t));
    for (int64_t k = 0; k < n; ++k) flag[k] = -1;
    for (int64_t k = 0; k < n; ++k) {
        flag[k] = (int32_t)k;
        cc[k] += 1; /* diagonal */
        for (int64_t p = bp[k]; p < bp[k + 1]; ++p) {
            int32_t i = bi[p];
            while (i < k && flag[i] != k) {
                flag[i] = (int32_t)k;
                cc[i] += 1;   /* L(k,i) != 0 */
                i = parent[i];
            }
        }
    }
    F->colptr = (int64_t *)malloc(sizeof(int64_t) * (n + 1));
    F->colptr[0] = 0;
    for (int64_t k = 0; k < n; ++k) F->colptr[k + 1] = F->colptr[k] + cc[k];
    F->nnz = F->colptr[n];
    F->rowidx = (int32_t *)malloc(sizeof(int32_t) * F->nnz);
    F->val = (double *)malloc(sizeof(double) * F->nnz);
    if (!F->rowidx || !F->val) return -1;

    /* numeric: row k of L solves L(0:k,0:k) l = B(0:k,k) */
    int64_t *fill = cc; /* reuse: next free slot per column */
    for (int64_t k = 0; k < n; ++k) fill[k] = F->colptr[k] + 1;
    double *x = (double *)calloc((size_t)n, sizeof(double));
    int32_t *pat = (int32_t *)malloc(sizeof(int32_t) * n);
    for (int64_t k = 0; k < n; ++k) flag[k] = -1;
    int status = 0;
    for (int64_t k = 0; k < n && !status; ++k) {
        int64_t np_ = 0;
        flag[k] = (int32_t)k;
        double d = 0.0;
        for (int64_t p = bp[k]; p < bp[k + 1]; ++p) {
            int32_t i = bi[p];
            if (i == k) { d += bv[p]; continue; }
            x[i] += bv[p];
            while (i < k && flag[i] != k) {
                flag[i] = (int32_t)k;
                pat[np_++] = i;
                i = parent[i];
            }
        }
        qsort(pat, (size_t)np_, sizeof(int32_t), cmp_i32);
        for (int64_t t = 0; t < np_; ++t) {
            int32_t j = pat[t];
            double lkj = x[j] / F->val[F->colptr[j]];
            x[j] = 0.0;
            for (int64_t p = F->colptr[j] + 1; p < fill[j]; ++p)
                x[F->rowidx[p]] -= F->val[p] * lkj;
            d -= lkj * lkj;
            F->rowidx[fill[j]] = (int32_t)k;
            F->val[fill[j]] = lkj;
            fill[j]++;
        }
        if (!(d > 0.0)) { status = (int)k + 1; break; }
        F->rowidx[F->colptr[k]] = (int32_t)k;
        F->val[F->colptr[k]] = sqrt(d);
    }
    free(x); free(pat); free(flag); free(cc); free(parent);
    free(bp); free(bi); free(bv);
    *out = F;
    return status;
}

/* b := A^{-1} b for nrhs right-hand sides stored column by column (stride n). */
void orc_chol_solve(const orc_chol *F, double *b, int64_t nrhs)
{
    int64_t n = F->n;
    double *y = (double *)malloc(sizeof(double) * n);
    for (int64_t r = 0; r < nrhs; ++r) {
        double *br = b + r * n;
        for (int64_t k = 0; k < n; ++k) y[k] = br[F->perm[k]];
        /* forward: L y = P b */
        for (int64_t j = 0; j < n; ++j) {
            double yj = y[j] / F->val[F->colptr[j]];
            y[j] = yj;
            for (int64_t p = F->colptr[j] + 1; p < F->colptr[j + 1]; ++p)
                y[F->rowidx[p]] -= F->val[p] * yj;
        }
        /* backward: L^T z = y */
        for (int64_t j = n - 1; j >= 0; --j) {
            double s = y[j];
            for (int64_t p = F->colptr[j] + 1; p < F->colptr[j + 1]; ++p)
                s -= F->val[p] * y[F->rowidx[p]];
            y[j] = s / F->val[F->colptr[j]];
        }
        for (int64_t k = 0; k < n; ++k) br[F->perm[k]] = y[k];
    }
    free(y);
}

int64_t orc_chol_nnz(const orc_chol *F) { return F->nnz; }

/* Copy out the factor (for tests on small systems): colptr[n+1], rowidx, val, perm. */
void orc_chol_export(const orc_chol *F, int64_t *colptr, int32_t *rowidx, double *val,
                     int32_t *perm)
{
    memcpy(colptr, F->colptr, sizeof(int64_t) * (F->n + 1));
    memcpy(rowidx, F->rowidx, sizeof(int32_t) * F->nnz);
    memcpy(val, F->val, sizeof(double) * F->nnz);
    memcpy(perm, F->perm, sizeof(int32_t) * F->n);
}

void orc_chol_free(orc_chol *F)
{
    if (!F) return;
    free(F->colptr); free(F->rowidx); free(F->val); free(F->perm); free(F->iperm);
    free(F);
}
