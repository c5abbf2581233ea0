/*
 * geometry.c -- host-side construction of the inputs of the selection hot path.
 *
 * Nothing here evaluates a covariance or takes a selection decision: it only
 * orders points and finds nearest neighbours, i.e. it builds the
 * ordering (Sec. 2.2, eq. maximin) and the candidate sets (Sec. 4, nearest
 * later-ordered neighbours) that both the GPU path and the CPU oracle consume.
 *
 * Coordinates are row-major [n][d] doubles, d <= 3.  Point ids are int32.
 * All entry points are plain C so Python can call them through ctypes.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define LEAF 12
#define MAXD 3

/* ------------------------------------------------------------------------ */
/* static kd-tree over a subset of points (ids [id0, id0 + n))               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int d;
    const double *x;  /* full coordinate array, [*][d] */
    int32_t *perm;    /* point ids in tree order */
    int32_t n;
    int32_t nnodes;
    int32_t *lo, *hi, *left, *right;
    double *bmin, *bmax; /* [node][MAXD] */
} kdtree;

static double coord(const kdtree *t, int32_t id, int k) { return t->x[(int64_t)id * t->d + k]; }

static void select_nth(kdtree *t, int32_t lo, int32_t hi, int32_t nth, int dim) {
    /* quickselect on perm[lo..hi) by coordinate dim, ties by id (deterministic) */
    int32_t *p = t->perm;
    while (hi - lo > 1) {
        int32_t mid = lo + (hi - lo) / 2;
        int32_t pid = p[mid];
        double pv = coord(t, pid, dim);
        int32_t tmp = p[mid]; p[mid] = p[hi - 1]; p[hi - 1] = tmp;
        int32_t store = lo;
        for (int32_t i = lo; i < hi - 1; ++i) {
            double v = coord(t, p[i], dim);
            if (v < pv || (v == pv && p[i] < pid)) {
                tmp = p[i]; p[i] = p[store]; p[store] = tmp;
                ++store;
            }
        }
        tmp = p[store]; p[store] = p[hi - 1]; p[hi - 1] = tmp;
        if (store == nth) return;
        if (nth < store) hi = store; else lo = store + 1;
    }
}

static int32_t build_node(kdtree *t, int32_t lo, int32_t hi) {
    int32_t me = t->nnodes++;
    t->lo[me] = lo; t->hi[me] = hi; t->left[me] = -1; t->right[me] = -1;
    double *mn = t->bmin + (int64_t)me * MAXD, *mx = t->bmax + (int64_t)me * MAXD;
    for (int k = 0; k < t->d; ++k) { mn[k] = INFINITY; mx[k] = -INFINITY; }
    for (int32_t i = lo; i < hi; ++i)
        for (int k = 0; k < t->d; ++k) {
            double v = coord(t, t->perm[i], k);
            if (v < mn[k]) mn[k] = v;
            if (v > mx[k]) mx[k] = v;
        }
    if (hi - lo <= LEAF) return me;
    int dim = 0; double w = -1.0;
    for (int k = 0; k < t->d; ++k) if (mx[k] - mn[k] > w) { w = mx[k] - mn[k]; dim = k; }
    int32_t mid = lo + (hi - lo) / 2;
    select_nth(t, lo, hi, mid, dim);
    int32_t l = build_node(t, lo, mid);
    int32_t r = build_node(t, mid, hi);
    t->left[me] = l; t->right[me] = r;
    return me;
}

static void kd_build(kdtree *t, const double *x, int d, int32_t id0, int32_t n) {
    t->d = d; t->x = x; t->n = n; t->nnodes = 0;
    t->perm = (int32_t *)malloc(sizeof(int32_t) * (size_t)(n > 0 ? n : 1));
    for (int32_t i = 0; i < n; ++i) t->perm[i] = id0 + i;
    int32_t cap = 4 * (n / (LEAF / 2) + 2);
    t->lo = (int32_t *)malloc(sizeof(int32_t) * cap);
    t->hi = (int32_t *)malloc(sizeof(int32_t) * cap);
    t->left = (int32_t *)malloc(sizeof(int32_t) * cap);
    t->right = (int32_t *)malloc(sizeof(int32_t) * cap);
    t->bmin = (double *)malloc(sizeof(double) * (size_t)cap * MAXD);
    t->bmax = (double *)malloc(sizeof(double) * (size_t)cap * MAXD);
    if (n > 0) build_node(t, 0, n);
}

static void kd_free(kdtree *t) {
    free(t->perm); free(t->lo); free(t->hi); free(t->left); free(t->right); free(t->bmin); free(t->bmax);
}

static double box_d2(const kdtree *t, int32_t node, const double *q) {
    const double *mn = t->bmin + (int64_t)node * MAXD, *mx = t->bmax + (int64_t)node * MAXD;
    double s = 0.0;
    for (int k = 0; k < t->d; ++k) {
        double e = 0.0;
        if (q[k] < mn[k]) e = mn[k] - q[k]; else if (q[k] > mx[k]) e = q[k] - mx[k];
        s += e * e;
    }
    return s;
}

static double pt_d2(const kdtree *t, int32_t id, const double *q) {
    double s = 0.0;
    for (int k = 0; k < t->d; ++k) { double e = coord(t, id, k) - q[k]; s += e * e; }
    return s;
}

/* ------------------------------------------------------------------------ */
/* bounded max-heap of (d2, id): worst (largest d2, then largest id) on top */
/* ------------------------------------------------------------------------ */
typedef struct { double d2; int32_t id; } nbr;

static int nbr_worse(nbr a, nbr b) { return a.d2 > b.d2 || (a.d2 == b.d2 && a.id > b.id); }

static void heap_push(nbr *h, int32_t *sz, int32_t cap, nbr v) {
    if (*sz < cap) {
        int32_t i = (*sz)++;
        h[i] = v;
        while (i > 0) {
            int32_t p = (i - 1) / 2;
            if (!nbr_worse(h[i], h[p])) break;
            nbr tmp = h[i]; h[i] = h[p]; h[p] = tmp; i = p;
        }
    } else if (nbr_worse(h[0], v)) {
        int32_t i = 0; h[0] = v;
        for (;;) {
            int32_t l = 2 * i + 1, r = l + 1, m = i;
            if (l < *sz && nbr_worse(h[l], h[m])) m = l;
            if (r < *sz && nbr_worse(h[r], h[m])) m = r;
            if (m == i) break;
            nbr tmp = h[i]; h[i] = h[m]; h[m] = tmp; i = m;
        }
    }
}

static int nbr_cmp(const void *a, const void *b) {
    const nbr *x = (const nbr *)a, *y = (const nbr *)b;
    if (x->d2 < y->d2) return -1;
    if (x->d2 > y->d2) return 1;
    return (x->id > y->id) - (x->id < y->id);
}

/* filter: id > min_id and (ell == NULL or ell[id] <= ell_max) and (taken == NULL or !taken[id]) */
typedef struct { int32_t min_id; const double *ell; double ell_max; const uint8_t *taken; } kfilter;

static int accept(const kfilter *f, int32_t id) {
    if (id <= f->min_id) return 0;
    if (f->ell && !(f->ell[id] <= f->ell_max)) return 0;
    if (f->taken && f->taken[id]) return 0;
    return 1;
}

/* k nearest accepted points of q; fills h (unsorted), returns count */
static int32_t kd_knn(const kdtree *t, const double *q, int32_t k, const kfilter *f, nbr *h, int32_t *stack) {
    int32_t sz = 0, top = 0;
    if (t->n == 0 || k <= 0) return 0;
    stack[top++] = 0;
    while (top > 0) {
        int32_t node = stack[--top];
        if (sz == k && box_d2(t, node, q) > h[0].d2) continue;
        if (t->left[node] < 0) {
            for (int32_t i = t->lo[node]; i < t->hi[node]; ++i) {
                int32_t id = t->perm[i];
                if (!accept(f, id)) continue;
                nbr v = {pt_d2(t, id, q), id};
                heap_push(h, &sz, k, v);
            }
        } else {
            int32_t l = t->left[node], r = t->right[node];
            double dl = box_d2(t, l, q), dr = box_d2(t, r, q);
            /* push the farther child first so the nearer one is visited first */
            if (dl <= dr) { stack[top++] = r; stack[top++] = l; }
            else { stack[top++] = l; stack[top++] = r; }
        }
    }
    return sz;
}

/* ------------------------------------------------------------------------ */
/* reverse-maximin ordering (Sec. 2.2, eq. maximin), p = 1                    */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t *heap, *where; double *key; int32_t n; } maxheap;

static int mh_before(const maxheap *m, int32_t a, int32_t b) {
    return m->key[a] > m->key[b] || (m->key[a] == m->key[b] && a < b);
}
static void mh_swap(maxheap *m, int32_t i, int32_t j) {
    int32_t a = m->heap[i], b = m->heap[j];
    m->heap[i] = b; m->heap[j] = a; m->where[b] = i; m->where[a] = j;
}
static void mh_down(maxheap *m, int32_t i) {
    for (;;) {
        int32_t l = 2 * i + 1, r = l + 1, best = i;
        if (l < m->n && mh_before(m, m->heap[l], m->heap[best])) best = l;
        if (r < m->n && mh_before(m, m->heap[r], m->heap[best])) best = r;
        if (best == i) return;
        mh_swap(m, i, best); i = best;
    }
}

/* order[pos] = point id; ell[pos] = distance of that point to all later points
 * (infinity for the last one).  The last point is point 0; ties go to the
 * smaller id. */
int csel_geo_reverse_maximin(const double *x, int32_t n, int32_t d, int32_t *order, double *ell) {
    if (n <= 0 || d < 1 || d > MAXD) return -1;
    kdtree t; kd_build(&t, x, d, 0, n);
    double *dist2 = (double *)malloc(sizeof(double) * n);
    uint8_t *done = (uint8_t *)calloc(n, 1);
    maxheap m; m.heap = (int32_t *)malloc(sizeof(int32_t) * n); m.where = (int32_t *)malloc(sizeof(int32_t) * n);
    m.key = dist2; m.n = 0;
    const double *x0 = x;
    for (int32_t j = 0; j < n; ++j) {
        double s = 0.0;
        for (int k = 0; k < d; ++k) { double e = x[(int64_t)j * d + k] - x0[k]; s += e * e; }
        dist2[j] = s;
    }
    order[n - 1] = 0; ell[n - 1] = INFINITY; done[0] = 1;
    for (int32_t j = 1; j < n; ++j) { m.heap[m.n] = j; m.where[j] = m.n; m.n++; }
    m.where[0] = -1;
    for (int32_t i = m.n / 2 - 1; i >= 0; --i) mh_down(&m, i);
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (t.nnodes + 8));
    for (int32_t pos = n - 2; pos >= 0; --pos) {
        int32_t p = m.heap[0];
        mh_swap(&m, 0, m.n - 1); m.n--; m.where[p] = -1;
        if (m.n > 0) mh_down(&m, 0);
        order[pos] = p; ell[pos] = sqrt(dist2[p]); done[p] = 1;
        double r2 = dist2[p];
        const double *q = x + (int64_t)p * d;
        int32_t top = 0; stack[top++] = 0;
        while (top > 0) {
            int32_t node = stack[--top];
            if (box_d2(&t, node, q) >= r2) continue;
            if (t.left[node] < 0) {
                for (int32_t i = t.lo[node]; i < t.hi[node]; ++i) {
                    int32_t j = t.perm[i];
                    if (done[j]) continue;
                    double dd = pt_d2(&t, j, q);
                    if (dd < dist2[j]) {
                        dist2[j] = dd;
                        mh_down(&m, m.where[j]); /* key decreased in a max-heap */
                    }
                }
            } else { stack[top++] = t.left[node]; stack[top++] = t.right[node]; }
        }
    }
    free(stack); free(m.heap); free(m.where); free(done); free(dist2); kd_free(&t);
    return 0;
}

/* ------------------------------------------------------------------------ */
/* chunked "later" trees: tree c covers ids [a_c, n); used for queries that   */
/* only accept ids above some threshold                                       */
/* ------------------------------------------------------------------------ */
typedef struct { int32_t nchunks; int32_t *a; kdtree *trees; } laterforest;

static void forest_build(laterforest *F, const double *x, int32_t n, int32_t d) {
    int32_t cap = 8, cnt = 0;
    int32_t *starts = (int32_t *)malloc(sizeof(int32_t) * cap);
    int32_t b = n;
    while (b > 0) {
        int32_t m = (n - b) / 4; if (m < 64) m = 64;
        int32_t a = b - m; if (a < 0) a = 0;
        if (cnt == cap) { cap *= 2; starts = (int32_t *)realloc(starts, sizeof(int32_t) * cap); }
        starts[cnt++] = a; b = a;
    }
    F->nchunks = cnt; F->a = starts;
    F->trees = (kdtree *)malloc(sizeof(kdtree) * cnt);
#pragma omp parallel for schedule(dynamic, 1)
    for (int32_t c = 0; c < cnt; ++c) kd_build(&F->trees[c], x, d, starts[c], n - starts[c]);
}

static void forest_free(laterforest *F) {
    for (int32_t c = 0; c < F->nchunks; ++c) kd_free(&F->trees[c]);
    free(F->trees); free(F->a);
}

/* the smallest tree that still holds every id > min_id */
static const kdtree *forest_pick(const laterforest *F, int32_t min_id) {
    /* starts are decreasing with c */
    for (int32_t c = 0; c < F->nchunks; ++c)
        if (F->a[c] <= min_id + 1) return &F->trees[c];
    return &F->trees[F->nchunks - 1];
}

/* pool[i][0..len_i) = the C nearest points with id > i, ascending (distance, id);
 * len_i = min(C, n-1-i); unused slots are -1.  x is in ordering-position order. */
int csel_geo_later_knn(const double *x, int32_t n, int32_t d, int32_t C, int32_t *pool, int32_t *len) {
    if (n <= 0 || d < 1 || d > MAXD || C < 0) return -1;
    laterforest F; forest_build(&F, x, n, d);
    int32_t maxnodes = 0;
    for (int32_t c = 0; c < F.nchunks; ++c) if (F.trees[c].nnodes > maxnodes) maxnodes = F.trees[c].nnodes;
#pragma omp parallel
    {
        nbr *h = (nbr *)malloc(sizeof(nbr) * (C > 0 ? C : 1));
        int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (maxnodes + 8));
#pragma omp for schedule(dynamic, 256)
        for (int32_t i = 0; i < n; ++i) {
            int32_t want = n - 1 - i; if (want > C) want = C;
            kfilter f = {i, NULL, 0.0, NULL};
            int32_t got = kd_knn(forest_pick(&F, i), x + (int64_t)i * d, want, &f, h, stack);
            qsort(h, got, sizeof(nbr), nbr_cmp);
            int32_t *row = pool + (int64_t)i * C;
            for (int32_t j = 0; j < C; ++j) row[j] = j < got ? h[j].id : -1;
            len[i] = got;
        }
        free(h); free(stack);
    }
    forest_free(&F);
    return 0;
}

/* As csel_geo_later_knn, for the query positions q[0..nq) only: row r of
 * pool/len belongs to position q[r]. */
int csel_geo_later_knn_subset(const double *x, int32_t n, int32_t d, int32_t C, int32_t nq, const int32_t *q,
                              int32_t *pool, int32_t *len) {
    if (n <= 0 || d < 1 || d > MAXD || C < 0 || nq < 0) return -1;
    laterforest F; forest_build(&F, x, n, d);
    int32_t maxnodes = 0;
    for (int32_t c = 0; c < F.nchunks; ++c) if (F.trees[c].nnodes > maxnodes) maxnodes = F.trees[c].nnodes;
#pragma omp parallel
    {
        nbr *h = (nbr *)malloc(sizeof(nbr) * (C > 0 ? C : 1));
        int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (maxnodes + 8));
#pragma omp for schedule(dynamic, 64)
        for (int32_t r = 0; r < nq; ++r) {
            int32_t i = q[r];
            int32_t *row = pool + (int64_t)r * C;
            if (i < 0 || i >= n) {
                for (int32_t j = 0; j < C; ++j) row[j] = -1;
                len[r] = 0;
                continue;
            }
            int32_t want = n - 1 - i; if (want > C) want = C;
            kfilter f = {i, NULL, 0.0, NULL};
            int32_t got = kd_knn(forest_pick(&F, i), x + (int64_t)i * d, want, &f, h, stack);
            qsort(h, got, sizeof(nbr), nbr_cmp);
            for (int32_t j = 0; j < C; ++j) row[j] = j < got ? h[j].id : -1;
            len[r] = got;
        }
        free(h); free(stack);
    }
    forest_free(&F);
    return 0;
}

/* Groups of nearby columns (supernodes).  Repeatedly take the earliest
 * unassigned id p and join to it up to m_g - 1 of its nearest unassigned later
 * ids j with ell[j] <= lambda * ell[p].  members are listed in increasing id.
 * sizes[g] are pre-drawn group sizes (cycled if exhausted).  Returns the
 * number of groups; group_ptr has n + 1 slots, members n slots. */
int32_t csel_geo_make_groups(const double *x, const double *ell, int32_t n, int32_t d, const int32_t *sizes,
                             int32_t nsizes, double lambda, int32_t *group_ptr, int32_t *members) {
    if (n <= 0 || d < 1 || d > MAXD || nsizes <= 0) return -1;
    kdtree t; kd_build(&t, x, d, 0, n);
    uint8_t *taken = (uint8_t *)calloc(n, 1);
    int32_t maxm = 1;
    for (int32_t s = 0; s < nsizes; ++s) if (sizes[s] > maxm) maxm = sizes[s];
    nbr *h = (nbr *)malloc(sizeof(nbr) * maxm);
    int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (t.nnodes + 8));
    int32_t g = 0, p = 0, fill = 0;
    group_ptr[0] = 0;
    for (;;) {
        while (p < n && taken[p]) ++p;
        if (p >= n) break;
        int32_t m = sizes[g % nsizes];
        if (m < 1) m = 1;
        kfilter f = {p, ell, lambda * ell[p], taken};
        if (!(ell[p] < INFINITY)) f.ell = NULL;
        int32_t got = kd_knn(&t, x + (int64_t)p * d, m - 1, &f, h, stack);
        qsort(h, got, sizeof(nbr), nbr_cmp);
        /* members sorted by id */
        int32_t base = fill;
        members[fill++] = p; taken[p] = 1;
        for (int32_t j = 0; j < got; ++j) { members[fill++] = h[j].id; taken[h[j].id] = 1; }
        for (int32_t a = base + 1; a < fill; ++a)
            for (int32_t b2 = a; b2 > base && members[b2 - 1] > members[b2]; --b2) {
                int32_t tmp = members[b2]; members[b2] = members[b2 - 1]; members[b2 - 1] = tmp;
            }
        ++g; group_ptr[g] = fill;
    }
    free(stack); free(h); free(taken); kd_free(&t);
    return g;
}

/* Union pools for groups: the C points nearest to any member (distance = min
 * over members), restricted to ids > max(member) when later_only, else to ids
 * of the candidate set [cand0, cand1).  Ascending (distance, id).  When
 * later_only is 0, x must hold the candidates at ids [cand0, cand1) and the
 * members anywhere. */
static int nbr_id_cmp(const void *a, const void *b) {
    const nbr *x = (const nbr *)a, *y = (const nbr *)b;
    if (x->id != y->id) return (x->id > y->id) - (x->id < y->id);
    return (x->d2 > y->d2) - (x->d2 < y->d2);
}

int csel_geo_group_pools(const double *x, int32_t n, int32_t d, int32_t n_groups, const int32_t *group_ptr,
                         const int32_t *members, int32_t later_only, int32_t cand0, int32_t cand1, int32_t C,
                         int32_t *pool, int32_t *len) {
    if (n <= 0 || d < 1 || d > MAXD || C < 0) return -1;
    /* later_only: 0 = the ids in [cand0, cand1); 1 = points after the
       group's last member; 2 = per member, points after that member (the
       partial, non-adjacent case), members excluded */
    laterforest F; kdtree T; int use_forest = later_only != 0; int per_member = later_only == 2;
    int32_t maxnodes = 0;
    if (use_forest) {
        forest_build(&F, x, n, d);
        for (int32_t c = 0; c < F.nchunks; ++c) if (F.trees[c].nnodes > maxnodes) maxnodes = F.trees[c].nnodes;
    } else {
        kd_build(&T, x, d, cand0, cand1 - cand0);
        maxnodes = T.nnodes;
    }
    int32_t maxm = 1;
    for (int32_t g = 0; g < n_groups; ++g) if (group_ptr[g + 1] - group_ptr[g] > maxm) maxm = group_ptr[g + 1] - group_ptr[g];
#pragma omp parallel
    {
        nbr *h = (nbr *)malloc(sizeof(nbr) * (size_t)(C + maxm + 1));
        nbr *all = (nbr *)malloc(sizeof(nbr) * (size_t)(C + maxm + 1) * maxm);
        int32_t *stack = (int32_t *)malloc(sizeof(int32_t) * (maxnodes + 8));
#pragma omp for schedule(dynamic, 16)
        for (int32_t g = 0; g < n_groups; ++g) {
            int32_t b = group_ptr[g], e = group_ptr[g + 1];
            int32_t mx = -1;
            for (int32_t q = b; q < e; ++q) if (members[q] > mx) mx = members[q];
            const kdtree *tree = use_forest ? forest_pick(&F, mx) : &T;
            kfilter f = {use_forest ? mx : cand0 - 1, NULL, 0.0, NULL};
            int32_t tot = 0;
            const int32_t m = e - b;
            for (int32_t q = b; q < e; ++q) {
                int32_t got;
                if (per_member) {
                    /* the member's own later neighbours (m more, as later
                       members are dropped below) */
                    kfilter fq = {members[q], NULL, 0.0, NULL};
                    got = kd_knn(forest_pick(&F, members[q]), x + (int64_t)members[q] * d, C + m, &fq, h, stack);
                } else {
                    got = kd_knn(tree, x + (int64_t)members[q] * d, C, &f, h, stack);
                }
                memcpy(all + tot, h, sizeof(nbr) * got); tot += got;
            }
            /* keep each id once with its smallest distance (and no member) */
            qsort(all, tot, sizeof(nbr), nbr_id_cmp);
            int32_t u = 0;
            for (int32_t j = 0; j < tot; ++j) {
                if (u > 0 && all[u - 1].id == all[j].id) continue;
                int is_member = 0;
                if (per_member)
                    for (int32_t q = b; q < e; ++q) is_member |= members[q] == all[j].id;
                if (!is_member) all[u++] = all[j];
            }
            qsort(all, u, sizeof(nbr), nbr_cmp);
            int32_t keep = u < C ? u : C;
            int32_t *row = pool + (int64_t)g * C;
            for (int32_t j = 0; j < C; ++j) row[j] = j < keep ? all[j].id : -1;
            len[g] = keep;
        }
        free(h); free(all); free(stack);
    }
    if (use_forest) forest_free(&F); else kd_free(&T);
    return 0;
}
