/*
 * dt_oracle.c -- CPU oracle for the Delaunay triangulation.
 *
 * TEST INFRASTRUCTURE ONLY.  Only tests/, the smoke check and the benchmark's
 * CPU-baseline leg may load this library.  It shares no code with the GPU
 * path (paper_1902_07554_amd/csrc) and never calls it.
 *
 * What it computes: the set of finite simplices of DT(P) for P in R^D,
 * D in {2,3} -- the triangulation in which no input point lies strictly
 * inside the circumsphere of any simplex (paper, Section "Delaunay
 * Triangulations").  The paper assumes general position, where DT(P) is
 * unique.  Ties are broken by a symbolic perturbation of the lifting map:
 * the paraboloid height of point i is |p_i|^2 + eps_i with
 * eps_{id} >> eps_{id'} whenever id < id' (id = global point id).  This
 * makes the result the unique regular triangulation of the perturbed
 * lifted points, independent of insertion order and of any division of the
 * input, which is what lets the divide-and-conquer method reproduce it.
 *
 * Method: plain incremental Bowyer-Watson with an infinite vertex.  For
 * each point: walk to a cell in conflict, grow the conflict region (cells
 * whose circumsphere strictly contains the point, or hull cells whose facet
 * the point sees), delete it and connect the point to its boundary facets.
 *
 * Predicates are exact: a floating-point evaluation whose rounding error is
 * bounded a priori (bound derived in the comments of in_filter/or_filter),
 * falling back to exact big-integer arithmetic on the doubles' integer
 * mantissas.  Conventions (own, stated here, pinned by tests):
 *   Orient1(p_0..p_D) = det [ p_i  1 ]               ((D+1)x(D+1))
 *   In(p_0..p_D, q)   = det [ p_i  |p_i|^2  1 ; q |q|^2 1 ]   ((D+2)x(D+2))
 * With Orient1(cell) > 0, q is strictly inside the circumsphere iff In > 0.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#include <float.h>

/* ------------------------------------------------------------------ */
/* Signed big integers with 32-bit limbs.                              */
/* Worst case: doubles span 2^-1074..2^1024 (2098 bits); a 3D insphere   */
/* term has degree 5 -> about 10.5k bits -> 330 limbs.                   */
/* ------------------------------------------------------------------ */
#define BL 352
typedef struct { int n; int neg; uint32_t d[BL]; } big;

static void bzero_(big *r) { r->n = 0; r->neg = 0; }

static void bnorm(big *r) {
    while (r->n > 0 && r->d[r->n - 1] == 0) r->n--;
    if (r->n == 0) r->neg = 0;
}

static int bcmpmag(const big *a, const big *b) {
    if (a->n != b->n) return a->n < b->n ? -1 : 1;
    for (int i = a->n - 1; i >= 0; i--)
        if (a->d[i] != b->d[i]) return a->d[i] < b->d[i] ? -1 : 1;
    return 0;
}

/* r = |a| + |b|  (r must not alias a or b) */
static void baddmag(big *r, const big *a, const big *b) {
    int n = a->n > b->n ? a->n : b->n;
    uint64_t c = 0;
    for (int i = 0; i < n; i++) {
        uint64_t s = c;
        if (i < a->n) s += a->d[i];
        if (i < b->n) s += b->d[i];
        r->d[i] = (uint32_t)s;
        c = s >> 32;
    }
    r->n = n;
    if (c) r->d[r->n++] = (uint32_t)c;
}

/* r = |a| - |b| with |a| >= |b|  (r must not alias a or b) */
static void bsubmag(big *r, const big *a, const big *b) {
    int64_t br = 0;
    for (int i = 0; i < a->n; i++) {
        int64_t s = (int64_t)a->d[i] - br - (i < b->n ? (int64_t)b->d[i] : 0);
        br = s < 0;
        r->d[i] = (uint32_t)(s + (br ? ((int64_t)1 << 32) : 0));
    }
    r->n = a->n;
}

/* r = a + b (r must not alias a or b) */
static void badd(big *r, const big *a, const big *b) {
    if (a->neg == b->neg) {
        baddmag(r, a, b);
        r->neg = a->neg;
    } else if (bcmpmag(a, b) >= 0) {
        bsubmag(r, a, b);
        r->neg = a->neg;
    } else {
        bsubmag(r, b, a);
        r->neg = b->neg;
    }
    bnorm(r);
}

/* r = a - b (r must not alias a or b) */
static void bsub(big *r, const big *a, const big *b) {
    big t = *b;
    if (t.n) t.neg = !t.neg;
    badd(r, a, &t);
}

/* r = a * b (r must not alias a or b) */
static void bmul(big *r, const big *a, const big *b) {
    if (a->n == 0 || b->n == 0) { bzero_(r); return; }
    int n = a->n + b->n;
    memset(r->d, 0, sizeof(uint32_t) * (size_t)n);
    for (int i = 0; i < a->n; i++) {
        uint64_t c = 0;
        for (int j = 0; j < b->n; j++) {
            uint64_t t = (uint64_t)a->d[i] * b->d[j] + r->d[i + j] + c;
            r->d[i + j] = (uint32_t)t;
            c = t >> 32;
        }
        int k = i + b->n;
        while (c) {
            uint64_t t = (uint64_t)r->d[k] + c;
            r->d[k] = (uint32_t)t;
            c = t >> 32;
            k++;
        }
    }
    r->n = n;
    r->neg = a->neg ^ b->neg;
    bnorm(r);
}

static int bsign(const big *a) { return a->n == 0 ? 0 : (a->neg ? -1 : 1); }

/* Exponent of the least significant bit of x's 53-bit integer mantissa. */
static int lsb_exp(double x) {
    int ex;
    frexp(x, &ex);
    return ex - 53;
}

/* r = x * 2^(-E), exact; requires lsb_exp(x) >= E. */
static void bfromd(big *r, double x, int E) {
    bzero_(r);
    if (x == 0.0) return;
    int ex;
    double f = frexp(x, &ex);
    int64_t m = (int64_t)ldexp(f, 53);
    int sh = ex - 53 - E;
    int neg = m < 0;
    uint64_t um = neg ? (uint64_t)(-m) : (uint64_t)m;
    int w = sh / 32, b = sh % 32;
    unsigned __int128 v = (unsigned __int128)um << b;
    for (int i = 0; i < w; i++) r->d[i] = 0;
    r->d[w] = (uint32_t)v;
    r->d[w + 1] = (uint32_t)(v >> 32);
    r->d[w + 2] = (uint32_t)(v >> 64);
    r->n = w + 3;
    r->neg = neg;
    bnorm(r);
}

/* Determinant of the square matrix formed by rows row..n-1 and the
 * columns in colmask (Laplace expansion along the first remaining row). */
static void bdet(big *r, big M[4][4], int n, int row, unsigned colmask) {
    if (row == n - 1) {
        for (int c = 0; c < 4; c++)
            if (colmask >> c & 1) { *r = M[row][c]; return; }
    }
    big acc, sub, t, nacc;
    bzero_(&acc);
    int sgn = 1;
    for (int c = 0; c < 4; c++) {
        if (!(colmask >> c & 1)) continue;
        bdet(&sub, M, n, row + 1, colmask & ~(1u << c));
        bmul(&t, &M[row][c], &sub);
        if (sgn < 0 && t.n) t.neg = !t.neg;
        badd(&nacc, &acc, &t);
        acc = nacc;
        sgn = -sgn;
    }
    *r = acc;
}

static int min_lsb_exp(int cnt, const double *const *P, int D) {
    int E = 1 << 20;
    for (int i = 0; i < cnt; i++)
        for (int k = 0; k < D; k++)
            if (P[i][k] != 0.0) {
                int e = lsb_exp(P[i][k]);
                if (e < E) E = e;
            }
    return E == (1 << 20) ? 0 : E;
}

/* sign of det[p_i - p_0]_{i=1..D}, exactly */
static int exact_orient_core(int D, const double *const *P) {
    int E = min_lsb_exp(D + 1, P, D);
    static __thread big c[4][3];
    static __thread big M[4][4];
    for (int i = 0; i <= D; i++)
        for (int k = 0; k < D; k++) bfromd(&c[i][k], P[i][k], E);
    for (int i = 1; i <= D; i++)
        for (int k = 0; k < D; k++) bsub(&M[i - 1][k], &c[i][k], &c[0][k]);
    big r;
    bdet(&r, M, D, 0, (1u << D) - 1);
    return bsign(&r);
}

/* sign of In(p_0..p_D, q) = det[p_i - q, |p_i - q|^2]_{i=0..D}, exactly */
static int exact_in_core(int D, const double *const *P) {
    int E = min_lsb_exp(D + 2, P, D);
    static __thread big c[5][3];
    static __thread big M[4][4];
    for (int i = 0; i <= D + 1; i++)
        for (int k = 0; k < D; k++) bfromd(&c[i][k], P[i][k], E);
    for (int i = 0; i <= D; i++) {
        big l, t, s;
        bzero_(&l);
        for (int k = 0; k < D; k++) {
            bsub(&M[i][k], &c[i][k], &c[D + 1][k]);
            bmul(&t, &M[i][k], &M[i][k]);
            badd(&s, &l, &t);
            l = s;
        }
        M[i][D] = l;
    }
    big r;
    bdet(&r, M, D + 1, 0, (1u << (D + 1)) - 1);
    return bsign(&r);
}

/* ------------------------------------------------------------------ */
/* Floating-point filters.                                             */
/* Each evaluates the same polynomial in double precision.  With every  */
/* operation rounding to nearest, the computed value is                 */
/*   sum_t term_t * prod_{j<=K} (1 + d_j),  |d_j| <= u = 2^-53,         */
/* where K counts, for the longest term, the rounded differences that   */
/* enter it (one per input factor, i.e. its degree) plus the rounded    */
/* products and sums on its path to the result.  Hence                  */
/* |err| <= gamma_K * P with P the same polynomial over absolute values, */
/* and the P computed in floating point is at least P*(1 - gamma_K).    */
/* gamma_K * P <= K*u*P_computed*(1 + O(K u)), so |value| > K*u*P_comp. */
/* certifies the sign up to that O(Ku) term; the bound used is twice    */
/* that, the factor 2 being slack.  Results near the underflow range go */
/* to the exact path.                                                   */
/* ------------------------------------------------------------------ */
#define U53 (DBL_EPSILON * 0.5)
#define TINY 1e-280

static int certify(double v, double perm, int K, int *sign) {
    if (!(perm < INFINITY) || perm < TINY) return 0;
    double bound = 2.0 * K * U53 * perm;
    if (v > bound) { *sign = 1; return 1; }
    if (v < -bound) { *sign = -1; return 1; }
    return 0;
}

/* det[p_i - p_0].  2D: degree 2, path mul, sub -> K = 2 + 2 = 4.
 * 3D: degree 3, path mul, sub (minor), mul, sub, add -> K = 3 + 5 = 8. */
static int or_filter(int D, const double *const *P, int *sign) {
    if (D == 2) {
        double ax = P[1][0] - P[0][0], ay = P[1][1] - P[0][1];
        double bx = P[2][0] - P[0][0], by = P[2][1] - P[0][1];
        double l = ax * by, r = ay * bx;
        return certify(l - r, fabs(l) + fabs(r), 4, sign);
    } else {
        double a[3], b[3], c[3];
        for (int k = 0; k < 3; k++) {
            a[k] = P[1][k] - P[0][k];
            b[k] = P[2][k] - P[0][k];
            c[k] = P[3][k] - P[0][k];
        }
        double m0 = b[1] * c[2] - b[2] * c[1];
        double m1 = b[0] * c[2] - b[2] * c[0];
        double m2 = b[0] * c[1] - b[1] * c[0];
        double p0 = fabs(b[1] * c[2]) + fabs(b[2] * c[1]);
        double p1 = fabs(b[0] * c[2]) + fabs(b[2] * c[0]);
        double p2 = fabs(b[0] * c[1]) + fabs(b[1] * c[0]);
        double v = a[0] * m0 - a[1] * m1 + a[2] * m2;
        double p = fabs(a[0]) * p0 + fabs(a[1]) * p1 + fabs(a[2]) * p2;
        return certify(v, p, 8, sign);
    }
}

/* det[p_i - q, |p_i - q|^2].
 * 2D: degree 4; path mul, add (height), mul, sub (minor), mul, sub, add
 *     -> K = 4 + 7 = 11.
 * 3D: degree 5; path mul, add, add (height), mul, sub (2x2 minor), mul,
 *     sub, add (3x3 minor), mul (height times minor), three accumulations
 *     (the first, from 0, is exact) -> K = 5 + 12 = 17. */
static int in_filter(int D, const double *const *P, int *sign) {
    const double *q = P[D + 1];
    if (D == 2) {
        double x[3], y[3], l[3], la[3];
        for (int i = 0; i < 3; i++) {
            x[i] = P[i][0] - q[0];
            y[i] = P[i][1] - q[1];
            l[i] = x[i] * x[i] + y[i] * y[i];
            la[i] = l[i];
        }
        double m0 = x[1] * y[2] - y[1] * x[2];
        double m1 = x[0] * y[2] - y[0] * x[2];
        double m2 = x[0] * y[1] - y[0] * x[1];
        double p0 = fabs(x[1] * y[2]) + fabs(y[1] * x[2]);
        double p1 = fabs(x[0] * y[2]) + fabs(y[0] * x[2]);
        double p2 = fabs(x[0] * y[1]) + fabs(y[0] * x[1]);
        double v = l[0] * m0 - l[1] * m1 + l[2] * m2;
        double p = la[0] * p0 + la[1] * p1 + la[2] * p2;
        return certify(v, p, 11, sign);
    } else {
        double d[4][3], l[4];
        for (int i = 0; i < 4; i++) {
            for (int k = 0; k < 3; k++) d[i][k] = P[i][k] - q[k];
            l[i] = d[i][0] * d[i][0] + d[i][1] * d[i][1] + d[i][2] * d[i][2];
        }
        double v = 0.0, p = 0.0;
        for (int i = 0; i < 4; i++) {
            int r[3], t = 0;
            for (int j = 0; j < 4; j++)
                if (j != i) r[t++] = j;
            const double *a = d[r[0]], *b = d[r[1]], *c = d[r[2]];
            double m0 = b[1] * c[2] - b[2] * c[1];
            double m1 = b[0] * c[2] - b[2] * c[0];
            double m2 = b[0] * c[1] - b[1] * c[0];
            double p0 = fabs(b[1] * c[2]) + fabs(b[2] * c[1]);
            double p1 = fabs(b[0] * c[2]) + fabs(b[2] * c[0]);
            double p2 = fabs(b[0] * c[1]) + fabs(b[1] * c[0]);
            double m3 = a[0] * m0 - a[1] * m1 + a[2] * m2;
            double q3 = fabs(a[0]) * p0 + fabs(a[1]) * p1 + fabs(a[2]) * p2;
            /* cofactor sign of entry (i, 3) of a 4x4 matrix: (-1)^(i+3) */
            double term = l[i] * m3;
            if ((i + 3) & 1) v -= term; else v += term;
            p += l[i] * q3;
        }
        return certify(v, p, 17, sign);
    }
}

/* sign of Orient1(p_0..p_D) = (-1)^D * sign det[p_i - p_0] */
static int orient1(int D, const double *const *P) {
    int s;
    if (!or_filter(D, P, &s)) s = exact_orient_core(D, P);
    return (D & 1) ? -s : s;
}

/* sign of In(p_0..p_D, q), unperturbed */
static int in_raw(int D, const double *const *P) {
    int s;
    if (!in_filter(D, P, &s)) s = exact_in_core(D, P);
    return s;
}

/* Sign of In with the perturbed lifting.  keys[i] orders the perturbation
 * (smaller key = larger perturbation).  In_pert = In + sum_i eps_i Cof_i,
 * where Cof_i, the cofactor of point i's height entry (row i, column D),
 * is (-1)^(i+D) * Orient1(the other D+1 points in their order).  The sign
 * is that of the first nonzero term in perturbation order. */
static int in_pert(int D, const double *const *P, const int64_t *keys) {
    int s = in_raw(D, P);
    if (s) return s;
    int ord[5];
    for (int i = 0; i < D + 2; i++) ord[i] = i;
    for (int i = 1; i < D + 2; i++)
        for (int j = i; j > 0 && keys[ord[j]] < keys[ord[j - 1]]; j--) {
            int t = ord[j]; ord[j] = ord[j - 1]; ord[j - 1] = t;
        }
    for (int t = 0; t < D + 2; t++) {
        int i = ord[t];
        const double *Q[4];
        int c = 0;
        for (int j = 0; j < D + 2; j++)
            if (j != i) Q[c++] = P[j];
        int o = orient1(D, Q);
        if (o) return ((i + D) & 1) ? -o : o;
    }
    return 0;
}

/* ------------------------------------------------------------------ */
/* Triangulation data.                                                  */
/* ------------------------------------------------------------------ */
#define INF_V (-1)

typedef struct {
    int D;
    int64_t n;
    const double *X;      /* n x D */
    const int64_t *key;   /* perturbation keys (global ids) */
    int32_t *cv;          /* cells x (D+1) vertex indices, INF_V = infinite vertex */
    int32_t *cn;          /* cells x (D+1) neighbour cell indices */
    int64_t *mark;        /* conflict-region stamp */
    int64_t *seen;        /* tested-and-not-in-conflict stamp */
    uint8_t *dead;
    int64_t ncells, cap;
    int32_t *freel;
    int64_t nfree;
} tri_t;

static const double *PT(const tri_t *T, int32_t v) { return T->X + (int64_t)v * T->D; }

static int grow(tri_t *T) {
    int64_t nc = T->cap ? T->cap * 2 : 1024;
    int V = T->D + 1;
    int32_t *cv = realloc(T->cv, sizeof(int32_t) * V * nc);
    int32_t *cn = realloc(T->cn, sizeof(int32_t) * V * nc);
    int64_t *mk = realloc(T->mark, sizeof(int64_t) * nc);
    int64_t *sn = realloc(T->seen, sizeof(int64_t) * nc);
    uint8_t *dd = realloc(T->dead, nc);
    int32_t *fl = realloc(T->freel, sizeof(int32_t) * nc);
    if (!cv || !cn || !mk || !sn || !dd || !fl) return -1;
    T->cv = cv; T->cn = cn; T->mark = mk; T->seen = sn; T->dead = dd; T->freel = fl;
    for (int64_t i = T->cap; i < nc; i++) { mk[i] = -1; sn[i] = -1; dd[i] = 1; }
    T->cap = nc;
    return 0;
}

static int32_t new_cell(tri_t *T) {
    if (T->nfree > 0) {
        int32_t c = T->freel[--T->nfree];
        T->dead[c] = 0;
        return c;
    }
    if (T->ncells == T->cap && grow(T)) return -1;
    int32_t c = (int32_t)T->ncells++;
    T->dead[c] = 0;
    T->mark[c] = -1;
    T->seen[c] = -1;
    return c;
}

/* Build the point list of cell c with the infinite vertex (if any) or
 * vertex slot `rep` replaced by point q.  Returns the infinite slot. */
static int cell_inf_slot(const tri_t *T, int32_t c) {
    const int32_t *v = T->cv + (int64_t)c * (T->D + 1);
    for (int i = 0; i <= T->D; i++)
        if (v[i] == INF_V) return i;
    return -1;
}

/* Conflict test of point q with cell c (see file header). */
static int conflict(const tri_t *T, int32_t c, int32_t q) {
    int D = T->D;
    const int32_t *v = T->cv + (int64_t)c * (D + 1);
    const double *P[5];
    int64_t k[5];
    int inf = cell_inf_slot(T, c);
    if (inf < 0) {
        for (int i = 0; i <= D; i++) { P[i] = PT(T, v[i]); k[i] = T->key[v[i]]; }
        P[D + 1] = PT(T, q);
        k[D + 1] = T->key[q];
        return in_pert(D, P, k) > 0;
    }
    for (int i = 0; i <= D; i++) P[i] = (i == inf) ? PT(T, q) : PT(T, v[i]);
    int o = orient1(D, P);
    if (o) return o > 0;
    /* q lies in the hyperplane of the hull facet: decide by the facet's own
     * (D-1)-dimensional circumsphere under the same perturbed lifting, using
     * an auxiliary point e off the hyperplane: the sphere through the facet
     * and e meets the hyperplane exactly in the facet's circumsphere. */
    const double *F[3];
    int nf = 0;
    for (int i = 0; i <= D; i++)
        if (i != inf) F[nf++] = PT(T, v[i]);
    int axis = -1;
    if (D == 2) {
        axis = (F[0][1] != F[1][1]) ? 0 : 1;
    } else {
        for (int a = 0; a < 3 && axis < 0; a++) {
            double pr[3][2];
            const double *pp[3];
            for (int j = 0; j < 3; j++) {
                int t = 0;
                for (int kk = 0; kk < 3; kk++)
                    if (kk != a) pr[j][t++] = F[j][kk];
                pp[j] = pr[j];
            }
            if (orient1(2, pp) != 0) axis = a;
        }
    }
    double e[3];
    for (int kk = 0; kk < D; kk++) e[kk] = F[0][kk];
    double a0 = F[0][axis];
    e[axis] = (a0 == 0.0) ? 1.0 : (fabs(a0) < 1e300 ? 2.0 * a0 : 0.5 * a0);
    for (int i = 0; i <= D; i++) {
        P[i] = (i == inf) ? e : PT(T, v[i]);
        k[i] = (i == inf) ? INT64_MAX : T->key[v[i]];
    }
    int oe = orient1(D, P);
    P[D + 1] = PT(T, q);
    k[D + 1] = T->key[q];
    int s = in_pert(D, P, k);
    return s != 0 && s == oe;
}

/* Visibility walk from cell `start` to a cell in conflict with q. */
static int32_t locate(const tri_t *T, int32_t start, int32_t q) {
    int D = T->D;
    int32_t c = start;
    for (int64_t steps = 0; steps < 4 * T->ncells + 16; steps++) {
        const int32_t *v = T->cv + (int64_t)c * (D + 1);
        int inf = cell_inf_slot(T, c);
        if (inf >= 0) {
            if (conflict(T, c, q)) return c;
            c = T->cn[(int64_t)c * (D + 1) + inf];
            continue;
        }
        int moved = 0;
        for (int i = 0; i <= D; i++) {
            const double *P[4];
            for (int j = 0; j <= D; j++) P[j] = (j == i) ? PT(T, q) : PT(T, v[j]);
            if (orient1(D, P) < 0) {
                c = T->cn[(int64_t)c * (D + 1) + i];
                moved = 1;
                break;
            }
        }
        if (!moved) return c;
    }
    return -1;
}

static int nbr_slot(const tri_t *T, int32_t c, int32_t of) {
    for (int i = 0; i <= T->D; i++)
        if (T->cn[(int64_t)c * (T->D + 1) + i] == of) return i;
    return -1;
}

typedef struct { int32_t a, b; int32_t cell; int32_t slot; } rkey_t;

static int rkey_cmp(const void *x, const void *y) {
    const rkey_t *p = x, *q = y;
    if (p->a != q->a) return p->a < q->a ? -1 : 1;
    if (p->b != q->b) return p->b < q->b ? -1 : 1;
    return 0;
}

/* Insert point q (Bowyer-Watson).  Returns a new cell or -1. */
static int32_t insert(tri_t *T, int32_t start, int32_t q, int64_t stamp,
                      int32_t **cav, int64_t *cavcap, rkey_t **rk, int64_t *rkcap) {
    int D = T->D, V = D + 1;
    int32_t c0 = locate(T, start, q);
    if (c0 < 0 || !conflict(T, c0, q)) return -1;
    int64_t nc = 0;
    (*cav)[nc++] = c0;
    T->mark[c0] = stamp;
    for (int64_t h = 0; h < nc; h++) {
        int32_t c = (*cav)[h];
        for (int i = 0; i < V; i++) {
            int32_t nb = T->cn[(int64_t)c * V + i];
            if (T->mark[nb] == stamp || T->seen[nb] == stamp) continue;
            if (conflict(T, nb, q)) {
                if (nc == *cavcap) {
                    *cavcap *= 2;
                    *cav = realloc(*cav, sizeof(int32_t) * *cavcap);
                    if (!*cav) return -1;
                }
                (*cav)[nc++] = nb;
                T->mark[nb] = stamp;
            } else {
                T->seen[nb] = stamp;
            }
        }
    }
    /* One new cell per boundary facet: the cavity cell with the vertex
     * opposite the facet replaced by q. */
    int64_t nk = 0;
    int32_t last = -1;
    for (int64_t h = 0; h < nc; h++) {
        int32_t c = (*cav)[h];
        for (int i = 0; i < V; i++) {
            int32_t nb = T->cn[(int64_t)c * V + i];
            if (T->mark[nb] == stamp) continue;
            int32_t x = new_cell(T);
            if (x < 0) return -1;
            for (int j = 0; j < V; j++) {
                T->cv[(int64_t)x * V + j] = (j == i) ? q : T->cv[(int64_t)c * V + j];
                T->cn[(int64_t)x * V + j] = -1;
            }
            T->cn[(int64_t)x * V + i] = nb;
            int s = nbr_slot(T, nb, c);
            T->cn[(int64_t)nb * V + s] = x;
            /* facets of x through q: key = the other D-1 vertices */
            for (int j = 0; j < V; j++) {
                if (j == i) continue;
                int32_t r[2];
                int t = 0;
                for (int l = 0; l < V; l++)
                    if (l != i && l != j) r[t++] = T->cv[(int64_t)x * V + l];
                if (D == 2) { r[1] = 0; }
                else if (r[0] > r[1]) { int32_t tt = r[0]; r[0] = r[1]; r[1] = tt; }
                if (nk == *rkcap) {
                    *rkcap *= 2;
                    *rk = realloc(*rk, sizeof(rkey_t) * *rkcap);
                    if (!*rk) return -1;
                }
                (*rk)[nk].a = r[0]; (*rk)[nk].b = r[1];
                (*rk)[nk].cell = x; (*rk)[nk].slot = j;
                nk++;
            }
            last = x;
        }
    }
    qsort(*rk, (size_t)nk, sizeof(rkey_t), rkey_cmp);
    for (int64_t h = 0; h + 1 < nk; h += 2) {
        rkey_t *p = &(*rk)[h], *o = &(*rk)[h + 1];
        if (rkey_cmp(p, o) != 0) return -1;
        T->cn[(int64_t)p->cell * V + p->slot] = o->cell;
        T->cn[(int64_t)o->cell * V + o->slot] = p->cell;
    }
    if (nk & 1) return -1;
    for (int64_t h = 0; h < nc; h++) {
        int32_t c = (*cav)[h];
        T->dead[c] = 1;
        T->freel[T->nfree++] = c;
    }
    return last;
}

/* ------------------------------------------------------------------ */
/* Input checks and insertion order.                                    */
/* ------------------------------------------------------------------ */
static const double *g_sortX;
static int g_sortD;
static int lex_cmp(const void *a, const void *b) {
    int64_t i = *(const int64_t *)a, j = *(const int64_t *)b;
    for (int k = 0; k < g_sortD; k++) {
        double x = g_sortX[i * g_sortD + k], y = g_sortX[j * g_sortD + k];
        if (x < y) return -1;
        if (x > y) return 1;
    }
    return 0;
}

typedef struct { uint64_t k; int64_t i; } ord_t;
static int ord_cmp(const void *a, const void *b) {
    const ord_t *p = a, *q = b;
    if (p->k != q->k) return p->k < q->k ? -1 : 1;
    return p->i < q->i ? -1 : (p->i > q->i);
}

static uint64_t mix64(uint64_t z) {
    z += 0x9E3779B97F4A7C15ull;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
    return z ^ (z >> 31);
}

static uint64_t spread(uint64_t x, int D) {
    uint64_t r = 0;
    int bits = D == 2 ? 26 : 17;
    for (int b = 0; b < bits; b++) r |= ((x >> b) & 1ull) << (b * D);
    return r;
}

/* Insertion order (only for speed; the result does not depend on it):
 * biased randomised rounds, Morton order inside each round. */
static ord_t *insertion_order(const double *X, int64_t n, int D) {
    double lo[3], hi[3];
    for (int k = 0; k < D; k++) { lo[k] = INFINITY; hi[k] = -INFINITY; }
    for (int64_t i = 0; i < n; i++)
        for (int k = 0; k < D; k++) {
            double x = X[i * D + k];
            if (x < lo[k]) lo[k] = x;
            if (x > hi[k]) hi[k] = x;
        }
    ord_t *o = malloc(sizeof(ord_t) * (size_t)n);
    if (!o) return NULL;
    int bits = D == 2 ? 26 : 17;
    double scale = (double)((1u << bits) - 1);
    for (int64_t i = 0; i < n; i++) {
        uint64_t m = 0;
        for (int k = 0; k < D; k++) {
            double ext = hi[k] - lo[k];
            double t = ext > 0 ? (X[i * D + k] - lo[k]) / ext : 0.0;
            uint64_t qv = (uint64_t)(t * scale);
            m |= spread(qv, D) << k;
        }
        uint64_t h = mix64((uint64_t)i);
        int r = 0;
        while (r < 6 && (h & 1)) { r++; h >>= 1; }
        o[i].k = ((uint64_t)(6 - r) << 58) | (m & ((1ull << 58) - 1));
        o[i].i = i;
    }
    qsort(o, (size_t)n, sizeof(ord_t), ord_cmp);
    return o;
}

/* ------------------------------------------------------------------ */
/* Public entry points (called through ctypes by the tests).            */
/* ------------------------------------------------------------------ */
enum { ORC_OK = 0, ORC_INVALID = -1, ORC_NONFINITE = -2, ORC_DUPLICATE = -3,
       ORC_DEGENERATE = -4, ORC_NOMEM = -5, ORC_INTERNAL = -7 };

int orc_orient(int D, const double *pts) {
    const double *P[4];
    for (int i = 0; i <= D; i++) P[i] = pts + i * D;
    return orient1(D, P);
}

/* pts: (D+2) x D, the last row is q; keys may be NULL (no perturbation). */
int orc_insphere(int D, const double *pts, const int64_t *keys) {
    const double *P[5];
    for (int i = 0; i < D + 2; i++) P[i] = pts + i * D;
    if (!keys) return in_raw(D, P);
    return in_pert(D, P, keys);
}

/* Delaunay triangulation.  keys: perturbation order per point (NULL: the
 * index).  On success *out holds m x (D+1) point indices (finite cells);
 * free with orc_free. */
int orc_dt(const double *X, const int64_t *keys, int64_t n, int D,
           int32_t **out, int64_t *m_out) {
    *out = NULL;
    *m_out = 0;
    if ((D != 2 && D != 3) || n < 0) return ORC_INVALID;
    for (int64_t i = 0; i < n * D; i++)
        if (!isfinite(X[i])) return ORC_NONFINITE;
    if (n < D + 1) return ORC_DEGENERATE;
    int64_t *ix = malloc(sizeof(int64_t) * (size_t)n);
    int64_t *kk = NULL;
    if (!ix) return ORC_NOMEM;
    for (int64_t i = 0; i < n; i++) ix[i] = i;
    g_sortX = X;
    g_sortD = D;
    qsort(ix, (size_t)n, sizeof(int64_t), lex_cmp);
    for (int64_t i = 0; i + 1 < n; i++)
        if (lex_cmp(&ix[i], &ix[i + 1]) == 0) { free(ix); return ORC_DUPLICATE; }
    free(ix);
    if (!keys) {
        kk = malloc(sizeof(int64_t) * (size_t)n);
        if (!kk) return ORC_NOMEM;
        for (int64_t i = 0; i < n; i++) kk[i] = i;
        keys = kk;
    }
    ord_t *ord = insertion_order(X, n, D);
    if (!ord) { free(kk); return ORC_NOMEM; }

    /* initial simplex: first D+1 affinely independent points in order */
    int64_t init[4];
    int ni = 1;
    init[0] = 0;
    for (int64_t t = 1; t < n && ni < D + 1; t++) {
        const double *P[4];
        int ok;
        if (ni == 1) {
            ok = 1;  /* distinct points */
        } else if (ni == 2 && D == 3) {
            /* not collinear: some coordinate projection has nonzero orient */
            ok = 0;
            for (int a = 0; a < 3 && !ok; a++) {
                double pr[3][2];
                const double *pp[3];
                int64_t src[3] = { ord[init[0]].i, ord[init[1]].i, ord[t].i };
                for (int j = 0; j < 3; j++) {
                    int u = 0;
                    for (int kx = 0; kx < 3; kx++)
                        if (kx != a) pr[j][u++] = X[src[j] * 3 + kx];
                    pp[j] = pr[j];
                }
                ok = orient1(2, pp) != 0;
            }
        } else {
            for (int j = 0; j < ni; j++) P[j] = X + ord[init[j]].i * D;
            P[ni] = X + ord[t].i * D;
            ok = orient1(D, P) != 0;
        }
        if (ok) init[ni++] = t;
    }
    if (ni < D + 1) { free(ord); free(kk); return ORC_DEGENERATE; }

    tri_t T;
    memset(&T, 0, sizeof(T));
    T.D = D; T.n = n; T.X = X; T.key = keys;
    int V = D + 1;
    int32_t iv[4];
    for (int j = 0; j < V; j++) iv[j] = (int32_t)ord[init[j]].i;
    {
        const double *P[4];
        for (int j = 0; j < V; j++) P[j] = PT(&T, iv[j]);
        if (orient1(D, P) < 0) { int32_t t = iv[0]; iv[0] = iv[1]; iv[1] = t; }
    }
    int32_t c0 = new_cell(&T);
    int32_t ic[4];
    for (int j = 0; j < V; j++) T.cv[(int64_t)c0 * V + j] = iv[j];
    for (int i = 0; i < V; i++) {
        ic[i] = new_cell(&T);
        int32_t *w = T.cv + (int64_t)ic[i] * V;
        for (int j = 0; j < V; j++) w[j] = (j == i) ? INF_V : iv[j];
        /* swap two finite vertices so that the apex side is negative */
        int a = (i == 0) ? 1 : 0, b = (i <= 1) ? 2 : 1;
        int32_t t = w[a]; w[a] = w[b]; w[b] = t;
    }
    /* adjacency of the initial D+2 cells by brute-force facet matching */
    {
        int32_t cells[5];
        cells[0] = c0;
        for (int i = 0; i < V; i++) cells[i + 1] = ic[i];
        for (int x = 0; x < V + 1; x++)
            for (int s = 0; s < V; s++) {
                int32_t cx = cells[x];
                for (int y = 0; y < V + 1; y++) {
                    if (y == x) continue;
                    int32_t cy = cells[y];
                    /* facet s of cx shared with cy? */
                    int shared = 0;
                    for (int l = 0; l < V; l++) {
                        if (l == s) continue;
                        int32_t vv = T.cv[(int64_t)cx * V + l];
                        for (int r = 0; r < V; r++)
                            if (T.cv[(int64_t)cy * V + r] == vv) { shared++; break; }
                    }
                    if (shared == D) T.cn[(int64_t)cx * V + s] = cy;
                }
            }
    }
    int64_t cavcap = 256, rkcap = 1024;
    int32_t *cav = malloc(sizeof(int32_t) * cavcap);
    rkey_t *rk = malloc(sizeof(rkey_t) * rkcap);
    int32_t last = c0;
    int st = ORC_OK;
    int64_t stamp = 0;
    for (int64_t t = 0; t < n && st == ORC_OK; t++) {
        int skip = 0;
        for (int j = 0; j < V; j++) if (init[j] == t) skip = 1;
        if (skip) continue;
        int32_t x = insert(&T, last, (int32_t)ord[t].i, stamp++, &cav, &cavcap, &rk, &rkcap);
        if (x < 0) st = ORC_INTERNAL;
        else last = x;
    }
    free(cav);
    free(rk);
    free(ord);
    if (st == ORC_OK) {
        int64_t m = 0;
        for (int64_t c = 0; c < T.ncells; c++)
            if (!T.dead[c] && cell_inf_slot(&T, (int32_t)c) < 0) m++;
        int32_t *o = malloc(sizeof(int32_t) * (size_t)(m * V + 1));
        if (!o) st = ORC_NOMEM;
        else {
            int64_t w = 0;
            for (int64_t c = 0; c < T.ncells; c++)
                if (!T.dead[c] && cell_inf_slot(&T, (int32_t)c) < 0) {
                    for (int j = 0; j < V; j++) o[w * V + j] = T.cv[c * V + j];
                    w++;
                }
            *out = o;
            *m_out = m;
        }
    }
    free(T.cv); free(T.cn); free(T.mark); free(T.seen); free(T.dead); free(T.freel);
    free(kk);
    return st;
}

/* ------------------------------------------------------------------ */
/* Certificate of a claimed Delaunay triangulation.                      */
/* A set of full-dimensional simplices on the input points is DT(P)     */
/* (paper, Section "Delaunay Triangulations": no point inside any        */
/* simplex's circumsphere) when it is a triangulation of P that is       */
/* locally Delaunay at every interior facet:                            */
/*   - every facet lies in at most two simplices, the two of an interior */
/*     facet on opposite sides of it, the facets in one simplex are the  */
/*     convex hull's facets (checked by the caller), and the volumes sum */
/*     to the hull's volume (checked by the caller): the simplices then  */
/*     tile the convex hull exactly once;                               */
/*   - every point is a vertex (under the perturbed lifting every point */
/*     is a vertex of the lower hull);                                  */
/*   - for every interior facet, the apex of one simplex is outside the */
/*     other's circumsphere under the same perturbation as orc_dt: the   */
/*     lifted simplices then form a locally convex, hence convex, lower  */
/*     surface, which is the lower hull of the lifted points.           */
/* Counts of every violation are returned; the hull facets (in one      */
/* simplex only) are returned as sorted rows of D point indices.         */
/* ------------------------------------------------------------------ */
typedef struct {
    int64_t bad_rows;     /* an index out of range or repeated in a row   */
    int64_t flat;         /* simplices with Orient1 = 0                   */
    int64_t over_shared;  /* facets in more than two simplices            */
    int64_t interior;     /* facets in exactly two simplices              */
    int64_t hull;         /* facets in exactly one simplex                */
    int64_t same_side;    /* interior facets with both apexes on one side */
    int64_t not_local;    /* interior facets failing the empty-sphere test */
    int64_t unused;       /* points that are no vertex                    */
    int64_t edges;        /* distinct edges                               */
    double volume;        /* sum of the simplices' volumes                */
} orc_cert_t;

typedef struct { uint32_t a, b, row; int32_t j; } facet_t;

static int facet_cmp(const void *x, const void *y) {
    const facet_t *f = x, *g = y;
    if (f->a != g->a) return f->a < g->a ? -1 : 1;
    if (f->b != g->b) return f->b < g->b ? -1 : 1;
    return 0;
}
static int u32_cmp(const void *x, const void *y) {
    uint32_t a = *(const uint32_t *)x, b = *(const uint32_t *)y;
    return a < b ? -1 : (a > b);
}

int orc_certify(const double *X, const int64_t *keys, int64_t n, int D, const int32_t *rows,
                int64_t m, orc_cert_t *out, int32_t **hull_out, int64_t *nhull) {
    memset(out, 0, sizeof(*out));
    *hull_out = NULL;
    *nhull = 0;
    if ((D != 2 && D != 3) || n < 0 || m < 0) return ORC_INVALID;
    const int V = D + 1;
    int64_t *kk = NULL;
    if (!keys) {
        kk = malloc(sizeof(int64_t) * (size_t)(n + 1));
        if (!kk) return ORC_NOMEM;
        for (int64_t i = 0; i < n; i++) kk[i] = i;
        keys = kk;
    }
    uint8_t *used = calloc((size_t)n + 1, 1);
    int64_t *fcnt = calloc((size_t)n + 1, sizeof(int64_t));   /* facets per smallest vertex */
    int64_t *ecnt = calloc((size_t)n + 1, sizeof(int64_t));   /* edges per smallest vertex */
    int32_t *srt = malloc(sizeof(int32_t) * (size_t)(m * V + 1));
    uint8_t *okrow = malloc((size_t)m + 1);
    if (!used || !fcnt || !ecnt || !srt || !okrow) {
        free(used); free(fcnt); free(ecnt); free(srt); free(okrow); free(kk);
        return ORC_NOMEM;
    }
    long double vol = 0.0L;
    const double fact = (D == 2) ? 2.0 : 6.0;
    /* rows: validity, orientation, volume; sorted copies */
    for (int64_t r = 0; r < m; r++) {
        int32_t *v = srt + r * V;
        int ok = 1;
        for (int i = 0; i < V; i++) {
            v[i] = rows[r * V + i];
            if (v[i] < 0 || v[i] >= n) ok = 0;
        }
        for (int i = 1; i < V; i++)
            for (int j = i; j > 0 && v[j] < v[j - 1]; j--) {
                int32_t t = v[j]; v[j] = v[j - 1]; v[j - 1] = t;
            }
        for (int i = 1; i < V && ok; i++)
            if (v[i] == v[i - 1]) ok = 0;
        okrow[r] = (uint8_t)ok;
        if (!ok) { out->bad_rows++; continue; }
        const double *P[4];
        for (int i = 0; i < V; i++) P[i] = X + (int64_t)v[i] * D;
        if (orient1(D, P) == 0) out->flat++;
        double det;
        if (D == 2) {
            det = (P[1][0] - P[0][0]) * (P[2][1] - P[0][1]) - (P[1][1] - P[0][1]) * (P[2][0] - P[0][0]);
        } else {
            double a[3], b[3], c[3];
            for (int k = 0; k < 3; k++) {
                a[k] = P[1][k] - P[0][k];
                b[k] = P[2][k] - P[0][k];
                c[k] = P[3][k] - P[0][k];
            }
            det = a[0] * (b[1] * c[2] - b[2] * c[1]) - a[1] * (b[0] * c[2] - b[2] * c[0]) +
                  a[2] * (b[0] * c[1] - b[1] * c[0]);
        }
        vol += (long double)fabs(det) / fact;
        for (int i = 0; i < V; i++) used[v[i]] = 1;
        for (int j = 0; j < V; j++) fcnt[v[j == 0 ? 1 : 0]]++;
        for (int i = 0; i < V; i++)
            for (int j = i + 1; j < V; j++) ecnt[v[i]]++;
    }
    out->volume = (double)vol;
    for (int64_t i = 0; i < n; i++)
        if (!used[i]) out->unused++;
    /* bucket the facets by their smallest vertex (counting sort) */
    int64_t *fstart = malloc(sizeof(int64_t) * (size_t)(n + 1));
    int64_t *estart = malloc(sizeof(int64_t) * (size_t)(n + 1));
    if (!fstart || !estart) {
        free(used); free(fcnt); free(ecnt); free(srt); free(okrow); free(kk);
        free(fstart); free(estart);
        return ORC_NOMEM;
    }
    int64_t fs = 0, es = 0;
    for (int64_t i = 0; i < n; i++) {
        fstart[i] = fs; fs += fcnt[i]; fcnt[i] = fstart[i];
        estart[i] = es; es += ecnt[i]; ecnt[i] = estart[i];
    }
    fstart[n] = fs;
    estart[n] = es;
    facet_t *F = malloc(sizeof(facet_t) * (size_t)(fs + 1));
    uint32_t *E = malloc(sizeof(uint32_t) * (size_t)(es + 1));
    if (!F || !E) {
        free(used); free(fcnt); free(ecnt); free(srt); free(okrow); free(kk);
        free(fstart); free(estart); free(F); free(E);
        return ORC_NOMEM;
    }
    for (int64_t r = 0; r < m; r++) {
        if (!okrow[r]) continue;
        const int32_t *v = srt + r * V;
        for (int j = 0; j < V; j++) {
            int32_t f[3];
            int c = 0;
            for (int i = 0; i < V; i++)
                if (i != j) f[c++] = v[i];
            facet_t x;
            x.a = (uint32_t)f[1];
            x.b = (D == 3) ? (uint32_t)f[2] : 0u;
            x.row = (uint32_t)r;
            x.j = j;
            F[fcnt[f[0]]++] = x;
        }
        for (int i = 0; i < V; i++)
            for (int j = i + 1; j < V; j++) E[ecnt[v[i]]++] = (uint32_t)v[j];
    }
    /* distinct edges */
    for (int64_t u = 0; u < n; u++) {
        int64_t a = estart[u], b = estart[u + 1];
        if (b - a > 1) qsort(E + a, (size_t)(b - a), sizeof(uint32_t), u32_cmp);
        for (int64_t i = a; i < b; i++)
            if (i == a || E[i] != E[i - 1]) out->edges++;
    }
    /* facets: pairing, sides, local Delaunay */
    int64_t hcap = 1024, hn = 0;
    int32_t *H = malloc(sizeof(int32_t) * (size_t)hcap * D);
    int st = H ? ORC_OK : ORC_NOMEM;
    for (int64_t u = 0; u < n && st == ORC_OK; u++) {
        int64_t a = fstart[u], b = fstart[u + 1];
        if (b - a > 1) qsort(F + a, (size_t)(b - a), sizeof(facet_t), facet_cmp);
        for (int64_t i = a; i < b;) {
            int64_t e = i + 1;
            while (e < b && F[e].a == F[i].a && F[e].b == F[i].b) e++;
            int32_t fv[3] = {(int32_t)u, (int32_t)F[i].a, (int32_t)F[i].b};
            if (e - i > 2) {
                out->over_shared++;
            } else if (e - i == 1) {
                out->hull++;
                if (hn == hcap) {
                    int32_t *h2 = realloc(H, sizeof(int32_t) * (size_t)hcap * 2 * D);
                    if (!h2) { st = ORC_NOMEM; break; }
                    H = h2;
                    hcap *= 2;
                }
                for (int k = 0; k < D; k++) H[hn * D + k] = fv[k];
                hn++;
            } else {
                out->interior++;
                const int32_t *r1 = srt + (int64_t)F[i].row * V, *r2 = srt + (int64_t)F[i + 1].row * V;
                int32_t pa = r1[F[i].j], pb = r2[F[i + 1].j];
                const double *P[5];
                int64_t kq[5];
                for (int k = 0; k < D; k++) { P[k] = X + (int64_t)fv[k] * D; kq[k] = keys[fv[k]]; }
                P[D] = X + (int64_t)pa * D;
                kq[D] = keys[pa];
                int oa = orient1(D, P);
                P[D] = X + (int64_t)pb * D;
                int ob = orient1(D, P);
                if (oa == 0 || ob == 0 || oa == ob) out->same_side++;
                /* pb against the circumsphere of (facet, pa) */
                P[D] = X + (int64_t)pa * D;
                P[D + 1] = X + (int64_t)pb * D;
                kq[D + 1] = keys[pb];
                int s = in_pert(D, P, kq);
                if (oa == 0 || s == 0 || oa * s > 0) out->not_local++;
            }
            i = e;
        }
    }
    free(used); free(fcnt); free(ecnt); free(srt); free(okrow); free(kk);
    free(fstart); free(estart); free(F); free(E);
    if (st != ORC_OK) { free(H); return st; }
    *hull_out = H;
    *nhull = hn;
    return ORC_OK;
}

void orc_free(void *p) { free(p); }
