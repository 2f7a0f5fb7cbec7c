/*
 * fmm_oracle.c -- TEST INFRASTRUCTURE ONLY.
 *
 * A plain, slow, single-threaded FP64 CPU implementation of the symmetric fast
 * multipole gravity solve of Zhu, "A momentum conserving N-body scheme with
 * individual timesteps" (arXiv:1712.10116), plus O(N^2) direct summation.
 * Only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark may load this file's library.  The GPU product path never calls it
 * and shares no code, header, table or constant with it.
 *
 * What each function follows (all citations are to the paper):
 *   - cell-cell well-separation test, Eq. (1), with R read as the cell half side
 *     and the extra softening-separation rule of Sec. 2.3 (cells may interact
 *     through expansions only when farther apart than eps);
 *   - oct-tree built top down by recursion, splitting a cell while it holds more
 *     than n_crit (= leaf_size) particles (Sec. 2.3);
 *   - symmetric dual tree walk that opens BOTH cells when a pair is not well
 *     separated (Sec. 2.3, Algorithm 4), run on unordered cell pairs so every
 *     cell-cell (M2L) and leaf-leaf (P2P) interaction is applied to both sides
 *     (Sec. 2.1, Eq. (2): F_ij = -F_ji);
 *   - Cartesian Taylor expansions of total degree <= p about geometric cell
 *     centres (Sec. 2.1; the paper notes Cartesian and spherical-harmonic
 *     expansions are equivalent for 1/r and that Cartesian is faster at small p,
 *     Sec. 4.2);
 *   - Wendland C2 softened potential, Eq. (8), or Plummer softening.
 *
 * Derivatives D^k psi(R) are obtained by truncated multivariate power-series
 * composition: psi is a function of s = |R+u|^2 (+eps^2 for Plummer); it is
 * Taylor expanded in delta = 2 R.u + |u|^2 around s0 = |R|^2, every power of
 * delta is formed by explicit polynomial products truncated at degree p, and
 * D^k psi = k! [u^k].  No recurrence is used, so a wrong index in a recurrence
 * elsewhere cannot be mirrored here.
 *
 * Floating point: IEEE double, round to nearest even, compiled with
 * -ffp-contract=off so that every discrete decision (root box, Morton keys,
 * octant membership, well-separation) is a fixed sequence of correctly rounded
 * operations.
 */
#include <math.h>
#include <stdint.h>
#ifdef _OPENMP
#include <omp.h>
#endif
#include <stdlib.h>
#include <string.h>

#define ORC_MAXLEVEL 21         /* 21 bits per axis -> 63-bit Morton keys */
#define ORC_PMAX 10

enum { ORC_OK = 0, ORC_EINVAL = 1, ORC_ENOMEM = 2 };
enum { ORC_WENDLAND = 0, ORC_PLUMMER = 1 };

typedef struct {
    int p;            /* expansion order: maximum total degree              */
    double theta;     /* opening angle of Eq. (1)                           */
    double eps;       /* softening length                                   */
    int leaf_size;    /* n_crit: a cell with more particles than this splits */
    int kernel;       /* ORC_WENDLAND or ORC_PLUMMER                         */
} orc_params;

typedef struct {
    int level;
    uint64_t prefix;      /* Morton key of the first particle >> 3*(21-level) */
    int64_t begin, end;   /* range in Morton-sorted order                     */
    int nchild;
    int64_t child[8];
    double z[3];          /* geometric centre                                 */
    double h;             /* half side                                        */
} orc_node;

typedef struct { int64_t a, b; } orc_pair;

typedef struct orc_tree {
    orc_params prm;
    int64_t n;
    double *x[3];         /* active positions, active order                  */
    uint64_t *key;        /* Morton key per active slot                      */
    int64_t *perm;        /* sorted position -> active slot                  */
    double lo[3], hi[3], c[3], o[3], L, s;
    orc_node *nodes;
    int64_t n_nodes, cap_nodes;
    orc_pair *m2l;
    int64_t n_m2l, cap_m2l;
    orc_pair *p2p;
    int64_t n_p2p, cap_p2p;
    int depth;
} orc_tree;

/* ------------------------------------------------------------------------ */
/* multi-index bookkeeping: all (kx,ky,kz) with kx+ky+kz <= p               */
/* ------------------------------------------------------------------------ */
typedef struct {
    int p, K;
    int k[ORC_PMAX * ORC_PMAX * ORC_PMAX + 64][3];
    int idx[ORC_PMAX + 1][ORC_PMAX + 1][ORC_PMAX + 1];
    double fact[ORC_PMAX + 1];
    /* index of the sum of multi-indices a and b, or -1 beyond degree p */
    int sum[(ORC_PMAX + 1) * (ORC_PMAX + 2) * (ORC_PMAX + 3) / 6]
           [(ORC_PMAX + 1) * (ORC_PMAX + 2) * (ORC_PMAX + 3) / 6];
} orc_mi;

static void mi_init(orc_mi *mi, int p)
{
    mi->p = p;
    mi->K = 0;
    for (int a = 0; a <= ORC_PMAX; ++a)
        for (int b = 0; b <= ORC_PMAX; ++b)
            for (int c = 0; c <= ORC_PMAX; ++c) mi->idx[a][b][c] = -1;
    for (int deg = 0; deg <= p; ++deg)
        for (int a = deg; a >= 0; --a)
            for (int b = deg - a; b >= 0; --b) {
                int c = deg - a - b;
                mi->k[mi->K][0] = a;
                mi->k[mi->K][1] = b;
                mi->k[mi->K][2] = c;
                mi->idx[a][b][c] = mi->K;
                mi->K++;
            }
    mi->fact[0] = 1.0;
    for (int i = 1; i <= ORC_PMAX; ++i) mi->fact[i] = mi->fact[i - 1] * i;
    for (int a = 0; a < mi->K; ++a)
        for (int b = 0; b < mi->K; ++b) {
            int x = mi->k[a][0] + mi->k[b][0], y = mi->k[a][1] + mi->k[b][1],
                z = mi->k[a][2] + mi->k[b][2];
            mi->sum[a][b] = x + y + z > p ? -1 : mi->idx[x][y][z];
        }
}

static double ipow(double x, int e)
{
    double r = 1.0;
    for (int i = 0; i < e; ++i) r *= x;
    return r;
}

/* u^k / k! for one multi-index */
static double mono_over_fact(const orc_mi *mi, const double u[3], int t)
{
    const int *k = mi->k[t];
    return ipow(u[0], k[0]) / mi->fact[k[0]] * (ipow(u[1], k[1]) / mi->fact[k[1]]) *
           (ipow(u[2], k[2]) / mi->fact[k[2]]);
}

static int mi_sum_idx(const orc_mi *mi, int a, int b) { return mi->sum[a][b]; }

static int mi_deg(const orc_mi *mi, int t) { return mi->k[t][0] + mi->k[t][1] + mi->k[t][2]; }

static double mi_factorial(const orc_mi *mi, int t)
{
    return mi->fact[mi->k[t][0]] * mi->fact[mi->k[t][1]] * mi->fact[mi->k[t][2]];
}

/* ------------------------------------------------------------------------ */
/* pair kernels: potential psi(r) (negative) and g = psi'(r)/r              */
/* ------------------------------------------------------------------------ */

/* Eq. (8): Wendland C2 potential of unit mass, u = r/eps < 1; -1/r outside. */
double orc_wendland_phi(double r, double eps)
{
    if (r >= eps) return -1.0 / r;
    double u = r / eps;
    return (u * u * ((u * (u * (3.0 * u - 15.0) + 28.0) - 21.0) * u * u + 7.0) - 3.0) / eps;
}

/* g = (d phi/dr) / r for Eq. (8): differentiating the polynomial of Eq. (8)
 * term by term and dividing by r = u eps gives
 * (21u^5 - 90u^4 + 140u^3 - 84u^2 + 14) / eps^3 inside, 1/r^3 outside. */
double orc_wendland_g(double r, double eps)
{
    if (r >= eps) return 1.0 / (r * r * r);
    double u = r / eps;
    double poly = 21.0 * ipow(u, 5) - 90.0 * ipow(u, 4) + 140.0 * ipow(u, 3) - 84.0 * u * u + 14.0;
    return poly / (eps * eps * eps);
}

double orc_plummer_phi(double r, double eps) { return -1.0 / sqrt(r * r + eps * eps); }

double orc_plummer_g(double r, double eps)
{
    double s = r * r + eps * eps;
    return 1.0 / (s * sqrt(s));
}

/* (dg/dr)/r, for the force gradient (Sec. 4.1): -3/r^5 outside the Wendland
 * radius; inside, differentiating g's polynomial term by term and dividing by
 * r = u eps gives (105u^3 - 360u^2 + 420u - 168) / eps^5; Plummer:
 * -3 (r^2 + eps^2)^(-5/2). */
static double pair_dg_over_r(int kernel, double eps, double r)
{
    if (kernel == ORC_PLUMMER) {
        double s = r * r + eps * eps;
        return -3.0 / (s * s * sqrt(s));
    }
    if (r >= eps) return -3.0 / (r * r * r * r * r);
    double u = r / eps;
    double e5 = eps * eps * eps * eps * eps;
    return (105.0 * ipow(u, 3) - 360.0 * u * u + 420.0 * u - 168.0) / e5;
}

static void pair_kernel(int kernel, double eps, double r, double *phi, double *g)
{
    if (kernel == ORC_PLUMMER) {
        *phi = orc_plummer_phi(r, eps);
        *g = orc_plummer_g(r, eps);
    } else {
        *phi = orc_wendland_phi(r, eps);
        *g = orc_wendland_g(r, eps);
    }
}

/* ------------------------------------------------------------------------ */
/* direct summation: the plain definition the FMM approximates              */
/* ------------------------------------------------------------------------ */

/* acc_i = sum_{j != i} m_j g(r_ij) (x_j - x_i),  pot_i = sum_{j != i} m_j psi(r_ij)
 * for the sinks listed in `sinks` (indices into the n particles); sources are
 * all n particles.  pos is SoA: x[0..n), y[n..2n), z[2n..3n). */
int orc_direct(const double *pos, const double *mass, int64_t n, const int64_t *sinks,
               int64_t n_sinks, int kernel, double eps, double *acc, double *pot)
{
    if (n < 0 || n_sinks < 0) return ORC_EINVAL;
    const double *X = pos, *Y = pos + n, *Z = pos + 2 * n;
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t t = 0; t < n_sinks; ++t) {
        int64_t i = sinks ? sinks[t] : t;
        double ax = 0, ay = 0, az = 0, ph = 0;
        for (int64_t j = 0; j < n; ++j) {
            if (j == i) continue;
            double dx = X[j] - X[i], dy = Y[j] - Y[i], dz = Z[j] - Z[i];
            double r = sqrt(dx * dx + dy * dy + dz * dz);
            double phi, g;
            pair_kernel(kernel, eps, r, &phi, &g);
            ax += mass[j] * g * dx;
            ay += mass[j] * g * dy;
            az += mass[j] * g * dz;
            ph += mass[j] * phi;
        }
        acc[t] = ax;
        acc[n_sinks + t] = ay;
        acc[2 * n_sinks + t] = az;
        pot[t] = ph;
    }
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* D^k psi(R), |k| <= p, by truncated power-series composition              */
/* ------------------------------------------------------------------------ */
static void poly_mul(const orc_mi *mi, const double *a, const double *b, double *out)
{
    for (int t = 0; t < mi->K; ++t) out[t] = 0.0;
    for (int i = 0; i < mi->K; ++i) {
        if (a[i] == 0.0) continue;
        for (int j = 0; j < mi->K; ++j) {
            int t = mi_sum_idx(mi, i, j);
            if (t >= 0) out[t] += a[i] * b[j];
        }
    }
}

/* D[t] = d^{k_t} psi / dR^{k_t} at R, for psi(R) = -(|R|^2 + e2)^(-1/2);
 * e2 = 0 for the far field of the Wendland kernel (pure Newtonian beyond eps),
 * e2 = eps^2 for the Plummer kernel. */
void orc_derivs(const orc_mi *mi, const double R[3], double e2, double *D)
{
    const int K = mi->K, p = mi->p;
    double delta[ORC_PMAX * ORC_PMAX * ORC_PMAX + 64], pw[ORC_PMAX * ORC_PMAX * ORC_PMAX + 64],
        tmp[ORC_PMAX * ORC_PMAX * ORC_PMAX + 64];
    for (int t = 0; t < K; ++t) delta[t] = 0.0;
    /* delta(u) = 2 R.u + u.u */
    if (p >= 1) {
        delta[mi->idx[1][0][0]] = 2.0 * R[0];
        delta[mi->idx[0][1][0]] = 2.0 * R[1];
        delta[mi->idx[0][0][1]] = 2.0 * R[2];
    }
    if (p >= 2) {
        delta[mi->idx[2][0][0]] = 1.0;
        delta[mi->idx[0][2][0]] = 1.0;
        delta[mi->idx[0][0][2]] = 1.0;
    }
    double s0 = R[0] * R[0] + R[1] * R[1] + R[2] * R[2] + e2;
    /* Taylor coefficients of F(s) = -s^(-1/2) about s0:
     * c_n = F^(n)(s0)/n! = -binom(-1/2, n) s0^(-1/2-n) */
    double cn = -1.0 / sqrt(s0);
    for (int t = 0; t < K; ++t) { D[t] = 0.0; pw[t] = 0.0; }
    pw[0] = 1.0;                      /* delta^0 */
    for (int n = 0; n <= p; ++n) {
        for (int t = 0; t < K; ++t) D[t] += cn * pw[t];
        if (n == p) break;
        poly_mul(mi, pw, delta, tmp);
        memcpy(pw, tmp, sizeof(double) * K);
        cn = cn * (-0.5 - n) / (n + 1) / s0;
    }
    for (int t = 0; t < K; ++t) D[t] *= mi_factorial(mi, t);
}

/* exported for the test-suite: D^k psi for one R, laid out in the oracle's
 * multi-index order (degree ascending, then kx descending, then ky
 * descending); kout receives the (kx,ky,kz) triples. */
int orc_derivs_export(int p, const double R[3], double e2, double *D, int *kout)
{
    if (p < 0 || p > ORC_PMAX) return ORC_EINVAL;
    orc_mi *mi = (orc_mi *)malloc(sizeof(orc_mi));
    if (!mi) return ORC_ENOMEM;
    mi_init(mi, p);
    orc_derivs(mi, R, e2, D);
    for (int t = 0; t < mi->K; ++t) {
        kout[3 * t] = mi->k[t][0];
        kout[3 * t + 1] = mi->k[t][1];
        kout[3 * t + 2] = mi->k[t][2];
    }
    free(mi);
    return ORC_OK;
}

/* ------------------------------------------------------------------------ */
/* tree: root box, Morton keys, stable sort, recursive split                */
/* ------------------------------------------------------------------------ */
static uint64_t morton3(uint64_t qx, uint64_t qy, uint64_t qz)
{
    uint64_t key = 0;
    for (int b = 0; b < ORC_MAXLEVEL; ++b) {
        key |= ((qx >> b) & 1ull) << (3 * b + 2);
        key |= ((qy >> b) & 1ull) << (3 * b + 1);
        key |= ((qz >> b) & 1ull) << (3 * b);
    }
    return key;
}

static uint64_t quantise(double x, double o, double s)
{
    double q = floor((x - o) * s);
    const double qmax = (double)((1u << ORC_MAXLEVEL) - 1u);
    if (!(q >= 0.0)) q = 0.0;
    if (q > qmax) q = qmax;
    return (uint64_t)q;
}

static const orc_tree *g_sort_tree;
static int cmp_slot(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    uint64_t ka = g_sort_tree->key[a], kb = g_sort_tree->key[b];
    if (ka != kb) return ka < kb ? -1 : 1;
    return a < b ? -1 : (a > b ? 1 : 0);
}

static int push_node(orc_tree *t)
{
    if (t->n_nodes == t->cap_nodes) {
        int64_t cap = t->cap_nodes ? 2 * t->cap_nodes : 64;
        orc_node *nn = (orc_node *)realloc(t->nodes, sizeof(orc_node) * cap);
        if (!nn) return -1;
        t->nodes = nn;
        t->cap_nodes = cap;
    }
    t->n_nodes++;
    return 1;
}

static int64_t build_rec(orc_tree *t, int level, int64_t begin, int64_t end)
{
    if (!push_node(t)) return -1;
    int64_t id = t->n_nodes - 1;
    orc_node *nd = &t->nodes[id];
    memset(nd, 0, sizeof(*nd));
    nd->level = level;
    nd->begin = begin;
    nd->end = end;
    nd->prefix = t->n ? (t->key[t->perm[begin]] >> (3 * (ORC_MAXLEVEL - level))) : 0;
    if (level > t->depth) t->depth = level;
    /* geometry: centre and half side from the key prefix */
    uint64_t ic[3] = {0, 0, 0};
    for (int b = 0; b < level; ++b) {
        ic[0] |= ((nd->prefix >> (3 * b + 2)) & 1ull) << b;
        ic[1] |= ((nd->prefix >> (3 * b + 1)) & 1ull) << b;
        ic[2] |= ((nd->prefix >> (3 * b)) & 1ull) << b;
    }
    double w = ldexp(t->L, -level);
    for (int d = 0; d < 3; ++d) nd->z[d] = t->o[d] + ((double)ic[d] + 0.5) * w;
    nd->h = ldexp(t->L, -(level + 1));

    if (end - begin > t->prm.leaf_size && level < ORC_MAXLEVEL) {
        int shift = 3 * (ORC_MAXLEVEL - (level + 1));
        int64_t i = begin;
        int nc = 0;
        int64_t kids[8];
        while (i < end) {
            uint64_t oct = (t->key[t->perm[i]] >> shift) & 7ull;
            int64_t j = i;
            while (j < end && ((t->key[t->perm[j]] >> shift) & 7ull) == oct) ++j;
            int64_t c = build_rec(t, level + 1, i, j);
            if (c < 0) return -1;
            kids[nc++] = c;
            i = j;
        }
        nd = &t->nodes[id];  /* realloc may have moved the array */
        nd->nchild = nc;
        for (int k = 0; k < nc; ++k) nd->child[k] = kids[k];
    }
    return id;
}

/* Eq. (1) with R = half side, plus the softening-separation rule: the
 * minimum distance between the two cubes, bounded below by
 * |zA - zB| - sqrt(3)(hA + hB), must exceed eps.  Evaluated squared. */
static int well_separated(const orc_tree *t, const orc_node *A, const orc_node *B)
{
    double dx = A->z[0] - B->z[0];
    double dy = A->z[1] - B->z[1];
    double dz = A->z[2] - B->z[2];
    double d2 = (dx * dx + dy * dy) + dz * dz;
    double S = A->h + B->h;
    double th2 = t->prm.theta * t->prm.theta;
    int mac = d2 * th2 > S * S;
    double e = t->prm.eps + sqrt(3.0) * S;
    int sep = d2 > e * e;
    return mac && sep;
}

static int push_pair(orc_pair **arr, int64_t *n, int64_t *cap, int64_t a, int64_t b)
{
    if (*n == *cap) {
        int64_t c = *cap ? 2 * *cap : 256;
        orc_pair *na = (orc_pair *)realloc(*arr, sizeof(orc_pair) * c);
        if (!na) return -1;
        *arr = na;
        *cap = c;
    }
    (*arr)[*n].a = a < b ? a : b;
    (*arr)[*n].b = a < b ? b : a;
    (*n)++;
    return 0;
}

/* Symmetric dual walk over unordered cell pairs (Algorithm 4, open-both). */
static int walk(orc_tree *t, int64_t ia, int64_t ib)
{
    const orc_node *A = &t->nodes[ia], *B = &t->nodes[ib];
    if (ia == ib) {
        if (A->nchild == 0) return push_pair(&t->p2p, &t->n_p2p, &t->cap_p2p, ia, ia);
        for (int i = 0; i < A->nchild; ++i)
            for (int j = i; j < A->nchild; ++j)
                if (walk(t, A->child[i], A->child[j])) return -1;
        return 0;
    }
    if (well_separated(t, A, B)) return push_pair(&t->m2l, &t->n_m2l, &t->cap_m2l, ia, ib);
    if (A->nchild == 0 && B->nchild == 0)
        return push_pair(&t->p2p, &t->n_p2p, &t->cap_p2p, ia, ib);
    if (A->nchild == 0) {
        for (int j = 0; j < B->nchild; ++j)
            if (walk(t, ia, B->child[j])) return -1;
        return 0;
    }
    if (B->nchild == 0) {
        for (int i = 0; i < A->nchild; ++i)
            if (walk(t, A->child[i], ib)) return -1;
        return 0;
    }
    for (int i = 0; i < A->nchild; ++i)
        for (int j = 0; j < B->nchild; ++j)
            if (walk(t, A->child[i], B->child[j])) return -1;
    return 0;
}

static int cmp_pair(const void *pa, const void *pb)
{
    const orc_pair *a = (const orc_pair *)pa, *b = (const orc_pair *)pb;
    if (a->a != b->a) return a->a < b->a ? -1 : 1;
    if (a->b != b->b) return a->b < b->b ? -1 : 1;
    return 0;
}

void orc_tree_free(orc_tree *t)
{
    if (!t) return;
    for (int d = 0; d < 3; ++d) free(t->x[d]);
    free(t->key);
    free(t->perm);
    free(t->nodes);
    free(t->m2l);
    free(t->p2p);
    free(t);
}

/* Build the tree and the interaction lists for the active particles.
 * pos: SoA FP64 of n_total particles; active: n_active unique indices, or NULL
 * for all n_total in order. */
orc_tree *orc_tree_build(const double *pos, int64_t n_total, const int32_t *active,
                         int64_t n_active, const orc_params *prm)
{
    if (!prm || prm->p < 0 || prm->p > ORC_PMAX || prm->leaf_size < 1 || n_active < 0 ||
        !(prm->theta > 0.0) || prm->eps < 0.0)
        return NULL;
    orc_tree *t = (orc_tree *)calloc(1, sizeof(orc_tree));
    if (!t) return NULL;
    t->prm = *prm;
    t->n = n_active;
    int64_t n = n_active;
    for (int d = 0; d < 3; ++d) t->x[d] = (double *)malloc(sizeof(double) * (n ? n : 1));
    t->key = (uint64_t *)malloc(sizeof(uint64_t) * (n ? n : 1));
    t->perm = (int64_t *)malloc(sizeof(int64_t) * (n ? n : 1));
    if (!t->x[0] || !t->x[1] || !t->x[2] || !t->key || !t->perm) {
        orc_tree_free(t);
        return NULL;
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t g = active ? active[i] : i;
        for (int d = 0; d < 3; ++d) t->x[d][i] = pos[d * n_total + g];
    }
    /* root box */
    for (int d = 0; d < 3; ++d) {
        double lo = n ? t->x[d][0] : 0.0, hi = lo;
        for (int64_t i = 1; i < n; ++i) {
            if (t->x[d][i] < lo) lo = t->x[d][i];
            if (t->x[d][i] > hi) hi = t->x[d][i];
        }
        t->lo[d] = lo;
        t->hi[d] = hi;
        t->c[d] = 0.5 * (lo + hi);
    }
    double L = 0.0;
    for (int d = 0; d < 3; ++d) {
        double e = t->hi[d] - t->lo[d];
        if (e > L) L = e;
    }
    if (L == 0.0) L = 1.0;
    t->L = L;
    for (int d = 0; d < 3; ++d) t->o[d] = t->c[d] - 0.5 * L;
    t->s = 2097152.0 / L;  /* 2^21 / L */
    for (int64_t i = 0; i < n; ++i) {
        uint64_t q[3];
        for (int d = 0; d < 3; ++d) q[d] = quantise(t->x[d][i], t->o[d], t->s);
        t->key[i] = morton3(q[0], q[1], q[2]);
        t->perm[i] = i;
    }
    g_sort_tree = t;
    qsort(t->perm, (size_t)n, sizeof(int64_t), cmp_slot);
    g_sort_tree = NULL;
    if (n > 0) {
        if (build_rec(t, 0, 0, n) < 0 || walk(t, 0, 0) < 0) {
            orc_tree_free(t);
            return NULL;
        }
        qsort(t->m2l, (size_t)t->n_m2l, sizeof(orc_pair), cmp_pair);
        qsort(t->p2p, (size_t)t->n_p2p, sizeof(orc_pair), cmp_pair);
    }
    return t;
}

/* info[0..5] = n, n_nodes, n_m2l, n_p2p, depth, n_leaves */
void orc_tree_info(const orc_tree *t, int64_t *info)
{
    int64_t leaves = 0;
    for (int64_t i = 0; i < t->n_nodes; ++i) leaves += t->nodes[i].nchild == 0;
    info[0] = t->n;
    info[1] = t->n_nodes;
    info[2] = t->n_m2l;
    info[3] = t->n_p2p;
    info[4] = t->depth;
    info[5] = leaves;
}

/* Canonical export: nodes in pre-order, pairs (a <= b) sorted, perm as the
 * active slot of each Morton-sorted position.  Any pointer may be NULL. */
void orc_tree_export(const orc_tree *t, int64_t *perm, int32_t *level, uint64_t *prefix,
                     int64_t *begin, int64_t *end, int32_t *is_leaf, double *centre,
                     double *half, int64_t *m2l, int64_t *p2p, double *box)
{
    if (perm)
        for (int64_t i = 0; i < t->n; ++i) perm[i] = t->perm[i];
    for (int64_t i = 0; i < t->n_nodes; ++i) {
        const orc_node *nd = &t->nodes[i];
        if (level) level[i] = nd->level;
        if (prefix) prefix[i] = nd->prefix;
        if (begin) begin[i] = nd->begin;
        if (end) end[i] = nd->end;
        if (is_leaf) is_leaf[i] = nd->nchild == 0;
        if (centre)
            for (int d = 0; d < 3; ++d) centre[3 * i + d] = nd->z[d];
        if (half) half[i] = nd->h;
    }
    if (m2l)
        for (int64_t i = 0; i < t->n_m2l; ++i) {
            m2l[2 * i] = t->m2l[i].a;
            m2l[2 * i + 1] = t->m2l[i].b;
        }
    if (p2p)
        for (int64_t i = 0; i < t->n_p2p; ++i) {
            p2p[2 * i] = t->p2p[i].a;
            p2p[2 * i + 1] = t->p2p[i].b;
        }
    if (box) {
        for (int d = 0; d < 3; ++d) box[d] = t->o[d];
        box[3] = t->L;
        box[4] = t->s;
    }
}

/* ------------------------------------------------------------------------ */
/* evaluation: P2M, M2M, M2L (mutual), L2L, L2P, P2P (mutual)               */
/* ------------------------------------------------------------------------ */

/* Multipoles and locals of every node are written to Mout/Lout (n_nodes x K,
 * row-major) when non-NULL, for the test-suite. */
/* grad (optional, SoA 6 x n: xx, yy, zz, xy, xz, yz): the force gradient
 * d a_i / d x_i of every sink (the tidal tensor, Sec. 4.1), from the same
 * expansions: minus the Hessian of the local expansion at L2P, and for every
 * P2P pair the derivative of m g(r) d with respect to the sink's position,
 * -m (g I + (dg/dr)/r d d^T), d = x_j - x_i, applied to both sides. */
/* dvec (optional, SoA 3 x n in active order): instead of point masses the
 * sources are vectors m_j v_j, and the outputs become the field
 * u_i = sum_j m_j H(x_i - x_j) v_j, H = grad grad psi (the pair Hessian,
 * g I + (dg/dr)/r d d^T), written to acc, and Phi_i = sum_j m_j v_j . grad psi
 * (x_i - x_j), written to pot.  This is the derivative of the accelerations
 * along a displacement of every particle j by v_j: sum_{j != i} (d a_i /
 * d x_j) v_j.  Through the same expansions: a source's "dipole moments"
 * M[m] = -m_j sum_a v_a (x_j - z)^(m - e_a) / (m - e_a)! (the derivative of its
 * mass moments along v), the same M2M, M2L and L2L, and u = +grad of the
 * local expansion; the near part sums m_j H v_j over the P2P partners. */
static int tree_eval(const orc_tree *t, const double *mass_total, int64_t n_total,
                     const int32_t *active, const double *dvec, double *acc, double *pot,
                     double *grad, double *Mout, double *Lout)
{
    const int64_t n = t->n;
    if (n == 0) return ORC_OK;
    const int p = t->prm.p;
    orc_mi *mi = (orc_mi *)malloc(sizeof(orc_mi));
    if (!mi) return ORC_ENOMEM;
    mi_init(mi, p);
    const int K = mi->K;
    const int64_t NN = t->n_nodes;
    double *M = (double *)calloc((size_t)(NN * K), sizeof(double));
    double *Lc = (double *)calloc((size_t)(NN * K), sizeof(double));
    double *m = (double *)malloc(sizeof(double) * n);        /* mass, sorted order */
    double *sx[3];
    for (int d = 0; d < 3; ++d) sx[d] = (double *)malloc(sizeof(double) * n);
    double *ax = (double *)calloc((size_t)n, sizeof(double));
    double *ay = (double *)calloc((size_t)n, sizeof(double));
    double *az = (double *)calloc((size_t)n, sizeof(double));
    double *ph = (double *)calloc((size_t)n, sizeof(double));
    double *D = (double *)malloc(sizeof(double) * K);
    double *G = grad ? (double *)calloc((size_t)(6 * n), sizeof(double)) : NULL;
    double *V = dvec ? (double *)malloc(sizeof(double) * 3 * n) : NULL; /* sorted order */
    if (!M || !Lc || !m || !sx[0] || !sx[1] || !sx[2] || !ax || !ay || !az || !ph || !D ||
        (grad && !G) || (dvec && !V)) {
        free(mi); free(M); free(Lc); free(m); free(sx[0]); free(sx[1]); free(sx[2]);
        free(ax); free(ay); free(az); free(ph); free(D); free(G); free(V);
        return ORC_ENOMEM;
    }
    /* tensor component c = (a, b): xx, yy, zz, xy, xz, yz */
    static const int ca[6] = {0, 1, 2, 0, 0, 1}, cb[6] = {0, 1, 2, 1, 2, 2};
    for (int64_t i = 0; i < n; ++i) {
        int64_t slot = t->perm[i];
        int64_t g = active ? active[slot] : slot;
        m[i] = mass_total[g];
        for (int d = 0; d < 3; ++d) sx[d][i] = t->x[d][slot];
        if (V)
            for (int d = 0; d < 3; ++d) V[d * n + i] = dvec[d * n + slot];
    }
    (void)n_total;
    const double e2 = t->prm.kernel == ORC_PLUMMER ? t->prm.eps * t->prm.eps : 0.0;

    /* P2M at leaves: M[k] = sum_j m_j (x_j - z)^k / k! */
    for (int64_t c = 0; c < NN; ++c) {
        const orc_node *nd = &t->nodes[c];
        if (nd->nchild) continue;
        for (int64_t i = nd->begin; i < nd->end; ++i) {
            double u[3] = {sx[0][i] - nd->z[0], sx[1][i] - nd->z[1], sx[2][i] - nd->z[2]};
            if (!V) {
                for (int k = 0; k < K; ++k) M[c * K + k] += m[i] * mono_over_fact(mi, u, k);
                continue;
            }
            /* dipole moments: -m v . grad_x of (x - z)^k / k! */
            for (int k = 0; k < K; ++k) {
                const int *kk = mi->k[k];
                double s = 0.0;
                for (int a = 0; a < 3; ++a) {
                    if (kk[a] == 0) continue;
                    int e[3] = {kk[0], kk[1], kk[2]};
                    e[a] -= 1;
                    s += V[a * n + i] * mono_over_fact(mi, u, mi->idx[e[0]][e[1]][e[2]]);
                }
                M[c * K + k] -= m[i] * s;
            }
        }
    }
    /* M2M: children have larger pre-order ids than their parent */
    for (int64_t c = NN - 1; c >= 0; --c) {
        const orc_node *P = &t->nodes[c];
        for (int q = 0; q < P->nchild; ++q) {
            const orc_node *C = &t->nodes[P->child[q]];
            double d[3] = {C->z[0] - P->z[0], C->z[1] - P->z[1], C->z[2] - P->z[2]};
            for (int mm = 0; mm < K; ++mm) {
                const int *km = mi->k[mm];
                double acc_m = 0.0;
                for (int kk = 0; kk < K; ++kk) {
                    const int *kk3 = mi->k[kk];
                    if (kk3[0] > km[0] || kk3[1] > km[1] || kk3[2] > km[2]) continue;
                    int diff = mi->idx[km[0] - kk3[0]][km[1] - kk3[1]][km[2] - kk3[2]];
                    acc_m += M[P->child[q] * K + kk] * mono_over_fact(mi, d, diff);
                }
                M[c * K + mm] += acc_m;
            }
        }
    }
    /* M2L, mutual: D^k psi(R) formed once per unordered pair, R = zA - zB. */
    for (int64_t q = 0; q < t->n_m2l; ++q) {
        int64_t ia = t->m2l[q].a, ib = t->m2l[q].b;
        const orc_node *A = &t->nodes[ia], *B = &t->nodes[ib];
        double R[3] = {A->z[0] - B->z[0], A->z[1] - B->z[1], A->z[2] - B->z[2]};
        orc_derivs(mi, R, e2, D);
        for (int nn = 0; nn < K; ++nn) {
            int dn = mi_deg(mi, nn);
            double la = 0.0, lb = 0.0;
            for (int mm = 0; mm < K; ++mm) {
                int s = mi_sum_idx(mi, nn, mm);
                if (s < 0) continue;
                double sgn_m = (mi_deg(mi, mm) & 1) ? -1.0 : 1.0;
                la += sgn_m * M[ib * K + mm] * D[s];
                lb += M[ia * K + mm] * D[s];
            }
            Lc[ia * K + nn] += la;
            Lc[ib * K + nn] += ((dn & 1) ? -1.0 : 1.0) * lb;
        }
    }
    /* L2L: parents before children in pre-order */
    for (int64_t c = 0; c < NN; ++c) {
        const orc_node *P = &t->nodes[c];
        for (int q = 0; q < P->nchild; ++q) {
            int64_t ic = P->child[q];
            const orc_node *C = &t->nodes[ic];
            double d[3] = {C->z[0] - P->z[0], C->z[1] - P->z[1], C->z[2] - P->z[2]};
            for (int nn = 0; nn < K; ++nn) {
                const int *kn = mi->k[nn];
                double acc_n = 0.0;
                for (int kk = 0; kk < K; ++kk) {
                    const int *k3 = mi->k[kk];
                    if (k3[0] < kn[0] || k3[1] < kn[1] || k3[2] < kn[2]) continue;
                    int diff = mi->idx[k3[0] - kn[0]][k3[1] - kn[1]][k3[2] - kn[2]];
                    acc_n += Lc[c * K + kk] * mono_over_fact(mi, d, diff);
                }
                Lc[ic * K + nn] += acc_n;
            }
        }
    }
    /* L2P: potential and minus its gradient from the local expansion */
    for (int64_t c = 0; c < NN; ++c) {
        const orc_node *nd = &t->nodes[c];
        if (nd->nchild) continue;
        for (int64_t i = nd->begin; i < nd->end; ++i) {
            double u[3] = {sx[0][i] - nd->z[0], sx[1][i] - nd->z[1], sx[2][i] - nd->z[2]};
            double f = 0.0, g[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < K; ++k) {
                double mono = mono_over_fact(mi, u, k);
                f += mono * Lc[c * K + k];
                const int *kk = mi->k[k];
                if (kk[0] + kk[1] + kk[2] < p) {
                    g[0] += mono * Lc[c * K + mi->idx[kk[0] + 1][kk[1]][kk[2]]];
                    g[1] += mono * Lc[c * K + mi->idx[kk[0]][kk[1] + 1][kk[2]]];
                    g[2] += mono * Lc[c * K + mi->idx[kk[0]][kk[1]][kk[2] + 1]];
                }
            }
            ph[i] += f;
            ax[i] -= g[0];
            ay[i] -= g[1];
            az[i] -= g[2];
            if (G) { /* minus the Hessian: L[k + e_a + e_b] for |k| <= p - 2 */
                for (int k = 0; k < K; ++k) {
                    const int *kk = mi->k[k];
                    if (kk[0] + kk[1] + kk[2] > p - 2) continue;
                    double mono = mono_over_fact(mi, u, k);
                    for (int c6 = 0; c6 < 6; ++c6) {
                        int e[3] = {kk[0], kk[1], kk[2]};
                        e[ca[c6]] += 1;
                        e[cb[c6]] += 1;
                        G[c6 * n + i] -= mono * Lc[c * K + mi->idx[e[0]][e[1]][e[2]]];
                    }
                }
            }
        }
    }
    /* P2P, mutual: each unordered particle pair evaluated once */
    for (int64_t q = 0; q < t->n_p2p; ++q) {
        const orc_node *A = &t->nodes[t->p2p[q].a], *B = &t->nodes[t->p2p[q].b];
        int self = t->p2p[q].a == t->p2p[q].b;
        for (int64_t i = A->begin; i < A->end; ++i) {
            for (int64_t j = self ? i + 1 : B->begin; j < B->end; ++j) {
                double dx = sx[0][j] - sx[0][i], dy = sx[1][j] - sx[1][i],
                       dz = sx[2][j] - sx[2][i];
                double r = sqrt(dx * dx + dy * dy + dz * dz);
                double phi, g;
                pair_kernel(t->prm.kernel, t->prm.eps, r, &phi, &g);
                if (V) {
                    /* H v = g v + h (d . v) d with d = +-(x_j - x_i) (H is even);
                     * acc holds minus the field, as for masses */
                    const double h = pair_dg_over_r(t->prm.kernel, t->prm.eps, r);
                    const double vj[3] = {V[j], V[n + j], V[2 * n + j]};
                    const double vi[3] = {V[i], V[n + i], V[2 * n + i]};
                    const double dvj = dx * vj[0] + dy * vj[1] + dz * vj[2];
                    const double dvi = dx * vi[0] + dy * vi[1] + dz * vi[2];
                    ax[i] -= m[j] * (g * vj[0] + h * dvj * dx);
                    ay[i] -= m[j] * (g * vj[1] + h * dvj * dy);
                    az[i] -= m[j] * (g * vj[2] + h * dvj * dz);
                    ph[i] -= m[j] * g * dvj;  /* v_j . grad psi(x_i - x_j), x_i - x_j = -d */
                    ax[j] -= m[i] * (g * vi[0] + h * dvi * dx);
                    ay[j] -= m[i] * (g * vi[1] + h * dvi * dy);
                    az[j] -= m[i] * (g * vi[2] + h * dvi * dz);
                    ph[j] += m[i] * g * dvi;
                    continue;
                }
                ax[i] += m[j] * g * dx;
                ay[i] += m[j] * g * dy;
                az[i] += m[j] * g * dz;
                ph[i] += m[j] * phi;
                ax[j] -= m[i] * g * dx;
                ay[j] -= m[i] * g * dy;
                az[j] -= m[i] * g * dz;
                ph[j] += m[i] * phi;
                if (G) {
                    double h = pair_dg_over_r(t->prm.kernel, t->prm.eps, r);
                    double dv[3] = {dx, dy, dz};
                    for (int c6 = 0; c6 < 6; ++c6) {
                        double T = -h * dv[ca[c6]] * dv[cb[c6]] - (ca[c6] == cb[c6] ? g : 0.0);
                        G[c6 * n + i] += m[j] * T;
                        G[c6 * n + j] += m[i] * T;
                    }
                }
            }
        }
    }
    /* outputs in active order */
    const double sgn = V ? -1.0 : 1.0;  /* the vector field is +grad, acc is -grad */
    for (int64_t i = 0; i < n; ++i) {
        int64_t slot = t->perm[i];
        acc[slot] = sgn * ax[i];
        acc[n + slot] = sgn * ay[i];
        acc[2 * n + slot] = sgn * az[i];
        pot[slot] = ph[i];
        if (G)
            for (int c6 = 0; c6 < 6; ++c6) grad[c6 * n + slot] = G[c6 * n + i];
    }
    if (Mout) memcpy(Mout, M, sizeof(double) * NN * K);
    if (Lout) memcpy(Lout, Lc, sizeof(double) * NN * K);
    free(mi); free(M); free(Lc); free(m); free(sx[0]); free(sx[1]); free(sx[2]);
    free(ax); free(ay); free(az); free(ph); free(D); free(G); free(V);
    return ORC_OK;
}

int orc_tree_eval_ex(const orc_tree *t, const double *mass_total, int64_t n_total,
                     const int32_t *active, double *acc, double *pot, double *Mout, double *Lout)
{
    return tree_eval(t, mass_total, n_total, active, NULL, acc, pot, NULL, Mout, Lout);
}

int orc_tree_eval_grad(const orc_tree *t, const double *mass_total, int64_t n_total,
                       const int32_t *active, double *acc, double *pot, double *grad)
{
    if (!grad) return ORC_EINVAL;
    return tree_eval(t, mass_total, n_total, active, NULL, acc, pot, grad, NULL, NULL);
}

/* The field of vector sources m_j v_j (see tree_eval): u (SoA 3 x n) and
 * phi (n), active order; vec SoA 3 x n in active order. */
int orc_tree_eval_dipole(const orc_tree *t, const double *mass_total, int64_t n_total,
                         const int32_t *active, const double *vec, double *u, double *phi)
{
    if (!vec) return ORC_EINVAL;
    return tree_eval(t, mass_total, n_total, active, vec, u, phi, NULL, NULL, NULL);
}

int orc_tree_eval(const orc_tree *t, const double *mass_total, int64_t n_total,
                  const int32_t *active, double *acc, double *pot)
{
    return orc_tree_eval_ex(t, mass_total, n_total, active, acc, pot, NULL, NULL);
}

/* tree_eval's evaluation (point masses; acceleration and potential) spread
 * over OpenMP threads for timing on many cores, with every sum formed in the
 * order tree_eval forms it, so that the results equal tree_eval's bit for bit
 * whatever the thread count.  P2M and L2P are independent per leaf, M2M per
 * parent (levels deepest first) and L2L per child (levels root first).  The
 * mutual M2L and P2P loops, which add each pair's terms to both of its cells
 * in pair order, become gathers: every cell walks the pairs it belongs to in
 * increasing pair index and forms its own side's terms exactly as the pair
 * loop does (the derivative tensor and the pair kernel depend only on the
 * pair), so it receives the same terms in the same order.  The derivative
 * tensors are formed once per pair beforehand; the P2P pair kernel is
 * evaluated once per side. */
static int64_t *pair_members(const orc_pair *pr, int64_t np, int64_t nn, int64_t **start)
{
    int64_t *cnt = (int64_t *)calloc((size_t)(nn + 1), sizeof(int64_t));
    if (!cnt) return NULL;
    for (int64_t q = 0; q < np; ++q) {
        cnt[pr[q].a + 1]++;
        if (pr[q].b != pr[q].a) cnt[pr[q].b + 1]++;
    }
    for (int64_t c = 0; c < nn; ++c) cnt[c + 1] += cnt[c];
    int64_t *list = (int64_t *)malloc(sizeof(int64_t) * (size_t)(cnt[nn] ? cnt[nn] : 1));
    int64_t *fill = (int64_t *)malloc(sizeof(int64_t) * (size_t)(nn ? nn : 1));
    if (!list || !fill) {
        free(cnt); free(list); free(fill);
        return NULL;
    }
    memcpy(fill, cnt, sizeof(int64_t) * (size_t)nn);
    for (int64_t q = 0; q < np; ++q) {  /* increasing q within every cell */
        list[fill[pr[q].a]++] = q;
        if (pr[q].b != pr[q].a) list[fill[pr[q].b]++] = q;
    }
    free(fill);
    *start = cnt;
    return list;
}

int orc_tree_eval_par(const orc_tree *t, const double *mass_total, int64_t n_total,
                      const int32_t *active, double *acc, double *pot)
{
    const int64_t n = t->n;
    if (n == 0) return ORC_OK;
    (void)n_total;
    const int p = t->prm.p;
    orc_mi *mi = (orc_mi *)malloc(sizeof(orc_mi));
    if (!mi) return ORC_ENOMEM;
    mi_init(mi, p);
    const int K = mi->K;
    const int64_t NN = t->n_nodes;
    double *M = (double *)calloc((size_t)(NN * K), sizeof(double));
    double *Lc = (double *)calloc((size_t)(NN * K), sizeof(double));
    double *m = (double *)malloc(sizeof(double) * n);
    double *sx[3];
    for (int d = 0; d < 3; ++d) sx[d] = (double *)malloc(sizeof(double) * n);
    double *ax = (double *)calloc((size_t)n, sizeof(double));
    double *ay = (double *)calloc((size_t)n, sizeof(double));
    double *az = (double *)calloc((size_t)n, sizeof(double));
    double *ph = (double *)calloc((size_t)n, sizeof(double));
    int64_t *lvl_cnt = (int64_t *)calloc(ORC_MAXLEVEL + 2, sizeof(int64_t));
    int64_t *by_lvl = (int64_t *)malloc(sizeof(int64_t) * (size_t)(NN ? NN : 1));
    int64_t *m2l_start = NULL, *p2p_start = NULL;
    int64_t *m2l_of = pair_members(t->m2l, t->n_m2l, NN, &m2l_start);
    int64_t *p2p_of = pair_members(t->p2p, t->n_p2p, NN, &p2p_start);
    double *Dall = NULL;
    int rc = ORC_OK;
    if (!M || !Lc || !m || !sx[0] || !sx[1] || !sx[2] || !ax || !ay || !az || !ph || !lvl_cnt ||
        !by_lvl || !m2l_of || !p2p_of) {
        rc = ORC_ENOMEM;
        goto done;
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t slot = t->perm[i];
        int64_t g = active ? active[slot] : slot;
        m[i] = mass_total[g];
        for (int d = 0; d < 3; ++d) sx[d][i] = t->x[d][slot];
    }
    /* cells grouped by level, pre-order inside a level */
    for (int64_t c = 0; c < NN; ++c) lvl_cnt[t->nodes[c].level + 1]++;
    for (int l = 0; l <= ORC_MAXLEVEL; ++l) lvl_cnt[l + 1] += lvl_cnt[l];
    {
        int64_t fill[ORC_MAXLEVEL + 1];
        for (int l = 0; l <= ORC_MAXLEVEL; ++l) fill[l] = lvl_cnt[l];
        for (int64_t c = 0; c < NN; ++c) by_lvl[fill[t->nodes[c].level]++] = c;
    }
    const double e2 = t->prm.kernel == ORC_PLUMMER ? t->prm.eps * t->prm.eps : 0.0;

    /* P2M */
#pragma omp parallel for schedule(dynamic, 8)
    for (int64_t c = 0; c < NN; ++c) {
        const orc_node *nd = &t->nodes[c];
        if (nd->nchild) continue;
        for (int64_t i = nd->begin; i < nd->end; ++i) {
            double u[3] = {sx[0][i] - nd->z[0], sx[1][i] - nd->z[1], sx[2][i] - nd->z[2]};
            for (int k = 0; k < K; ++k) M[c * K + k] += m[i] * mono_over_fact(mi, u, k);
        }
    }
    /* M2M, deepest level first */
    for (int l = ORC_MAXLEVEL; l >= 0; --l) {
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t r = lvl_cnt[l]; r < lvl_cnt[l + 1]; ++r) {
            const int64_t c = by_lvl[r];
            const orc_node *P = &t->nodes[c];
            for (int q = 0; q < P->nchild; ++q) {
                const orc_node *C = &t->nodes[P->child[q]];
                double d[3] = {C->z[0] - P->z[0], C->z[1] - P->z[1], C->z[2] - P->z[2]};
                for (int mm = 0; mm < K; ++mm) {
                    const int *km = mi->k[mm];
                    double acc_m = 0.0;
                    for (int kk = 0; kk < K; ++kk) {
                        const int *kk3 = mi->k[kk];
                        if (kk3[0] > km[0] || kk3[1] > km[1] || kk3[2] > km[2]) continue;
                        int diff = mi->idx[km[0] - kk3[0]][km[1] - kk3[1]][km[2] - kk3[2]];
                        acc_m += M[P->child[q] * K + kk] * mono_over_fact(mi, d, diff);
                    }
                    M[c * K + mm] += acc_m;
                }
            }
        }
    }
    /* M2L: the derivative tensor of every pair (as the pair loop forms it),
     * then gathered per cell */
    Dall = (double *)malloc(sizeof(double) * (size_t)(t->n_m2l * K + 1));
    if (!Dall) {
        rc = ORC_ENOMEM;
        goto done;
    }
#pragma omp parallel for schedule(dynamic, 64)
    for (int64_t q = 0; q < t->n_m2l; ++q) {
        const orc_node *A = &t->nodes[t->m2l[q].a], *B = &t->nodes[t->m2l[q].b];
        double R[3] = {A->z[0] - B->z[0], A->z[1] - B->z[1], A->z[2] - B->z[2]};
        orc_derivs(mi, R, e2, Dall + q * K);
    }
#pragma omp parallel
    {
#pragma omp for schedule(dynamic, 4)
        for (int64_t x = 0; x < NN; ++x) {
            for (int64_t r = m2l_start[x]; r < m2l_start[x + 1]; ++r) {
                const int64_t q = m2l_of[r];
                int64_t ia = t->m2l[q].a, ib = t->m2l[q].b;
                const double *D = Dall + q * K;
                for (int nn = 0; nn < K; ++nn) {
                    int dn = mi_deg(mi, nn);
                    double la = 0.0, lb = 0.0;
                    for (int mm = 0; mm < K; ++mm) {
                        int s = mi_sum_idx(mi, nn, mm);
                        if (s < 0) continue;
                        double sgn_m = (mi_deg(mi, mm) & 1) ? -1.0 : 1.0;
                        if (x == ia)
                            la += sgn_m * M[ib * K + mm] * D[s];
                        else
                            lb += M[ia * K + mm] * D[s];
                    }
                    if (x == ia)
                        Lc[ia * K + nn] += la;
                    else
                        Lc[ib * K + nn] += ((dn & 1) ? -1.0 : 1.0) * lb;
                }
            }
        }
    }
    /* L2L, root level first */
    for (int l = 1; l <= ORC_MAXLEVEL; ++l) {
#pragma omp parallel for schedule(dynamic, 8)
        for (int64_t r = lvl_cnt[l - 1]; r < lvl_cnt[l]; ++r) {
            const int64_t c = by_lvl[r];
            const orc_node *P = &t->nodes[c];
            for (int q = 0; q < P->nchild; ++q) {
                int64_t ic = P->child[q];
                const orc_node *C = &t->nodes[ic];
                double d[3] = {C->z[0] - P->z[0], C->z[1] - P->z[1], C->z[2] - P->z[2]};
                for (int nn = 0; nn < K; ++nn) {
                    const int *kn = mi->k[nn];
                    double acc_n = 0.0;
                    for (int kk = 0; kk < K; ++kk) {
                        const int *k3 = mi->k[kk];
                        if (k3[0] < kn[0] || k3[1] < kn[1] || k3[2] < kn[2]) continue;
                        int diff = mi->idx[k3[0] - kn[0]][k3[1] - kn[1]][k3[2] - kn[2]];
                        acc_n += Lc[c * K + kk] * mono_over_fact(mi, d, diff);
                    }
                    Lc[ic * K + nn] += acc_n;
                }
            }
        }
    }
    /* L2P, then P2P gathered per leaf (pairs in increasing order; in a self
     * pair a particle first takes the terms of the particles before it, as
     * the second member of those pairs, then those of the particles after it) */
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t x = 0; x < NN; ++x) {
        const orc_node *X = &t->nodes[x];
        if (X->nchild) continue;
        for (int64_t i = X->begin; i < X->end; ++i) {
            double u[3] = {sx[0][i] - X->z[0], sx[1][i] - X->z[1], sx[2][i] - X->z[2]};
            double f = 0.0, g[3] = {0.0, 0.0, 0.0};
            for (int k = 0; k < K; ++k) {
                double mono = mono_over_fact(mi, u, k);
                f += mono * Lc[x * K + k];
                const int *kk = mi->k[k];
                if (kk[0] + kk[1] + kk[2] < p) {
                    g[0] += mono * Lc[x * K + mi->idx[kk[0] + 1][kk[1]][kk[2]]];
                    g[1] += mono * Lc[x * K + mi->idx[kk[0]][kk[1] + 1][kk[2]]];
                    g[2] += mono * Lc[x * K + mi->idx[kk[0]][kk[1]][kk[2] + 1]];
                }
            }
            ph[i] += f;
            ax[i] -= g[0];
            ay[i] -= g[1];
            az[i] -= g[2];
        }
        for (int64_t r = p2p_start[x]; r < p2p_start[x + 1]; ++r) {
            const int64_t q = p2p_of[r];
            const orc_node *A = &t->nodes[t->p2p[q].a], *B = &t->nodes[t->p2p[q].b];
            const int self = t->p2p[q].a == t->p2p[q].b;
            const int as_a = t->p2p[q].a == x;
            for (int64_t k = X->begin; k < X->end; ++k) {
                /* k as the second member: i over A (before k in a self pair) */
                if (!as_a || self) {
                    const int64_t iend = self ? k : A->end;
                    for (int64_t i = A->begin; i < iend; ++i) {
                        double dx = sx[0][k] - sx[0][i], dy = sx[1][k] - sx[1][i],
                               dz = sx[2][k] - sx[2][i];
                        double r2 = sqrt(dx * dx + dy * dy + dz * dz);
                        double phi, gg;
                        pair_kernel(t->prm.kernel, t->prm.eps, r2, &phi, &gg);
                        ax[k] -= m[i] * gg * dx;
                        ay[k] -= m[i] * gg * dy;
                        az[k] -= m[i] * gg * dz;
                        ph[k] += m[i] * phi;
                    }
                }
                /* k as the first member: j over B (after k in a self pair) */
                if (as_a) {
                    for (int64_t j = self ? k + 1 : B->begin; j < B->end; ++j) {
                        double dx = sx[0][j] - sx[0][k], dy = sx[1][j] - sx[1][k],
                               dz = sx[2][j] - sx[2][k];
                        double r2 = sqrt(dx * dx + dy * dy + dz * dz);
                        double phi, gg;
                        pair_kernel(t->prm.kernel, t->prm.eps, r2, &phi, &gg);
                        ax[k] += m[j] * gg * dx;
                        ay[k] += m[j] * gg * dy;
                        az[k] += m[j] * gg * dz;
                        ph[k] += m[j] * phi;
                    }
                }
            }
        }
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t slot = t->perm[i];
        acc[slot] = ax[i];
        acc[n + slot] = ay[i];
        acc[2 * n + slot] = az[i];
        pot[slot] = ph[i];
    }
done:
    free(mi); free(M); free(Lc); free(m); free(sx[0]); free(sx[1]); free(sx[2]);
    free(ax); free(ay); free(az); free(ph); free(lvl_cnt); free(by_lvl);
    free(m2l_start); free(m2l_of); free(p2p_start); free(p2p_of); free(Dall);
    return rc;
}

/* Threads used by orc_tree_eval_par (0: leave OpenMP's default). */
int orc_threads(int set)
{
#ifdef _OPENMP
    if (set > 0) omp_set_num_threads(set);
    return omp_get_max_threads();
#else
    (void)set;
    return 1;
#endif
}

/* The FMM result for selected sinks only, computed one sink at a time: the
 * upward pass (P2M, M2M) for every cell, then for each sink the M2L terms of
 * every cell on the path from the root to the sink's leaf (from the symmetric
 * list, each pair taken from the side of the path cell), L2L down that path,
 * L2P, and P2P over its leaf's partners.  By linearity this is the same
 * arithmetic as orc_tree_eval for those sinks, up to summation order.
 * sinks: active slots; outputs acc (SoA 3 x n_sinks), pot (n_sinks), and,
 * when grad is not NULL, the force gradient (SoA 6 x n_sinks: xx, yy, zz,
 * xy, xz, yz; Sec. 4.1) as orc_tree_eval_grad forms it: minus the Hessian of
 * the leaf's local expansion plus -m_j (g I + (dg/dr)/r d d^T) per partner. */
static int eval_sinks(const orc_tree *t, const double *mass_total, const int32_t *active,
                      const int64_t *sinks, int64_t n_sinks, double *acc, double *pot,
                      double *grad)
{
    static const int ca[6] = {0, 1, 2, 0, 0, 1}, cb[6] = {0, 1, 2, 1, 2, 2};
    const int64_t n = t->n, NN = t->n_nodes;
    if (n == 0 || n_sinks == 0) return ORC_OK;
    const int p = t->prm.p;
    orc_mi *mi = (orc_mi *)malloc(sizeof(orc_mi));
    if (!mi) return ORC_ENOMEM;
    mi_init(mi, p);
    const int K = mi->K;
    double *M = (double *)calloc((size_t)(NN * K), sizeof(double));
    double *m = (double *)malloc(sizeof(double) * n);
    int64_t *inv = (int64_t *)malloc(sizeof(int64_t) * n);
    int64_t *parent = (int64_t *)malloc(sizeof(int64_t) * NN);
    int64_t *deg = (int64_t *)calloc((size_t)NN + 1, sizeof(int64_t));
    int64_t *adj = (int64_t *)malloc(sizeof(int64_t) * (2 * t->n_m2l + 1));
    int64_t *pdeg = (int64_t *)calloc((size_t)NN + 1, sizeof(int64_t));
    int64_t *padj = (int64_t *)malloc(sizeof(int64_t) * (2 * t->n_p2p + 1));
    double *D = (double *)malloc(sizeof(double) * K);
    double *Lpath = (double *)malloc(sizeof(double) * K * (ORC_MAXLEVEL + 2));
    if (!M || !m || !inv || !parent || !deg || !adj || !pdeg || !padj || !D || !Lpath) {
        free(mi); free(M); free(m); free(inv); free(parent); free(deg); free(adj);
        free(pdeg); free(padj); free(D); free(Lpath);
        return ORC_ENOMEM;
    }
    for (int64_t i = 0; i < n; ++i) {
        int64_t slot = t->perm[i];
        m[i] = mass_total[active ? active[slot] : slot];
        inv[slot] = i;
    }
    parent[0] = -1;
    for (int64_t c = 0; c < NN; ++c)
        for (int q = 0; q < t->nodes[c].nchild; ++q) parent[t->nodes[c].child[q]] = c;
    /* upward pass, exactly as in orc_tree_eval_ex */
    for (int64_t c = 0; c < NN; ++c) {
        const orc_node *nd = &t->nodes[c];
        if (nd->nchild) continue;
        for (int64_t i = nd->begin; i < nd->end; ++i) {
            int64_t slot = t->perm[i];
            double u[3] = {t->x[0][slot] - nd->z[0], t->x[1][slot] - nd->z[1],
                           t->x[2][slot] - nd->z[2]};
            for (int k = 0; k < K; ++k) M[c * K + k] += m[i] * mono_over_fact(mi, u, k);
        }
    }
    for (int64_t c = NN - 1; c >= 0; --c) {
        const orc_node *P = &t->nodes[c];
        for (int q = 0; q < P->nchild; ++q) {
            const orc_node *C = &t->nodes[P->child[q]];
            double d[3] = {C->z[0] - P->z[0], C->z[1] - P->z[1], C->z[2] - P->z[2]};
            for (int mm = 0; mm < K; ++mm) {
                const int *km = mi->k[mm];
                double acc_m = 0.0;
                for (int kk = 0; kk < K; ++kk) {
                    const int *kk3 = mi->k[kk];
                    if (kk3[0] > km[0] || kk3[1] > km[1] || kk3[2] > km[2]) continue;
                    int diff = mi->idx[km[0] - kk3[0]][km[1] - kk3[1]][km[2] - kk3[2]];
                    acc_m += M[P->child[q] * K + kk] * mono_over_fact(mi, d, diff);
                }
                M[c * K + mm] += acc_m;
            }
        }
    }
    /* partner lists of every cell from the unordered pair lists */
    for (int64_t q = 0; q < t->n_m2l; ++q) { deg[t->m2l[q].a + 1]++; deg[t->m2l[q].b + 1]++; }
    for (int64_t c = 0; c < NN; ++c) deg[c + 1] += deg[c];
    {
        int64_t *fill = (int64_t *)calloc((size_t)NN, sizeof(int64_t));
        for (int64_t q = 0; q < t->n_m2l; ++q) {
            int64_t a = t->m2l[q].a, b = t->m2l[q].b;
            adj[deg[a] + fill[a]++] = b;
            adj[deg[b] + fill[b]++] = a;
        }
        for (int64_t q = 0; q < t->n_p2p; ++q) { pdeg[t->p2p[q].a + 1]++; if (t->p2p[q].a != t->p2p[q].b) pdeg[t->p2p[q].b + 1]++; }
        for (int64_t c = 0; c < NN; ++c) pdeg[c + 1] += pdeg[c];
        memset(fill, 0, sizeof(int64_t) * NN);
        for (int64_t q = 0; q < t->n_p2p; ++q) {
            int64_t a = t->p2p[q].a, b = t->p2p[q].b;
            padj[pdeg[a] + fill[a]++] = b;
            if (a != b) padj[pdeg[b] + fill[b]++] = a;
        }
        free(fill);
    }
    const double e2 = t->prm.kernel == ORC_PLUMMER ? t->prm.eps * t->prm.eps : 0.0;
    for (int64_t s = 0; s < n_sinks; ++s) {
        int64_t i = inv[sinks[s]];
        /* path from the root to the leaf holding sorted position i */
        int64_t path[ORC_MAXLEVEL + 2];
        int np = 0;
        int64_t c = 0;
        path[np++] = 0;
        while (t->nodes[c].nchild) {
            const orc_node *nd = &t->nodes[c];
            int64_t next = -1;
            for (int q = 0; q < nd->nchild; ++q) {
                const orc_node *ch = &t->nodes[nd->child[q]];
                if (i >= ch->begin && i < ch->end) next = nd->child[q];
            }
            c = next;
            path[np++] = c;
        }
        for (int lv = 0; lv < np; ++lv) {
            int64_t A = path[lv];
            const orc_node *NA = &t->nodes[A];
            double *L = Lpath + lv * K;
            for (int k = 0; k < K; ++k) L[k] = 0.0;
            for (int64_t q = deg[A]; q < deg[A + 1]; ++q) {
                int64_t B = adj[q];
                const orc_node *NB = &t->nodes[B];
                double R[3] = {NA->z[0] - NB->z[0], NA->z[1] - NB->z[1], NA->z[2] - NB->z[2]};
                orc_derivs(mi, R, e2, D);
                for (int nn = 0; nn < K; ++nn) {
                    double la = 0.0;
                    for (int mm = 0; mm < K; ++mm) {
                        int sidx = mi_sum_idx(mi, nn, mm);
                        if (sidx < 0) continue;
                        double sgn_m = (mi_deg(mi, mm) & 1) ? -1.0 : 1.0;
                        la += sgn_m * M[B * K + mm] * D[sidx];
                    }
                    L[nn] += la;
                }
            }
            if (lv > 0) {
                const orc_node *P = &t->nodes[path[lv - 1]];
                const double *Lp = Lpath + (lv - 1) * K;
                double d[3] = {NA->z[0] - P->z[0], NA->z[1] - P->z[1], NA->z[2] - P->z[2]};
                for (int nn = 0; nn < K; ++nn) {
                    const int *kn = mi->k[nn];
                    double acc_n = 0.0;
                    for (int kk = 0; kk < K; ++kk) {
                        const int *k3 = mi->k[kk];
                        if (k3[0] < kn[0] || k3[1] < kn[1] || k3[2] < kn[2]) continue;
                        int diff = mi->idx[k3[0] - kn[0]][k3[1] - kn[1]][k3[2] - kn[2]];
                        acc_n += Lp[kk] * mono_over_fact(mi, d, diff);
                    }
                    L[nn] += acc_n;
                }
            }
        }
        const orc_node *leaf = &t->nodes[c];
        const double *L = Lpath + (np - 1) * K;
        int64_t slot = t->perm[i];
        double xi[3] = {t->x[0][slot], t->x[1][slot], t->x[2][slot]};
        double u[3] = {xi[0] - leaf->z[0], xi[1] - leaf->z[1], xi[2] - leaf->z[2]};
        double f = 0.0, g[3] = {0.0, 0.0, 0.0};
        for (int k = 0; k < K; ++k) {
            double mono = mono_over_fact(mi, u, k);
            f += mono * L[k];
            const int *kk = mi->k[k];
            if (kk[0] + kk[1] + kk[2] < p) {
                g[0] += mono * L[mi->idx[kk[0] + 1][kk[1]][kk[2]]];
                g[1] += mono * L[mi->idx[kk[0]][kk[1] + 1][kk[2]]];
                g[2] += mono * L[mi->idx[kk[0]][kk[1]][kk[2] + 1]];
            }
        }
        double ax = -g[0], ay = -g[1], az = -g[2], ph = f;
        double G6[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
        if (grad) { /* minus the Hessian: L[k + e_a + e_b] for |k| <= p - 2 */
            for (int k = 0; k < K; ++k) {
                const int *kk = mi->k[k];
                if (kk[0] + kk[1] + kk[2] > p - 2) continue;
                double mono = mono_over_fact(mi, u, k);
                for (int c6 = 0; c6 < 6; ++c6) {
                    int e[3] = {kk[0], kk[1], kk[2]};
                    e[ca[c6]] += 1;
                    e[cb[c6]] += 1;
                    G6[c6] -= mono * L[mi->idx[e[0]][e[1]][e[2]]];
                }
            }
        }
        for (int64_t q = pdeg[c]; q < pdeg[c + 1]; ++q) {
            const orc_node *B = &t->nodes[padj[q]];
            for (int64_t j = B->begin; j < B->end; ++j) {
                if (j == i) continue;
                int64_t sj = t->perm[j];
                double dx = t->x[0][sj] - xi[0], dy = t->x[1][sj] - xi[1], dz = t->x[2][sj] - xi[2];
                double r = sqrt(dx * dx + dy * dy + dz * dz);
                double phi, gg;
                pair_kernel(t->prm.kernel, t->prm.eps, r, &phi, &gg);
                ax += m[j] * gg * dx;
                ay += m[j] * gg * dy;
                az += m[j] * gg * dz;
                ph += m[j] * phi;
                if (grad) {
                    double h = pair_dg_over_r(t->prm.kernel, t->prm.eps, r);
                    double dv[3] = {dx, dy, dz};
                    for (int c6 = 0; c6 < 6; ++c6)
                        G6[c6] += m[j] * (-h * dv[ca[c6]] * dv[cb[c6]] - (ca[c6] == cb[c6] ? gg : 0.0));
                }
            }
        }
        if (grad)
            for (int c6 = 0; c6 < 6; ++c6) grad[c6 * n_sinks + s] = G6[c6];
        acc[s] = ax;
        acc[n_sinks + s] = ay;
        acc[2 * n_sinks + s] = az;
        pot[s] = ph;
    }
    free(mi); free(M); free(m); free(inv); free(parent); free(deg); free(adj);
    free(pdeg); free(padj); free(D); free(Lpath);
    return ORC_OK;
}

int orc_tree_eval_sinks(const orc_tree *t, const double *mass_total, const int32_t *active,
                        const int64_t *sinks, int64_t n_sinks, double *acc, double *pot)
{
    return eval_sinks(t, mass_total, active, sinks, n_sinks, acc, pot, NULL);
}

int orc_tree_eval_sinks_grad(const orc_tree *t, const double *mass_total, const int32_t *active,
                             const int64_t *sinks, int64_t n_sinks, double *acc, double *pot,
                             double *grad)
{
    if (!grad) return ORC_EINVAL;
    return eval_sinks(t, mass_total, active, sinks, n_sinks, acc, pot, grad);
}

/* One complete FMM force evaluation: acceleration (SoA 3 x n_active) and
 * potential (n_active) of every active particle due to all active masses. */
int orc_fmm(const double *pos, const double *mass, int64_t n_total, const int32_t *active,
            int64_t n_active, const orc_params *prm, double *acc, double *pot)
{
    orc_tree *t = orc_tree_build(pos, n_total, active, n_active, prm);
    if (!t) return ORC_EINVAL;
    int rc = orc_tree_eval(t, mass, n_total, active, acc, pot);
    orc_tree_free(t);
    return rc;
}

/* Number of multi-indices of total degree <= p, as the oracle enumerates them. */
int orc_num_coeffs(int p) { return (p + 1) * (p + 2) * (p + 3) / 6; }
