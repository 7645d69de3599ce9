/*
 * Plain CPU FP64 oracle for screened orbital-space VMC.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library uses this file;
 * only the test-suite, the smoke check and the CPU-baseline leg of the
 * benchmark load it.  It shares no code, header or table with the GPU path.
 *
 * What it computes, each from its plain definition (Sabzevari & Sharma,
 * "Improved speed and scaling in orbital space variational Monte Carlo"):
 *
 *  - psi(N) = C[N] * exp(sum_{p<=q} J_pq n_p n_q) * det(theta[occ(N), 0:Ne])
 *    (section "Correlator product states and Slater determinant"): C[N] is the
 *    product over correlators l of the coefficient c_l[n_l(N)] of the local
 *    Fock state n_l(N) of the correlator's sites (spatial orbitals s_0..s_{k-1},
 *    k <= 5, n_l = sum_m (n_{s_m alpha} + 2 n_{s_m beta}) 4^m); no correlators
 *    means C = 1.  The Jastrow factor is the two-site correlator written on
 *    spin-orbitals (c_11 = e^J).
 *  - E_L[N, eps] = sum over M with |H_NM| above the screening threshold of
 *    H_NM psi(M)/psi(N), with the diagonal M = N always included (Eq. eloc:hci).
 *      singles: kept when S_ia = |h_ia| + sum_j |(ia|jj) - (ij|ja)| > eps
 *               (section "Reduced scaling evaluation of the local energy");
 *      doubles: kept when |<ab|ij> - <ab|ji>| > eps.
 *    Matrix elements are Slater-Condon elements between sorted determinants,
 *    with the fermionic sign obtained by applying the creation/annihilation
 *    operators to the bitstring.
 *  - Ratios psi(M)/psi(N), in two modes:
 *      ORC_DET   : every det(theta[M]) is a fresh LU factorisation;
 *      ORC_LEMMA : one fresh inverse of theta[N] per state, then the ratio of a
 *                  single is R_ai = sum_x theta_ax (theta[N]^-1)_xi and of a double
 *                  the 2x2 minor R_ai R_bj - R_bi R_aj (Eq. R and the text after
 *                  it), with the sign of the permutation that sorts M.
 *    The correlator ratio C[M]/C[N] is the ratio of the two products, each
 *    taken over every correlator, in both modes.  The Jastrow ratio is
 *    recomputed from scratch in ORC_DET; in ORC_LEMMA it is the change of the
 *    quadratic form sum_{p<=q} J_pq n_p n_q written out with the occupation
 *    change D = n(M) - n(N):  D.(J n) + (D.J D)/2 + sum_p J_pp D_p / 2.
 *  - CTMC (section "Continuous time Monte Carlo"): rates r = |psi(M)/psi(N)|
 *    over the same screened set, residence time t = 1/sum r, pick the smallest k
 *    whose running sum exceeds u*T, u from Philox4x64-10.
 *  - Gradient ratios (section "Local energy and Gradient ratios"):
 *    O_{J_pq} = n_p n_q, O_{theta_kx} = (theta[N]^-1)_{x, pos(k)} and
 *    O_{c_l[n]} = [n_l(N) = n] / c_l[n].
 *
 * Canonical candidate order: singles first (occupied i ascending, then a by
 * descending S_ia, ties by a), then doubles (occupied pairs i<j ascending
 * lexicographically, then a<b by descending |v|, ties by (a, b)).
 *
 * Conventions: spatial orbitals 0..n-1; spin-orbitals alpha 0..n-1, beta
 * n..2n-1; chemist-notation integrals (pq|rs) given as a canonical list.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_DET 0
#define ORC_LEMMA 1

typedef struct {
    int32_t type; /* 1 single, 2 double */
    int32_t i, j, a, b; /* j = b = -1 for singles */
    double h;          /* H_NM between sorted determinants */
    double ratio;      /* psi(M)/psi(N), sorted-determinant convention */
} orc_cand;

typedef struct {
    int32_t a, b;
    double v;
} orc_dentry;

typedef struct {
    int n, n_so, na, nb, ne, nw;
    double eps;
    double* h1;      /* n*n spatial */
    double* eri;     /* dense array over canonical compound indices */
    double* P;       /* build-time only: P[I][J][A][B] = (AI|BJ) */
    int64_t n_quad;
    double* S;       /* n_so*n_so singles bound S[i*n_so+a] */
    /* per spin-orbital pair (i<j): entries (a<b, v) with |v| > eps */
    int64_t* d_off;  /* n_so*n_so + 1 offsets, indexed i*n_so+j */
    orc_dentry* d_ent;
    double* J;       /* n_so*n_so symmetric */
    double* theta;   /* n_so*n_so row-major */
    /* correlator product state: n_corr correlators of ck[l] <= 5 sites
     * csite[5 l + m] (spatial orbitals), coefficients cc[coff[l] + n] */
    int n_corr;
    int* ck;
    int* csite;
    int64_t* coff;
    double* cc;
} orc_sys;

/* ---------------------------------------------------------------- indices */
static int64_t pair_idx(int64_t p, int64_t q) {
    int64_t hi = p > q ? p : q, lo = p > q ? q : p;
    return hi * (hi + 1) / 2 + lo;
}
static int64_t quad_idx(int p, int q, int r, int s) {
    int64_t a = pair_idx(p, q), b = pair_idx(r, s);
    int64_t hi = a > b ? a : b, lo = a > b ? b : a;
    return hi * (hi + 1) / 2 + lo;
}
static int spin_of(const orc_sys* s, int p) { return p >= s->n; }
static int spat(const orc_sys* s, int p) { return p % s->n; }

/* spatial chemist integral (PQ|RS) */
static double eri_sp(const orc_sys* s, int P, int Q, int R, int S) {
    return s->eri[quad_idx(P, Q, R, S)];
}
/* spin-orbital chemist integral (pq|rs) */
static double eri_so(const orc_sys* s, int p, int q, int r, int t) {
    if (spin_of(s, p) != spin_of(s, q) || spin_of(s, r) != spin_of(s, t)) return 0.0;
    return eri_sp(s, spat(s, p), spat(s, q), spat(s, r), spat(s, t));
}
static double h_so(const orc_sys* s, int p, int q) {
    if (spin_of(s, p) != spin_of(s, q)) return 0.0;
    return s->h1[spat(s, p) * s->n + spat(s, q)];
}

/* (ai|bj) over spin-orbitals through the dense copy P[I][J][A][B] = (AI|BJ) */
static double p_so(const orc_sys* s, int a, int i, int b, int j) {
    if (spin_of(s, a) != spin_of(s, i) || spin_of(s, b) != spin_of(s, j)) return 0.0;
    int n = s->n;
    return s->P[(((size_t)spat(s, i) * n + spat(s, j)) * n + spat(s, a)) * n + spat(s, b)];
}
/* antisymmetrised double element <ab||ij> = (ai|bj) - (aj|bi) */
static double v_double(const orc_sys* s, int i, int j, int a, int b) {
    return p_so(s, a, i, b, j) - p_so(s, a, j, b, i);
}

/* --------------------------------------------------------------- bitstrings */
static int occ_test(const uint64_t* w, int p) { return (int)((w[p >> 6] >> (p & 63)) & 1u); }
static void occ_set(uint64_t* w, int p) { w[p >> 6] |= (uint64_t)1 << (p & 63); }
static void occ_clr(uint64_t* w, int p) { w[p >> 6] &= ~((uint64_t)1 << (p & 63)); }
static int occ_below(const uint64_t* w, int p) { /* number of occupied orbitals < p */
    int c = 0;
    for (int k = 0; k < p; ++k) c += occ_test(w, k);
    return c;
}
static int occ_list(const orc_sys* s, const uint64_t* w, int* out) {
    int c = 0;
    for (int p = 0; p < s->n_so; ++p)
        if (occ_test(w, p)) out[c++] = p;
    return c;
}

/* apply annihilator a_p: returns sign, clears bit; 0 if empty */
static int apply_annihilate(uint64_t* w, int p) {
    if (!occ_test(w, p)) return 0;
    int sg = (occ_below(w, p) & 1) ? -1 : 1;
    occ_clr(w, p);
    return sg;
}
/* apply creator a_p^dagger: returns sign, sets bit; 0 if occupied */
static int apply_create(uint64_t* w, int p) {
    if (occ_test(w, p)) return 0;
    int sg = (occ_below(w, p) & 1) ? -1 : 1;
    occ_set(w, p);
    return sg;
}

/* ------------------------------------------------------------ dense algebra */
/* LU with partial pivoting, in place (row-major m x m). Returns log|det| and
 * writes the sign; sign 0 means singular. perm receives the row permutation. */
static double lu_factor(double* A, int m, int* perm, int* sign) {
    int sg = 1;
    double logabs = 0.0;
    for (int k = 0; k < m; ++k) perm[k] = k;
    for (int k = 0; k < m; ++k) {
        int piv = k;
        double best = fabs(A[k * m + k]);
        for (int r = k + 1; r < m; ++r)
            if (fabs(A[r * m + k]) > best) { best = fabs(A[r * m + k]); piv = r; }
        if (best == 0.0) { *sign = 0; return -INFINITY; }
        if (piv != k) {
            for (int c = 0; c < m; ++c) { double t = A[k * m + c]; A[k * m + c] = A[piv * m + c]; A[piv * m + c] = t; }
            int t = perm[k]; perm[k] = perm[piv]; perm[piv] = t;
            sg = -sg;
        }
        double d = A[k * m + k];
        if (d < 0) sg = -sg;
        logabs += log(fabs(d));
        for (int r = k + 1; r < m; ++r) {
            double f = A[r * m + k] / d;
            A[r * m + k] = f;
            for (int c = k + 1; c < m; ++c) A[r * m + c] -= f * A[k * m + c];
        }
    }
    *sign = sg;
    return logabs;
}

/* inverse from an LU factorisation: Ainv (row-major) with A*Ainv = I */
static void lu_inverse(const double* LU, const int* perm, int m, double* Ainv, double* col) {
    for (int e = 0; e < m; ++e) {
        /* solve A x = e_e: P A = L U, so L U x = P e_e */
        for (int r = 0; r < m; ++r) col[r] = (perm[r] == e) ? 1.0 : 0.0;
        for (int r = 0; r < m; ++r) {
            double acc = col[r];
            for (int c = 0; c < r; ++c) acc -= LU[r * m + c] * col[c];
            col[r] = acc;
        }
        for (int r = m - 1; r >= 0; --r) {
            double acc = col[r];
            for (int c = r + 1; c < m; ++c) acc -= LU[r * m + c] * col[c];
            col[r] = acc / LU[r * m + r];
        }
        for (int r = 0; r < m; ++r) Ainv[r * m + e] = col[r];
    }
}

/* log|det theta[rows, 0:ne]| and its sign, rows in the given order */
static double slater_logdet(const orc_sys* s, const int* rows, int* sign, double* work, int* perm) {
    int m = s->ne;
    for (int r = 0; r < m; ++r)
        for (int c = 0; c < m; ++c) work[r * m + c] = s->theta[rows[r] * s->n_so + c];
    return lu_factor(work, m, perm, sign);
}

/* Jastrow exponent sum_{p<=q} J_pq n_p n_q for a sorted occupied list */
static double log_jastrow(const orc_sys* s, const int* occ, int m) {
    double acc = 0.0;
    for (int x = 0; x < m; ++x)
        for (int y = x; y < m; ++y) acc += s->J[occ[x] * s->n_so + occ[y]];
    return acc;
}

/* local Fock state of correlator l in the determinant occ_bits */
static int64_t cps_state(const orc_sys* s, int l, const uint64_t* occ_bits) {
    int64_t idx = 0, w = 1;
    for (int m = 0; m < s->ck[l]; ++m) {
        int site = s->csite[5 * l + m];
        idx += w * (occ_test(occ_bits, site) + 2 * occ_test(occ_bits, s->n + site));
        w *= 4;
    }
    return idx;
}

/* log|C[N]| over every correlator; *sign receives the sign (0 if a
 * coefficient is zero) */
static double log_cps(const orc_sys* s, const uint64_t* occ_bits, int* sign) {
    double acc = 0.0;
    int sg = 1;
    for (int l = 0; l < s->n_corr; ++l) {
        double c = s->cc[s->coff[l] + cps_state(s, l, occ_bits)];
        if (c == 0.0) { *sign = 0; return -INFINITY; }
        if (c < 0.0) sg = -sg;
        acc += log(fabs(c));
    }
    *sign = sg;
    return acc;
}

/* ------------------------------------------------------------------ create */
orc_sys* orc_create(int n, int na, int nb, const double* h1, int64_t n_eri, const int32_t* eri_idx,
                    const double* eri_val, double eps) {
    orc_sys* s = (orc_sys*)calloc(1, sizeof(orc_sys));
    s->n = n; s->n_so = 2 * n; s->na = na; s->nb = nb; s->ne = na + nb;
    s->nw = (s->n_so + 63) / 64;
    s->eps = eps;
    s->h1 = (double*)malloc(sizeof(double) * n * n);
    memcpy(s->h1, h1, sizeof(double) * n * n);
    int64_t npair = (int64_t)n * (n + 1) / 2;
    s->n_quad = npair * (npair + 1) / 2;
    s->eri = (double*)calloc((size_t)s->n_quad, sizeof(double));
    for (int64_t k = 0; k < n_eri; ++k) {
        const int32_t* q = eri_idx + 4 * k;
        s->eri[quad_idx(q[0], q[1], q[2], q[3])] = eri_val[k];
    }
    int nso = s->n_so;
    /* singles bound S_ia, sum over all spin-orbitals j in ascending order */
    s->S = (double*)calloc((size_t)nso * nso, sizeof(double));
    for (int i = 0; i < nso; ++i)
        for (int a = 0; a < nso; ++a) {
            if (a == i || spin_of(s, a) != spin_of(s, i)) continue;
            double acc = fabs(h_so(s, i, a));
            for (int j = 0; j < nso; ++j) {
                double c = eri_so(s, i, a, j, j);
                double x = eri_so(s, i, j, j, a);
                acc += fabs(c - x);
            }
            s->S[i * nso + a] = acc;
        }
    /* doubles: for every spin-orbital pair i<j, all a<b (disjoint from i,j)
     * with |v| > eps.  Walker independent, so built once.  The loop reads the
     * integrals through a dense copy P[I][J][A][B] = (AI|BJ) (same values as
     * the canonical store, laid out so the inner loops over a, b are
     * contiguous); it is freed after the build. */
    {
        size_t n4 = (size_t)n * n * n * n;
        s->P = (double*)malloc(sizeof(double) * n4);
        for (int I = 0; I < n; ++I)
            for (int J = 0; J < n; ++J)
                for (int A = 0; A < n; ++A)
                    for (int B = 0; B < n; ++B)
                        s->P[(((size_t)I * n + J) * n + A) * n + B] = eri_sp(s, A, I, B, J);
    }
    s->d_off = (int64_t*)calloc((size_t)nso * nso + 1, sizeof(int64_t));
    int64_t* cnt = (int64_t*)calloc((size_t)nso * nso, sizeof(int64_t));
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < nso; ++i)
        for (int j = i + 1; j < nso; ++j) {
            int64_t c = 0;
            for (int a = 0; a < nso; ++a) {
                if (a == i || a == j) continue;
                for (int b = a + 1; b < nso; ++b) {
                    if (b == i || b == j) continue;
                    if (spin_of(s, a) + spin_of(s, b) != spin_of(s, i) + spin_of(s, j)) continue;
                    if (fabs(v_double(s, i, j, a, b)) > eps) ++c;
                }
            }
            cnt[i * nso + j] = c;
        }
    for (int64_t k = 0; k < (int64_t)nso * nso; ++k) s->d_off[k + 1] = s->d_off[k] + cnt[k];
    s->d_ent = (orc_dentry*)malloc(sizeof(orc_dentry) * (size_t)(s->d_off[(int64_t)nso * nso] + 1));
#pragma omp parallel for schedule(dynamic)
    for (int i = 0; i < nso; ++i)
        for (int j = i + 1; j < nso; ++j) {
            int64_t o = s->d_off[i * nso + j];
            for (int a = 0; a < nso; ++a) {
                if (a == i || a == j) continue;
                for (int b = a + 1; b < nso; ++b) {
                    if (b == i || b == j) continue;
                    if (spin_of(s, a) + spin_of(s, b) != spin_of(s, i) + spin_of(s, j)) continue;
                    double v = v_double(s, i, j, a, b);
                    if (fabs(v) > eps) { s->d_ent[o].a = a; s->d_ent[o].b = b; s->d_ent[o].v = v; ++o; }
                }
            }
        }
    free(cnt);
    free(s->P);
    s->P = NULL;
    s->J = (double*)calloc((size_t)nso * nso, sizeof(double));
    s->theta = (double*)calloc((size_t)nso * nso, sizeof(double));
    return s;
}

void orc_destroy(orc_sys* s) {
    if (!s) return;
    free(s->h1); free(s->eri); free(s->S); free(s->d_off); free(s->d_ent); free(s->J); free(s->theta);
    free(s->ck); free(s->csite); free(s->coff); free(s->cc);
    free(s);
}

int64_t orc_num_double_entries(const orc_sys* s) { return s->d_off[(int64_t)s->n_so * s->n_so]; }

/* J packed upper triangle (p<=q row by row), theta n_so x n_so row-major */
void orc_set_params(orc_sys* s, const double* J_packed, const double* theta) {
    int nso = s->n_so;
    int64_t k = 0;
    for (int p = 0; p < nso; ++p)
        for (int q = p; q < nso; ++q) {
            s->J[p * nso + q] = J_packed[k];
            s->J[q * nso + p] = J_packed[k];
            ++k;
        }
    memcpy(s->theta, theta, sizeof(double) * nso * nso);
}

/* Correlators: n_corr of them, correlator l on the sites[5 l + m] (m < k,
 * k = number of entries >= 0 before the first -1, at most 5, distinct spatial
 * orbitals), with 4^k coefficients each, concatenated in coeffs.  n_corr = 0
 * removes the correlator factor.  Returns the number of coefficients, or -1
 * on a malformed site list. */
int64_t orc_set_cps(orc_sys* s, int n_corr, const int32_t* sites, const double* coeffs) {
    free(s->ck); free(s->csite); free(s->coff); free(s->cc);
    s->ck = NULL; s->csite = NULL; s->coff = NULL; s->cc = NULL;
    s->n_corr = 0;
    if (n_corr <= 0) return 0;
    s->ck = (int*)calloc((size_t)n_corr, sizeof(int));
    s->csite = (int*)malloc(sizeof(int) * 5 * (size_t)n_corr);
    s->coff = (int64_t*)calloc((size_t)n_corr + 1, sizeof(int64_t));
    for (int l = 0; l < n_corr; ++l) {
        int k = 0;
        while (k < 5 && sites[5 * l + k] >= 0) ++k;
        if (k == 0) return -1;
        for (int m = 0; m < 5; ++m) s->csite[5 * l + m] = (m < k) ? sites[5 * l + m] : -1;
        for (int m = 0; m < k; ++m) {
            if (sites[5 * l + m] >= s->n) return -1;
            for (int m2 = 0; m2 < m; ++m2)
                if (sites[5 * l + m2] == sites[5 * l + m]) return -1;
        }
        s->ck[l] = k;
        s->coff[l + 1] = s->coff[l] + ((int64_t)1 << (2 * k));
    }
    s->cc = (double*)malloc(sizeof(double) * (size_t)s->coff[n_corr]);
    memcpy(s->cc, coeffs, sizeof(double) * (size_t)s->coff[n_corr]);
    s->n_corr = n_corr;
    return s->coff[n_corr];
}

int64_t orc_num_cps_params(const orc_sys* s) { return s->n_corr ? s->coff[s->n_corr] : 0; }

/* singles bound table, for inspection: out[n_so*n_so] */
void orc_singles_bound(const orc_sys* s, double* out) {
    memcpy(out, s->S, sizeof(double) * s->n_so * s->n_so);
}

/* doubles of pair (i<j) with |v| > eps, sorted by (-|v|, a, b); returns count */
static int cmp_dentry(const void* x, const void* y) {
    const orc_dentry* u = (const orc_dentry*)x;
    const orc_dentry* w = (const orc_dentry*)y;
    double au = fabs(u->v), aw = fabs(w->v);
    if (au > aw) return -1;
    if (au < aw) return 1;
    if (u->a != w->a) return u->a < w->a ? -1 : 1;
    if (u->b != w->b) return u->b < w->b ? -1 : 1;
    return 0;
}
int64_t orc_pair_doubles(const orc_sys* s, int i, int j, int32_t* ab_out, double* v_out, int64_t cap) {
    int64_t o = s->d_off[i * s->n_so + j], e = s->d_off[i * s->n_so + j + 1];
    int64_t m = e - o;
    orc_dentry* tmp = (orc_dentry*)malloc(sizeof(orc_dentry) * (size_t)(m + 1));
    memcpy(tmp, s->d_ent + o, sizeof(orc_dentry) * (size_t)m);
    qsort(tmp, (size_t)m, sizeof(orc_dentry), cmp_dentry);
    for (int64_t k = 0; k < m && k < cap; ++k) {
        ab_out[2 * k] = tmp[k].a; ab_out[2 * k + 1] = tmp[k].b; v_out[k] = tmp[k].v;
    }
    free(tmp);
    return m;
}

/* ----------------------------------------------------------------- diagonal */
static double h_diag(const orc_sys* s, const int* occ, int m) {
    double acc = 0.0;
    for (int x = 0; x < m; ++x) acc += h_so(s, occ[x], occ[x]);
    for (int x = 0; x < m; ++x)
        for (int y = x + 1; y < m; ++y) {
            int i = occ[x], j = occ[y];
            acc += eri_so(s, i, i, j, j) - eri_so(s, i, j, j, i);
        }
    return acc;
}

double orc_hdiag(const orc_sys* s, const uint64_t* occ_bits) {
    int* occ = (int*)malloc(sizeof(int) * s->n_so);
    int m = occ_list(s, occ_bits, occ);
    double r = h_diag(s, occ, m);
    free(occ);
    return r;
}

/* log|psi| and sign for one determinant */
double orc_log_psi(const orc_sys* s, const uint64_t* occ_bits, int* sign_out) {
    int* occ = (int*)malloc(sizeof(int) * s->n_so);
    int m = occ_list(s, occ_bits, occ);
    double* work = (double*)malloc(sizeof(double) * s->ne * s->ne);
    int* perm = (int*)malloc(sizeof(int) * s->ne);
    int sg = 0;
    double ld = (m == s->ne) ? slater_logdet(s, occ, &sg, work, perm) : -INFINITY;
    double lj = log_jastrow(s, occ, m);
    int sc = 1;
    double lc = log_cps(s, occ_bits, &sc);
    free(occ); free(work); free(perm);
    *sign_out = sg * sc;
    return ld + lj + lc;
}

/* ----------------------------------------------------------- local energy */
typedef struct {
    int a;
    double S;
} orc_sentry;
static int cmp_sentry(const void* x, const void* y) {
    const orc_sentry* u = (const orc_sentry*)x;
    const orc_sentry* w = (const orc_sentry*)y;
    if (u->S > w->S) return -1;
    if (u->S < w->S) return 1;
    return (u->a < w->a) ? -1 : (u->a > w->a);
}

typedef struct {
    /* scratch for one walker */
    int* occ;
    int* occ_m;
    int* iwork;     /* 2 ne ints for the parity count */
    double* work;
    double* work2;
    int* perm;
    double* Binv;   /* ne x ne inverse of theta[N] (lemma mode) */
    double* R;      /* n_so x ne */
    double* v;      /* n_so: (J n)_p = sum_{q occupied} J_pq (lemma mode) */
    orc_sentry* sl;
    orc_dentry* dl;
    orc_cand* cand; /* candidates of the last evaluation, when stored */
    int64_t cand_cap;
} orc_ws;

static orc_ws* ws_alloc(const orc_sys* s) {
    orc_ws* w = (orc_ws*)calloc(1, sizeof(orc_ws));
    int ne = s->ne, nso = s->n_so;
    w->occ = (int*)malloc(sizeof(int) * nso);
    w->occ_m = (int*)malloc(sizeof(int) * nso);
    w->iwork = (int*)malloc(sizeof(int) * 2 * ne + 8);
    w->work = (double*)malloc(sizeof(double) * ne * ne + 8);
    w->work2 = (double*)malloc(sizeof(double) * ne + 8);
    w->perm = (int*)malloc(sizeof(int) * ne + 8);
    w->Binv = (double*)malloc(sizeof(double) * ne * ne + 8);
    w->R = (double*)malloc(sizeof(double) * nso * ne + 8);
    w->v = (double*)malloc(sizeof(double) * nso + 8);
    w->sl = (orc_sentry*)malloc(sizeof(orc_sentry) * nso + 8);
    int64_t maxrow = 0;
    for (int64_t k = 0; k < (int64_t)nso * nso; ++k) {
        int64_t l = s->d_off[k + 1] - s->d_off[k];
        if (l > maxrow) maxrow = l;
    }
    w->dl = (orc_dentry*)malloc(sizeof(orc_dentry) * (size_t)(maxrow + 1));
    return w;
}
static void ws_free(orc_ws* w) {
    free(w->occ); free(w->occ_m); free(w->iwork); free(w->work); free(w->work2); free(w->perm); free(w->Binv);
    free(w->R); free(w->v); free(w->sl); free(w->dl); free(w->cand); free(w);
}

/* number of inversions of a[0..m-1] (pairs x < y with a[x] > a[y]), counted
 * while merge-sorting it in place; tmp holds m ints */
static int64_t count_inversions(int* a, int* tmp, int m) {
    if (m < 2) return 0;
    int h = m / 2;
    int64_t inv = count_inversions(a, tmp, h) + count_inversions(a + h, tmp, m - h);
    int x = 0, y = h, k = 0;
    while (x < h && y < m) {
        if (a[y] < a[x]) { inv += h - x; tmp[k++] = a[y++]; }
        else tmp[k++] = a[x++];
    }
    while (x < h) tmp[k++] = a[x++];
    while (y < m) tmp[k++] = a[y++];
    memcpy(a, tmp, sizeof(int) * (size_t)m);
    return inv;
}

/* parity (+1/-1) of the permutation that sorts rows[0..m-1] ascending: the
 * parity of its inversion count; work holds 2m ints */
static int sort_parity(const int* rows, int m, int* work) {
    memcpy(work, rows, sizeof(int) * (size_t)m);
    return (count_inversions(work, work + m, m) & 1) ? -1 : 1;
}

static void store_cand(orc_ws* w, int64_t k, int type, int i, int j, int a, int b, double h, double ratio) {
    if (k >= w->cand_cap) {
        int64_t cap = w->cand_cap ? 2 * w->cand_cap : 4096;
        while (cap <= k) cap *= 2;
        w->cand = (orc_cand*)realloc(w->cand, sizeof(orc_cand) * (size_t)cap);
        w->cand_cap = cap;
    }
    orc_cand* c = w->cand + k;
    c->type = type; c->i = i; c->j = j; c->a = a; c->b = b; c->h = h; c->ratio = ratio;
}

/* psi(M)/psi(N) from scratch: M given by its unsorted row list (N's list with
 * replaced entries) and its occupation bits; sorted-determinant convention. */
static double ratio_det(const orc_sys* s, orc_ws* w, const int* occ_m_unsorted, const uint64_t* bits_m,
                        double logN, int signN) {
    int m = s->ne;
    int* sorted = w->occ_m;
    memcpy(sorted, occ_m_unsorted, sizeof(int) * m);
    /* insertion sort */
    for (int x = 1; x < m; ++x) {
        int v = sorted[x], y = x - 1;
        while (y >= 0 && sorted[y] > v) { sorted[y + 1] = sorted[y]; --y; }
        sorted[y + 1] = v;
    }
    int sg, sc;
    double ld = slater_logdet(s, sorted, &sg, w->work, w->perm);
    if (sg == 0) return 0.0;
    double lc = log_cps(s, bits_m, &sc);
    if (sc == 0) return 0.0;
    double lj = log_jastrow(s, sorted, m);
    return (double)(sg * sc * signN) * exp(ld + lj + lc - logN);
}

/* Change of the Jastrow exponent sum_{p<=q} J_pq n_p n_q when the occupation
 * changes by D (entries d[k] = +-1 at orbitals o[k], k < nd): with n the
 * occupation of N and v = J n, the quadratic form changes by
 * D.v + (D.J D)/2 + sum_p J_pp D_p / 2 (symmetric J, n_p^2 = n_p). */
static double jastrow_change(const orc_sys* s, const double* v, const int* o, const int* d, int nd) {
    int nso = s->n_so;
    double lin = 0.0, quad = 0.0, diag = 0.0;
    for (int k = 0; k < nd; ++k) {
        lin += d[k] * v[o[k]];
        diag += d[k] * s->J[o[k] * nso + o[k]];
        for (int l = 0; l < nd; ++l) quad += d[k] * d[l] * s->J[o[k] * nso + o[l]];
    }
    return lin + 0.5 * quad + 0.5 * diag;
}

/*
 * Local energy of one walker.  Writes E_L, T = sum of rates and the number of
 * candidates; with `store` the candidates are kept in w->cand in canonical
 * order.  Returns 0 on success, -1 if psi(N) = 0, -2 for a wrong electron count.
 */
static int eloc_one(const orc_sys* s, orc_ws* w, const uint64_t* occ_bits, int mode, double* eloc_out,
                    double* T_out, int64_t* ncand_out, int store, double* hnn_out) {
    int nso = s->n_so, ne = s->ne;
    int m = occ_list(s, occ_bits, w->occ);
    if (m != ne) return -2;
    int* occ = w->occ;
    int signN, signC;
    double logdetN = slater_logdet(s, occ, &signN, w->work, w->perm);
    if (signN == 0) return -1;
    double logcN = log_cps(s, occ_bits, &signC);
    if (signC == 0) return -1;
    double logjN = log_jastrow(s, occ, ne);
    double logN = logdetN + logjN + logcN;
    if (mode == ORC_LEMMA) {
        /* fresh inverse of theta[N] and R = theta[:, 0:ne] theta[N]^-1 */
        for (int r = 0; r < ne; ++r)
            for (int c = 0; c < ne; ++c) w->work[r * ne + c] = s->theta[occ[r] * nso + c];
        int sg;
        lu_factor(w->work, ne, w->perm, &sg);
        lu_inverse(w->work, w->perm, ne, w->Binv, w->work2);
        for (int a = 0; a < nso; ++a)
            for (int p = 0; p < ne; ++p) {
                double acc = 0.0;
                for (int x = 0; x < ne; ++x) acc += s->theta[a * nso + x] * w->Binv[x * ne + p];
                w->R[a * ne + p] = acc;
            }
        /* v = J n(N) for the Jastrow change */
        for (int p = 0; p < nso; ++p) {
            double acc = 0.0;
            for (int y = 0; y < ne; ++y) acc += s->J[p * nso + occ[y]];
            w->v[p] = acc;
        }
    }
    double hnn = h_diag(s, occ, ne);
    double el = hnn, T = 0.0;
    int64_t nc = 0;
    uint64_t bits[16];
    int* rows = (int*)malloc(sizeof(int) * ne);

    /* singles */
    for (int x = 0; x < ne; ++x) {
        int i = occ[x];
        int ns = 0;
        for (int a = 0; a < nso; ++a) {
            if (occ_test(occ_bits, a) || spin_of(s, a) != spin_of(s, i)) continue;
            if (s->S[i * nso + a] > s->eps) { w->sl[ns].a = a; w->sl[ns].S = s->S[i * nso + a]; ++ns; }
        }
        qsort(w->sl, (size_t)ns, sizeof(orc_sentry), cmp_sentry);
        for (int k = 0; k < ns; ++k) {
            int a = w->sl[k].a;
            /* sign of a_a^dagger a_i applied to |N>; bits becomes M */
            memcpy(bits, occ_bits, sizeof(uint64_t) * s->nw);
            int g = apply_annihilate(bits, i);
            g *= apply_create(bits, a);
            double hel = h_so(s, i, a);
            for (int y = 0; y < ne; ++y) {
                int j = occ[y];
                if (j == i) continue;
                hel += eri_so(s, a, i, j, j) - eri_so(s, a, j, j, i);
            }
            hel *= (double)g;
            double ratio;
            memcpy(rows, occ, sizeof(int) * ne);
            rows[x] = a;
            if (mode == ORC_DET) {
                ratio = ratio_det(s, w, rows, bits, logN, signN * signC);
            } else {
                double detr = w->R[a * ne + x] * (double)sort_parity(rows, ne, w->iwork);
                int o[2] = {a, i}, d[2] = {1, -1};
                int sc;
                double lc = log_cps(s, bits, &sc);
                double cr = (sc == 0) ? 0.0 : (double)(sc * signC) * exp(lc - logcN);
                ratio = detr * cr * exp(jastrow_change(s, w->v, o, d, 2));
            }
            el += hel * ratio;
            T += fabs(ratio);
            if (store) store_cand(w, nc, 1, i, -1, a, -1, hel, ratio);
            ++nc;
        }
    }
    /* doubles */
    for (int x = 0; x < ne; ++x)
        for (int y = x + 1; y < ne; ++y) {
            int i = occ[x], j = occ[y];
            int64_t o0 = s->d_off[i * nso + j], e = s->d_off[i * nso + j + 1];
            int nd = 0;
            for (int64_t k = o0; k < e; ++k) {
                const orc_dentry* dd = s->d_ent + k;
                if (occ_test(occ_bits, dd->a) || occ_test(occ_bits, dd->b)) continue;
                w->dl[nd++] = *dd;
            }
            qsort(w->dl, (size_t)nd, sizeof(orc_dentry), cmp_dentry);
            for (int k = 0; k < nd; ++k) {
                int a = w->dl[k].a, b = w->dl[k].b;
                memcpy(bits, occ_bits, sizeof(uint64_t) * s->nw);
                int g = apply_annihilate(bits, i);
                g *= apply_annihilate(bits, j);
                g *= apply_create(bits, b);
                g *= apply_create(bits, a);
                /* |M> = g * a_a^+ a_b^+ a_j a_i |N> sorted; <M|H|N> = g <ab||ij> */
                double hel = (double)g * w->dl[k].v;
                double ratio;
                memcpy(rows, occ, sizeof(int) * ne);
                rows[x] = a;
                rows[y] = b;
                if (mode == ORC_DET) {
                    ratio = ratio_det(s, w, rows, bits, logN, signN * signC);
                } else {
                    double minor = w->R[a * ne + x] * w->R[b * ne + y] - w->R[b * ne + x] * w->R[a * ne + y];
                    double detr = minor * (double)sort_parity(rows, ne, w->iwork);
                    int o[4] = {a, b, i, j}, d[4] = {1, 1, -1, -1};
                    int sc;
                    double lc = log_cps(s, bits, &sc);
                    double cr = (sc == 0) ? 0.0 : (double)(sc * signC) * exp(lc - logcN);
                    ratio = detr * cr * exp(jastrow_change(s, w->v, o, d, 4));
                }
                el += hel * ratio;
                T += fabs(ratio);
                if (store) store_cand(w, nc, 2, i, j, a, b, hel, ratio);
                ++nc;
            }
        }
    free(rows);
    *eloc_out = el;
    *T_out = T;
    *ncand_out = nc;
    if (hnn_out) *hnn_out = hnn;
    return 0;
}

int orc_local_energy(const orc_sys* s, const uint64_t* occ_bits, int mode, double* eloc, double* T,
                     int64_t* ncand, orc_cand* cand, int64_t cap, double* hnn) {
    orc_ws* w = ws_alloc(s);
    int rc = eloc_one(s, w, occ_bits, mode, eloc, T, ncand, cand != NULL, hnn);
    if (rc == 0 && cand)
        for (int64_t k = 0; k < *ncand && k < cap; ++k) cand[k] = w->cand[k];
    ws_free(w);
    return rc;
}

/* batch over walkers (OpenMP over walkers); status[w] = return code */
void orc_local_energy_batch(const orc_sys* s, int64_t nwalk, const uint64_t* occ_bits, int mode,
                            double* eloc, double* T, int64_t* ncand, int32_t* status, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        orc_ws* w = ws_alloc(s);
#pragma omp for schedule(dynamic)
        for (int64_t k = 0; k < nwalk; ++k) {
            int64_t nc = 0;
            status[k] = eloc_one(s, w, occ_bits + k * s->nw, mode, eloc + k, T + k, &nc, 0, NULL);
            ncand[k] = nc;
        }
        ws_free(w);
    }
}

int orc_max_threads(void) {
#ifdef _OPENMP
    return omp_get_max_threads();
#else
    return 1;
#endif
}

/* ------------------------------------------------------------------ Philox */
/* Philox4x64-10 block function (Salmon, Moraes, Dror, Shaw, SC'11). */
void orc_philox4x64_10(const uint64_t ctr_in[4], const uint64_t key_in[2], uint64_t out[4]) {
    const uint64_t M0 = 0xD2E7470EE14C6C93ULL, M1 = 0xCA5A826395121157ULL;
    const uint64_t W0 = 0x9E3779B97F4A7C15ULL, W1 = 0xBB67AE8584CAA73BULL;
    uint64_t c0 = ctr_in[0], c1 = ctr_in[1], c2 = ctr_in[2], c3 = ctr_in[3];
    uint64_t k0 = key_in[0], k1 = key_in[1];
    for (int r = 0; r < 10; ++r) {
        unsigned __int128 p0 = (unsigned __int128)M0 * c0;
        unsigned __int128 p1 = (unsigned __int128)M1 * c2;
        uint64_t hi0 = (uint64_t)(p0 >> 64), lo0 = (uint64_t)p0;
        uint64_t hi1 = (uint64_t)(p1 >> 64), lo1 = (uint64_t)p1;
        uint64_t n0 = hi1 ^ c1 ^ k0, n1 = lo1, n2 = hi0 ^ c3 ^ k1, n3 = lo0;
        c0 = n0; c1 = n1; c2 = n2; c3 = n3;
        k0 += W0; k1 += W1;
    }
    out[0] = c0; out[1] = c1; out[2] = c2; out[3] = c3;
}

/* u in [0,1): 53 high bits of word 0 of Philox(ctr=(step,0,0,0), key=(seed, walker)) */
double orc_uniform(uint64_t seed, uint64_t walker, uint64_t step) {
    uint64_t ctr[4] = {step, 0, 0, 0}, key[2] = {seed, walker}, out[4];
    orc_philox4x64_10(ctr, key, out);
    return (double)(out[0] >> 11) * (1.0 / 9007199254740992.0);
}

/* -------------------------------------------------------------------- CTMC */
/* The CTMC move of one state (section "Continuous time Monte Carlo"): E_L and
 * the rates r = |psi(M)/psi(N)| over the screened connected set, t = 1/T,
 * u from Philox, the smallest candidate index k whose running sum exceeds u*T
 * (the last positive-rate candidate if rounding leaves none).  Nothing is
 * changed; pick_out = {type, i, j, a, b} (type 0 = no move), *margin_out = the
 * smallest |u*T - C_k| / T over the running sums C_k. */
static int ctmc_eval(const orc_sys* s, orc_ws* w, const uint64_t* occ_bits, int mode, uint64_t seed,
                     uint64_t walker, uint64_t step, double* eloc, double* tres, int32_t* pick_out,
                     double* margin_out) {
    double el, T;
    int64_t nc;
    pick_out[0] = 0; pick_out[1] = pick_out[2] = pick_out[3] = pick_out[4] = -1;
    *tres = 0.0;
    *margin_out = 0.0;
    int rc = eloc_one(s, w, occ_bits, mode, &el, &T, &nc, 1, NULL);
    if (rc != 0) return rc;
    *eloc = el;
    if (!(T > 0.0)) return -3;
    *tres = 1.0 / T;
    double u = orc_uniform(seed, walker, step);
    double target = u * T;
    double run = 0.0, margin = INFINITY;
    int64_t pick = -1, last_pos = -1;
    for (int64_t k = 0; k < nc; ++k) {
        double r = fabs(w->cand[k].ratio);
        if (r > 0.0) last_pos = k;
        run += r;
        double d = fabs(target - run);
        if (d < margin) margin = d;
        if (pick < 0 && run > target) pick = k;
    }
    if (pick < 0) pick = last_pos;
    *margin_out = margin / T;
    const orc_cand* c = w->cand + pick;
    pick_out[0] = c->type; pick_out[1] = c->i; pick_out[2] = c->j; pick_out[3] = c->a; pick_out[4] = c->b;
    return 0;
}

/*
 * One CTMC move of walker `walker` at step `step` (ctmc_eval), applied to
 * occ_bits in place.  Returns 0, or a negative code when psi(N) = 0 or the
 * set is empty.
 */
int orc_ctmc_step(const orc_sys* s, uint64_t* occ_bits, int mode, uint64_t seed, uint64_t walker, uint64_t step,
                  double* eloc, double* tres, int32_t* pick_out, double* margin_out) {
    orc_ws* w = ws_alloc(s);
    int rc = ctmc_eval(s, w, occ_bits, mode, seed, walker, step, eloc, tres, pick_out, margin_out);
    if (rc == 0) {
        occ_clr(occ_bits, pick_out[1]);
        occ_set(occ_bits, pick_out[3]);
        if (pick_out[0] == 2) { occ_clr(occ_bits, pick_out[2]); occ_set(occ_bits, pick_out[4]); }
    }
    ws_free(w);
    return rc;
}

/* Teacher-forced evaluation of n independent states (OpenMP over states):
 * state k is the determinant occ_bits[k] of walker walker[k] at step step[k];
 * each gets its E_L, t, pick and margin as from orc_ctmc_step, without any
 * move being applied.  rc[k] = the return code. */
void orc_eval_states(const orc_sys* s, int64_t n, const uint64_t* occ_bits, int mode, uint64_t seed,
                     const int64_t* walker, const int64_t* step, double* eloc, double* tres, int32_t* pick,
                     double* margin, int32_t* rc, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        orc_ws* w = ws_alloc(s);
#pragma omp for schedule(dynamic)
        for (int64_t k = 0; k < n; ++k) {
            eloc[k] = NAN;
            rc[k] = ctmc_eval(s, w, occ_bits + k * s->nw, mode, seed, (uint64_t)walker[k], (uint64_t)step[k],
                              eloc + k, tres + k, pick + 5 * k, margin + k);
        }
        ws_free(w);
    }
}

/* ---------------------------------------------------------- gradient ratios */
/*
 * O_k for one walker, length n_so(n_so+1)/2 + n_so*n_so (+ the correlator
 * coefficients when correlators are set):
 *   Jastrow part (packed p<=q): n_p n_q;
 *   orbital part theta_kx (row-major): (theta[N]^-1)_{x, pos(k)} for occupied k
 *   and x < Ne, zero otherwise; pos(k) = row of k in the sorted theta[N];
 *   correlator part c_l[n]: 1/c_l[n] where n is the correlator's local Fock
 *   state in N, zero elsewhere.
 */
int orc_logderiv(const orc_sys* s, const uint64_t* occ_bits, double* out) {
    int nso = s->n_so, ne = s->ne;
    int64_t nj = (int64_t)nso * (nso + 1) / 2;
    int* occ = (int*)malloc(sizeof(int) * nso);
    int m = occ_list(s, occ_bits, occ);
    if (m != ne) { free(occ); return -2; }
    int64_t k = 0;
    for (int p = 0; p < nso; ++p)
        for (int q = p; q < nso; ++q) out[k++] = (double)(occ_test(occ_bits, p) * occ_test(occ_bits, q));
    double* A = (double*)malloc(sizeof(double) * ne * ne);
    double* Ainv = (double*)malloc(sizeof(double) * ne * ne);
    double* col = (double*)malloc(sizeof(double) * ne);
    int* perm = (int*)malloc(sizeof(int) * ne);
    for (int r = 0; r < ne; ++r)
        for (int c = 0; c < ne; ++c) A[r * ne + c] = s->theta[occ[r] * nso + c];
    int sg;
    lu_factor(A, ne, perm, &sg);
    double* th = out + nj;
    memset(th, 0, sizeof(double) * nso * nso);
    if (sg != 0) {
        lu_inverse(A, perm, ne, Ainv, col);
        for (int r = 0; r < ne; ++r)
            for (int x = 0; x < ne; ++x) th[occ[r] * nso + x] = Ainv[x * ne + r];
    }
    if (s->n_corr) {
        double* oc = th + (int64_t)nso * nso;
        memset(oc, 0, sizeof(double) * (size_t)s->coff[s->n_corr]);
        for (int l = 0; l < s->n_corr; ++l) {
            int64_t e = s->coff[l] + cps_state(s, l, occ_bits);
            oc[e] = 1.0 / s->cc[e];
        }
    }
    free(occ); free(A); free(Ainv); free(col); free(perm);
    return sg == 0 ? -1 : 0;
}

/* n_steps CTMC moves for each of nwalk walkers (OpenMP over walkers, each
 * walker sequential); occ_bits updated in place, eloc/tres [nwalk][n_steps]. */
void orc_ctmc_batch(const orc_sys* s, int64_t nwalk, uint64_t* occ_bits, int mode, uint64_t seed, uint64_t step0,
                    int n_steps, double* eloc, double* tres, int32_t* status, int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
#endif
#pragma omp parallel
    {
        orc_ws* w = ws_alloc(s);
#pragma omp for schedule(dynamic)
        for (int64_t k = 0; k < nwalk; ++k) {
            int32_t pick[5];
            double margin;
            uint64_t* bits = occ_bits + k * s->nw;
            status[k] = 0;
            for (int st = 0; st < n_steps; ++st) {
                int rc = ctmc_eval(s, w, bits, mode, seed, (uint64_t)k, step0 + (uint64_t)st, eloc + k * n_steps + st,
                                   tres + k * n_steps + st, pick, &margin);
                if (rc != 0) { status[k] = rc; break; }
                occ_clr(bits, pick[1]);
                occ_set(bits, pick[3]);
                if (pick[0] == 2) { occ_clr(bits, pick[2]); occ_set(bits, pick[4]); }
            }
        }
        ws_free(w);
    }
}
