/*
 * mgr_oracle.c -- plain, slow FP64 CPU oracle for MGR-preconditioned FGMRES.
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the independent reference that the
 * HIP library is checked against.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load it.  It shares no code, header,
 * table or helper with the GPU library, and the GPU library never calls it.
 *
 * Source of every step: Bui, Osei-Kuffuor, Castelletto, White, Falgout,
 * "Multigrid reduction preconditioning framework for coupled processes in
 * porous and fractured media" (arXiv 2101.11649):
 *   - block system by physical field ............ Sec. 1, eq. (1)
 *   - C/F partition, block LDU, Schur complement  Sec. 2, eq. (2)
 *   - ideal P and R ............................... Sec. 2, eq. (3)
 *   - Jacobi P + injection R ...................... Sec. 2, eq. (4)
 *   - Jacobi P + Jacobi R ......................... Sec. 2, eq. (5)
 *   - multilevel MGR V-cycle ...................... Sec. 2, Algorithm 1
 *   - Petrov-Galerkin coarse operator R A P ....... Sec. 2 (text after eq. (3))
 *   - AMG coarse solve / BoomerAMG settings ....... Sec. 4.1 (implementation details)
 *   - right-preconditioned GMRES .................. Sec. 4.1
 * Where the paper leaves a choice open the oracle takes these readings:
 *   - GMRES is the flexible right-preconditioned form (Saad 1993), classical
 *     Gram-Schmidt applied twice, Givens rotations, x0 = 0, converged when the
 *     Arnoldi residual estimate reaches rtol*||b|| and the true residual agrees.
 *   - HMIS coarsening is replaced by PMIS (De Sterck, Yang, Heys 2006), its
 *     parallel half, with splitmix64 random weights and an index tie-break.
 *   - Hybrid L1 Gauss-Seidel is replaced by L1 Jacobi (Baker et al. 2011).
 *   - Interpolation is Stueben's direct interpolation with positive
 *     off-diagonals lumped into the diagonal.
 *   - The coarsest AMG level is solved by LU with partial pivoting.
 * Floating point: build with -O2 -ffp-contract=off (no fused multiply-add, no
 * fast-math), so every product and sum is rounded exactly as written.
 */
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define ORC_OK 0
#define ORC_NOT_CONVERGED 1
#define ORC_ERR_ARG (-1)
#define ORC_ERR_ZERO_PIVOT (-3)
#define ORC_ERR_BAD_LABELS (-5)
#define ORC_ERR_UNSUPPORTED (-6)
#define AMG_INTERP_DIRECT 0
#define AMG_INTERP_EXT_I 1
#define AMG_SMOOTH_L1_JACOBI 0
#define AMG_SMOOTH_HYBRID_GS 1

#define FRELAX_JACOBI 0
#define FRELAX_BLOCK_JACOBI 1
#define FRELAX_ILU0 2
#define FRELAX_AMG 3
#define RESTRICT_INJECTION 0
#define RESTRICT_JACOBI 1

/* Threads: the solve phase (matvec, residuals, the MGR and AMG cycles, the
 * FGMRES vector work) runs its row loops with OpenMP; every row or entry is
 * still computed by one thread in the same order, and dot products use fixed
 * chunks, so results do not depend on the thread count.  Setup is serial. */
#define PAR_OK(n) ((n) > 4096)

#define MAX_AMG_LEVELS 40
#define MAX_MGR_LEVELS 8
#define MAX_DENSE 2048

/* ------------------------------------------------------------------------- */
/* Scalar CSR matrix (row pointers, column indices ascending, values).         */
/* ------------------------------------------------------------------------- */
typedef struct {
    int nr, nc;
    int *rp, *ci;
    double *v;
} Csr;

static void *xmalloc(size_t bytes) {
    void *p = malloc(bytes ? bytes : 1);
    if (!p) { fprintf(stderr, "oracle: out of memory (%zu bytes)\n", bytes); abort(); }
    return p;
}
static void *xcalloc(size_t n, size_t sz) {
    void *p = calloc(n ? n : 1, sz ? sz : 1);
    if (!p) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
    return p;
}

static Csr csr_alloc(int nr, int nc, long nnz) {
    Csr a;
    a.nr = nr; a.nc = nc;
    a.rp = (int *)xcalloc((size_t)nr + 1, sizeof(int));
    a.ci = (int *)xmalloc((size_t)nnz * sizeof(int));
    a.v = (double *)xmalloc((size_t)nnz * sizeof(double));
    return a;
}
static void csr_free(Csr *a) {
    free(a->rp); free(a->ci); free(a->v);
    a->rp = NULL; a->ci = NULL; a->v = NULL; a->nr = a->nc = 0;
}
static long csr_nnz(const Csr *a) { return a->rp ? a->rp[a->nr] : 0; }

static Csr csr_copy(const Csr *a) {
    Csr b = csr_alloc(a->nr, a->nc, csr_nnz(a));
    memcpy(b.rp, a->rp, ((size_t)a->nr + 1) * sizeof(int));
    memcpy(b.ci, a->ci, (size_t)csr_nnz(a) * sizeof(int));
    memcpy(b.v, a->v, (size_t)csr_nnz(a) * sizeof(double));
    return b;
}

/* The entries a_ij of A with label[i] == label[j] (the separate-component
 * approximation of a block whose unknowns carry field labels). */
static Csr csr_same_label(const Csr *a, const int *label) {
    Csr c;
    c.nr = a->nr; c.nc = a->nc;
    c.rp = (int *)xcalloc((size_t)a->nr + 1, sizeof(int));
    for (int i = 0; i < a->nr; ++i) {
        int cnt = 0;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) cnt += label[a->ci[p]] == label[i];
        c.rp[i + 1] = c.rp[i] + cnt;
    }
    int nnz = c.rp[a->nr];
    c.ci = (int *)xmalloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(int));
    c.v = (double *)xmalloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    for (int i = 0, q = 0; i < a->nr; ++i)
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p)
            if (label[a->ci[p]] == label[i]) { c.ci[q] = a->ci[p]; c.v[q] = a->v[p]; ++q; }
    return c;
}

/* y = A x, each row summed left to right. */
static void csr_matvec(const Csr *a, const double *x, double *y) {
    #pragma omp parallel for schedule(static) if (PAR_OK(a->nr))
    for (int i = 0; i < a->nr; ++i) {
        double s = 0.0;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) s += a->v[p] * x[a->ci[p]];
        y[i] = s;
    }
}

/* r = b - A x */
static void csr_residual(const Csr *a, const double *b, const double *x, double *r) {
    #pragma omp parallel for schedule(static) if (PAR_OK(a->nr))
    for (int i = 0; i < a->nr; ++i) {
        double s = 0.0;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) s += a->v[p] * x[a->ci[p]];
        r[i] = b[i] - s;
    }
}

/* Transpose by a counting sort over rows, so each output row is sorted. */
static Csr csr_transpose(const Csr *a) {
    long nnz = csr_nnz(a);
    Csr t = csr_alloc(a->nc, a->nr, nnz);
    for (long p = 0; p < nnz; ++p) t.rp[a->ci[p] + 1]++;
    for (int j = 0; j < a->nc; ++j) t.rp[j + 1] += t.rp[j];
    int *next = (int *)xmalloc((size_t)(a->nc + 1) * sizeof(int));
    memcpy(next, t.rp, (size_t)(a->nc + 1) * sizeof(int));
    for (int i = 0; i < a->nr; ++i)
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            int q = next[a->ci[p]]++;
            t.ci[q] = i;
            t.v[q] = a->v[p];
        }
    free(next);
    return t;
}

static int cmp_int(const void *x, const void *y) {
    int a = *(const int *)x, b = *(const int *)y;
    return (a > b) - (a < b);
}

/* C = A B by Gustavson's row-by-row method.  For every output entry (i,j) the
 * sum starts at 0.0 and adds a_ik * b_kj for k in the order the entries of row i
 * of A are stored (ascending column).  The output pattern is the symbolic one:
 * every (i,j) reached by some product is kept, explicit zeros included. */
static Csr csr_spgemm(const Csr *a, const Csr *b) {
    int *mark = (int *)xmalloc((size_t)(b->nc > 0 ? b->nc : 1) * sizeof(int));
    for (int j = 0; j < b->nc; ++j) mark[j] = -1;
    int *rp = (int *)xcalloc((size_t)a->nr + 1, sizeof(int));
    for (int i = 0; i < a->nr; ++i) {
        int cnt = 0;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            int k = a->ci[p];
            for (int q = b->rp[k]; q < b->rp[k + 1]; ++q) {
                int j = b->ci[q];
                if (mark[j] != i) { mark[j] = i; cnt++; }
            }
        }
        rp[i + 1] = rp[i] + cnt;
    }
    Csr c;
    c.nr = a->nr; c.nc = b->nc; c.rp = rp;
    c.ci = (int *)xmalloc((size_t)rp[a->nr] * sizeof(int));
    c.v = (double *)xmalloc((size_t)rp[a->nr] * sizeof(double));
    double *acc = (double *)xmalloc((size_t)(b->nc > 0 ? b->nc : 1) * sizeof(double));
    for (int j = 0; j < b->nc; ++j) mark[j] = -1;
    for (int i = 0; i < a->nr; ++i) {
        int *list = c.ci + rp[i];
        int len = 0;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            int k = a->ci[p];
            double av = a->v[p];
            for (int q = b->rp[k]; q < b->rp[k + 1]; ++q) {
                int j = b->ci[q];
                if (mark[j] != i) { mark[j] = i; acc[j] = 0.0; list[len++] = j; }
                acc[j] += av * b->v[q];
            }
        }
        qsort(list, (size_t)len, sizeof(int), cmp_int);
        for (int t = 0; t < len; ++t) c.v[rp[i] + t] = acc[list[t]];
    }
    free(mark); free(acc);
    return c;
}

/* C = A + B on the union pattern; where both are present the value is a + b. */
static Csr csr_add(const Csr *a, const Csr *b) {
    int *rp = (int *)xcalloc((size_t)a->nr + 1, sizeof(int));
    for (int i = 0; i < a->nr; ++i) {
        int p = a->rp[i], pe = a->rp[i + 1], q = b->rp[i], qe = b->rp[i + 1], cnt = 0;
        while (p < pe || q < qe) {
            if (q >= qe || (p < pe && a->ci[p] < b->ci[q])) p++;
            else if (p >= pe || b->ci[q] < a->ci[p]) q++;
            else { p++; q++; }
            cnt++;
        }
        rp[i + 1] = rp[i] + cnt;
    }
    Csr c;
    c.nr = a->nr; c.nc = a->nc; c.rp = rp;
    c.ci = (int *)xmalloc((size_t)rp[a->nr] * sizeof(int));
    c.v = (double *)xmalloc((size_t)rp[a->nr] * sizeof(double));
    for (int i = 0; i < a->nr; ++i) {
        int p = a->rp[i], pe = a->rp[i + 1], q = b->rp[i], qe = b->rp[i + 1], o = rp[i];
        while (p < pe || q < qe) {
            if (q >= qe || (p < pe && a->ci[p] < b->ci[q])) { c.ci[o] = a->ci[p]; c.v[o] = a->v[p]; p++; }
            else if (p >= pe || b->ci[q] < a->ci[p]) { c.ci[o] = b->ci[q]; c.v[o] = b->v[q]; q++; }
            else { c.ci[o] = a->ci[p]; c.v[o] = a->v[p] + b->v[q]; p++; q++; }
            o++;
        }
    }
    return c;
}

static void csr_negate(Csr *a) {
    long nnz = csr_nnz(a);
    for (long p = 0; p < nnz; ++p) a->v[p] = -a->v[p];
}

/* Rows `rows[0..nrows)` of A, keeping only columns with colmap[j] >= 0 and
 * renumbering them to colmap[j]; column order is preserved. */
static Csr csr_extract(const Csr *a, const int *rows, int nrows, const int *colmap, int ncols) {
    int *rp = (int *)xcalloc((size_t)nrows + 1, sizeof(int));
    for (int r = 0; r < nrows; ++r) {
        int i = rows[r], cnt = 0;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) if (colmap[a->ci[p]] >= 0) cnt++;
        rp[r + 1] = rp[r] + cnt;
    }
    Csr c;
    c.nr = nrows; c.nc = ncols; c.rp = rp;
    c.ci = (int *)xmalloc((size_t)rp[nrows] * sizeof(int));
    c.v = (double *)xmalloc((size_t)rp[nrows] * sizeof(double));
    for (int r = 0; r < nrows; ++r) {
        int i = rows[r], o = rp[r];
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            int m = colmap[a->ci[p]];
            if (m >= 0) { c.ci[o] = m; c.v[o] = a->v[p]; o++; }
        }
    }
    return c;
}

/* Scalar CSR of a block-CSR matrix (b x b row-major blocks).  An exact zero
 * inside a stored block is not an entry of the operator (it contributes to no
 * product or sum), so it is left out, except on the diagonal, which is always
 * stored. */
static Csr bsr_expand(int b, int nbr, int nbc, const int *rp, const int *ci, const double *val) {
    long nnzb = rp[nbr];
    Csr a = csr_alloc(nbr * b, nbc * b, nnzb * b * b);
    long o = 0;
    for (int I = 0; I < nbr; ++I)
        for (int r = 0; r < b; ++r) {
            int row = I * b + r;
            for (int p = rp[I]; p < rp[I + 1]; ++p)
                for (int c = 0; c < b; ++c) {
                    int col = ci[p] * b + c;
                    double v = val[(long)p * b * b + r * b + c];
                    if (v == 0.0 && col != row) continue;
                    a.ci[o] = col;
                    a.v[o] = v;
                    o++;
                }
            a.rp[row + 1] = (int)o;
        }
    return a;
}

/* Dot product in fixed chunks of DOT_CHUNK entries: each chunk is summed left
 * to right, then the chunk sums left to right, so the result is the same
 * whatever the number of threads (one chunk: the plain left-to-right sum). */
#define DOT_CHUNK 8192
static double dot(int n, const double *x, const double *y) {
    int nch = (n + DOT_CHUNK - 1) / DOT_CHUNK;
    if (nch <= 1) {
        double s = 0.0;
        for (int i = 0; i < n; ++i) s += x[i] * y[i];
        return s;
    }
    double *part = (double *)xmalloc((size_t)nch * sizeof(double));
    #pragma omp parallel for schedule(static)
    for (int c = 0; c < nch; ++c) {
        int i1 = (c + 1) * DOT_CHUNK < n ? (c + 1) * DOT_CHUNK : n;
        double s = 0.0;
        for (int i = c * DOT_CHUNK; i < i1; ++i) s += x[i] * y[i];
        part[c] = s;
    }
    double s = 0.0;
    for (int c = 0; c < nch; ++c) s += part[c];
    free(part);
    return s;
}
static double nrm2(int n, const double *x) { return sqrt(dot(n, x, x)); }

/* ------------------------------------------------------------------------- */
/* Dense LU with partial pivoting (the coarsest-level "Gaussian elimination", */
/* Sec. 4.1).  Pivot = largest |entry| in the column, ties to the lower row.   */
/* ------------------------------------------------------------------------- */
static int lu_factor(int n, double *m, int *piv) {
    for (int c = 0; c < n; ++c) {
        int p = c;
        double best = fabs(m[(long)c * n + c]);
        for (int r = c + 1; r < n; ++r) {
            double t = fabs(m[(long)r * n + c]);
            if (t > best) { best = t; p = r; }
        }
        piv[c] = p;
        if (!(best > 0.0) || !isfinite(best)) return ORC_ERR_ZERO_PIVOT;
        if (p != c)
            for (int k = 0; k < n; ++k) {
                double t = m[(long)c * n + k];
                m[(long)c * n + k] = m[(long)p * n + k];
                m[(long)p * n + k] = t;
            }
        for (int r = c + 1; r < n; ++r) {
            double l = m[(long)r * n + c] / m[(long)c * n + c];
            m[(long)r * n + c] = l;
            for (int k = c + 1; k < n; ++k) m[(long)r * n + k] -= l * m[(long)c * n + k];
        }
    }
    return ORC_OK;
}

/* Solve (P A) x = P b given the packed LU of P A, or A^T x = b when trans. */
static void lu_solve(int n, const double *m, const int *piv, const double *b, double *x, int trans) {
    if (!trans) {
        for (int i = 0; i < n; ++i) x[i] = b[i];
        for (int c = 0; c < n; ++c) if (piv[c] != c) { double t = x[c]; x[c] = x[piv[c]]; x[piv[c]] = t; }
        for (int i = 0; i < n; ++i) {               /* L y = P b, unit diagonal */
            double s = x[i];
            for (int k = 0; k < i; ++k) s -= m[(long)i * n + k] * x[k];
            x[i] = s;
        }
        for (int i = n - 1; i >= 0; --i) {          /* U x = y */
            double s = x[i];
            for (int k = i + 1; k < n; ++k) s -= m[(long)i * n + k] * x[k];
            x[i] = s / m[(long)i * n + i];
        }
    } else {
        /* A^T = U^T L^T P, so solve U^T y = b, L^T w = y, x = P^T w. */
        for (int i = 0; i < n; ++i) x[i] = b[i];
        for (int i = 0; i < n; ++i) {
            double s = x[i];
            for (int k = 0; k < i; ++k) s -= m[(long)k * n + i] * x[k];
            x[i] = s / m[(long)i * n + i];
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = x[i];
            for (int k = i + 1; k < n; ++k) s -= m[(long)k * n + i] * x[k];
            x[i] = s;
        }
        for (int c = n - 1; c >= 0; --c) if (piv[c] != c) { double t = x[c]; x[c] = x[piv[c]]; x[piv[c]] = t; }
    }
}

/* Gauss-Jordan inverse with partial pivoting of a small dense block (the
 * block-Jacobi F-relaxation operator).  The arithmetic order is fixed: scale
 * the pivot row by 1/pivot, then subtract f * pivot_row from every other row. */
static int small_inverse(int bs, const double *blk, double *inv) {
    double a[16], e[16];
    for (int i = 0; i < bs * bs; ++i) a[i] = blk[i];
    for (int i = 0; i < bs; ++i) for (int j = 0; j < bs; ++j) e[i * bs + j] = (i == j) ? 1.0 : 0.0;
    for (int c = 0; c < bs; ++c) {
        int p = c;
        double best = fabs(a[c * bs + c]);
        for (int r = c + 1; r < bs; ++r) if (fabs(a[r * bs + c]) > best) { best = fabs(a[r * bs + c]); p = r; }
        if (!(best > 0.0) || !isfinite(best)) return ORC_ERR_ZERO_PIVOT;
        if (p != c)
            for (int k = 0; k < bs; ++k) {
                double t = a[c * bs + k]; a[c * bs + k] = a[p * bs + k]; a[p * bs + k] = t;
                t = e[c * bs + k]; e[c * bs + k] = e[p * bs + k]; e[p * bs + k] = t;
            }
        double ip = 1.0 / a[c * bs + c];
        for (int k = 0; k < bs; ++k) { a[c * bs + k] = a[c * bs + k] * ip; e[c * bs + k] = e[c * bs + k] * ip; }
        for (int r = 0; r < bs; ++r) {
            if (r == c) continue;
            double f = a[r * bs + c];
            for (int k = 0; k < bs; ++k) {
                a[r * bs + k] = a[r * bs + k] - f * a[c * bs + k];
                e[r * bs + k] = e[r * bs + k] - f * e[c * bs + k];
            }
        }
    }
    for (int i = 0; i < bs * bs; ++i) inv[i] = e[i];
    return ORC_OK;
}

/* ------------------------------------------------------------------------- */
/* splitmix64 (Steele, Lea, Flood, OOPSLA 2014): output number k of the        */
/* generator seeded with `seed` is mix(seed + k * 0x9E3779B97F4A7C15).         */
/* ------------------------------------------------------------------------- */
static uint64_t splitmix64_at(uint64_t seed, uint64_t k) {
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}
/* Uniform [0,1) number for point i on AMG level `level`: top 53 bits. */
static double pmis_uniform(uint64_t seed, int level, int i) {
    uint64_t k = ((uint64_t)(unsigned)level << 32) + (uint64_t)(unsigned)i + 1ULL;
    return (double)(splitmix64_at(seed, k) >> 11) * (1.0 / 9007199254740992.0);
}

/* ------------------------------------------------------------------------- */
/* Classical AMG pieces (the coarse-grid solver of Sec. 4.1).                  */
/* ------------------------------------------------------------------------- */

/* Strength of connection: j in S_i iff j != i (and label_j == label_i when
 * labels are given, the unknown-based approach) and -a_ij >= theta * max_k(-a_ik)
 * with the max over the same off-diagonal set; S_i is empty when that max <= 0. */
static void amg_strength(const Csr *a, double theta, const int *label, unsigned char *strong) {
    for (int i = 0; i < a->nr; ++i) {
        double mx = 0.0;
        int have = 0;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            int j = a->ci[p];
            if (j == i || (label && label[j] != label[i])) continue;
            double t = -a->v[p];
            if (!have || t > mx) { mx = t; have = 1; }
        }
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            int j = a->ci[p];
            strong[p] = 0;
            if (!have || !(mx > 0.0)) continue;
            if (j == i || (label && label[j] != label[i])) continue;
            if (-a->v[p] >= theta * mx) strong[p] = 1;
        }
    }
}

/* PMIS (De Sterck, Yang, Heys, SIAM J. Matrix Anal. Appl. 27 (2006)).
 * cf: +1 = C, -1 = F.  Weight w_i = |S^T_i| + u_i; points nobody depends on
 * start as F; each synchronous round selects the undecided points whose
 * (w, index) beats every undecided neighbour in S_i and S^T_i, makes them C,
 * and makes F every undecided point that strongly depends on a new C point. */
static int amg_pmis(const Csr *a, const unsigned char *strong, uint64_t seed, int level, int *cf) {
    int n = a->nr;
    long nnz = csr_nnz(a);
    int *lam = (int *)xcalloc((size_t)n, sizeof(int));
    for (long p = 0; p < nnz; ++p) if (strong[p]) lam[a->ci[p]]++;
    /* transpose of the strength graph: row j lists the i with j in S_i */
    int *trp = (int *)xcalloc((size_t)n + 1, sizeof(int));
    for (int j = 0; j < n; ++j) trp[j + 1] = trp[j] + lam[j];
    int *tci = (int *)xmalloc((size_t)(trp[n] > 0 ? trp[n] : 1) * sizeof(int));
    int *nxt = (int *)xmalloc((size_t)n * sizeof(int));
    for (int j = 0; j < n; ++j) nxt[j] = trp[j];
    for (int i = 0; i < n; ++i)
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) if (strong[p]) tci[nxt[a->ci[p]]++] = i;
    double *w = (double *)xmalloc((size_t)n * sizeof(double));
    int undecided = 0;
    for (int i = 0; i < n; ++i) {
        w[i] = (double)lam[i] + pmis_uniform(seed, level, i);
        cf[i] = (lam[i] == 0) ? -1 : 0;
        if (!cf[i]) undecided++;
    }
    unsigned char *newc = (unsigned char *)xcalloc((size_t)n, 1);
    int rounds = 0;
    while (undecided > 0) {
        rounds++;
        for (int i = 0; i < n; ++i) {
            newc[i] = 0;
            if (cf[i] != 0) continue;
            int best = 1;
            for (int p = a->rp[i]; p < a->rp[i + 1] && best; ++p) {
                if (!strong[p]) continue;
                int j = a->ci[p];
                if (cf[j] == 0 && (w[j] > w[i] || (w[j] == w[i] && j > i))) best = 0;
            }
            for (int q = trp[i]; q < trp[i + 1] && best; ++q) {
                int j = tci[q];
                if (cf[j] == 0 && (w[j] > w[i] || (w[j] == w[i] && j > i))) best = 0;
            }
            newc[i] = (unsigned char)best;
        }
        for (int i = 0; i < n; ++i) if (newc[i]) cf[i] = 1;
        for (int i = 0; i < n; ++i) {
            if (cf[i] != 0) continue;
            for (int p = a->rp[i]; p < a->rp[i + 1]; ++p)
                if (strong[p] && newc[a->ci[p]]) { cf[i] = -1; break; }
        }
        undecided = 0;
        for (int i = 0; i < n; ++i) if (cf[i] == 0) undecided++;
    }
    free(lam); free(trp); free(tci); free(nxt); free(w); free(newc);
    return rounds;
}

/* Direct interpolation (Stueben, J. Comput. Appl. Math. 128 (2001)): for an
 * F-point i with interpolatory set C_i = S_i intersect C,
 *   w_ij = -(alpha_i * a_ij) / atilde_ii,  alpha_i = neg_i / cs_i,
 *   neg_i = sum_{k != i, a_ik < 0} a_ik,   cs_i = sum_{k in C_i} a_ik,
 *   atilde_ii = a_ii + sum_{k != i, a_ik > 0} a_ik,
 * every sum taken left to right over the row.  C-rows are unit rows; F-rows with
 * an empty C_i are zero.  With labels only same-label couplings are used. */
static int amg_direct_interp_cols(const Csr *a, const unsigned char *strong, const int *cf, const int *label,
                                  int identity_cols, Csr *pout) {
    int n = a->nr;
    int *cidx = (int *)xmalloc((size_t)n * sizeof(int));
    int nc = 0;
    for (int i = 0; i < n; ++i) cidx[i] = (cf[i] == 1) ? nc++ : -1;
    if (identity_cols) {
        /* columns are the points themselves (an n x n operator) */
        for (int i = 0; i < n; ++i) if (cf[i] == 1) cidx[i] = i;
        nc = n;
    }
    int *rp = (int *)xcalloc((size_t)n + 1, sizeof(int));
    for (int i = 0; i < n; ++i) {
        int cnt = 0;
        if (cf[i] == 1) cnt = 1;
        else
            for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) if (strong[p] && cf[a->ci[p]] == 1) cnt++;
        rp[i + 1] = rp[i] + cnt;
    }
    Csr pm;
    pm.nr = n; pm.nc = nc; pm.rp = rp;
    pm.ci = (int *)xmalloc((size_t)(rp[n] > 0 ? rp[n] : 1) * sizeof(int));
    pm.v = (double *)xmalloc((size_t)(rp[n] > 0 ? rp[n] : 1) * sizeof(double));
    int status = ORC_OK;
    for (int i = 0; i < n; ++i) {
        int o = rp[i];
        if (cf[i] == 1) { pm.ci[o] = cidx[i]; pm.v[o] = 1.0; continue; }
        if (rp[i + 1] == rp[i]) continue;
        double aii = 0.0, neg = 0.0, pos = 0.0, cs = 0.0;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            int k = a->ci[p];
            double v = a->v[p];
            if (k == i) { aii = v; continue; }
            if (label && label[k] != label[i]) continue;
            if (v < 0.0) neg += v;
            else if (v > 0.0) pos += v;
            if (strong[p] && cf[k] == 1) cs += v;
        }
        double atil = aii + pos;
        if (!(atil > 0.0)) status = ORC_ERR_UNSUPPORTED;
        double alpha = neg / cs;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            int k = a->ci[p];
            if (strong[p] && cf[k] == 1) {
                pm.ci[o] = cidx[k];
                pm.v[o] = -(alpha * a->v[p]) / atil;
                o++;
            }
        }
    }
    free(cidx);
    *pout = pm;
    return status;
}

static int amg_direct_interp(const Csr *a, const unsigned char *strong, const int *cf, const int *label,
                             Csr *pout) {
    return amg_direct_interp_cols(a, strong, cf, label, 0, pout);
}

/* Multi-pass interpolation (Stueben, J. Comput. Appl. Math. 128 (2001)), the
 * interpolation of an aggressively coarsened level, where many F-points have no
 * strong C-neighbour.  Pass 1 is direct interpolation.  In each further pass,
 * every F-point still without interpolation whose strong neighbours include
 * points interpolated before this pass (C-points, or F-points of earlier
 * passes) takes the direct-interpolation weights w_ij over those neighbours
 * (their couplings play the part of C_i) and substitutes their interpolation:
 * P_i = sum_j w_ij P_j, formed as the product W P of the pass's weight operator
 * (unit rows for the points interpolated before) with the current P, in
 * Gustavson order.  F-points reached by no pass keep zero rows. */
static int amg_multipass_interp(const Csr *a, const unsigned char *strong, const int *cf, const int *label,
                                Csr *pout) {
    int n = a->nr;
    Csr P;
    int status = amg_direct_interp_cols(a, strong, cf, label, 0, &P);
    int *cfm = (int *)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    while (status == ORC_OK) {
        for (int i = 0; i < n; ++i) cfm[i] = (cf[i] == 1 || P.rp[i + 1] > P.rp[i]) ? 1 : -1;
        int reach = 0;
        for (int i = 0; i < n && !reach; ++i) {
            if (cfm[i] == 1) continue;
            for (int p = a->rp[i]; p < a->rp[i + 1]; ++p)
                if (strong[p] && cfm[a->ci[p]] == 1) { reach = 1; break; }
        }
        if (!reach) break;
        Csr W;
        status = amg_direct_interp_cols(a, strong, cfm, label, 1, &W);
        Csr Pn = csr_spgemm(&W, &P);
        csr_free(&W);
        csr_free(&P);
        P = Pn;
    }
    free(cfm);
    *pout = P;
    return status;
}

/* Aggressive coarsening of one level (Stueben 2001: coarse points at distance
 * two).  PMIS on the strength graph S gives a first set C1.  On C1, point j is
 * a second-order strong neighbour of i (i != j) when one or two strong
 * connections lead from i to j (j in S_i, or j in S_k for some k in S_i, any
 * intermediate point).  PMIS again on that graph of C1 points, with the random
 * weights of stream (seed, level + 64) indexed by the position in C1, keeps
 * the final C-points; the other points of C1 become F.  cf: +1 = C, -1 = F. */
static void amg_aggressive_split(const Csr *a, const unsigned char *strong, uint64_t seed, int level, int *cf) {
    int n = a->nr;
    amg_pmis(a, strong, seed, level, cf);
    int *c1 = (int *)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(int));
    int n1 = 0;
    for (int i = 0; i < n; ++i) c1[i] = (cf[i] == 1) ? n1++ : -1;
    int *mark = (int *)xmalloc((size_t)(n1 > 0 ? n1 : 1) * sizeof(int));
    int *list = (int *)xmalloc((size_t)(n1 > 0 ? n1 : 1) * sizeof(int));
    Csr g;
    g.nr = g.nc = n1;
    g.rp = (int *)xcalloc((size_t)n1 + 1, sizeof(int));
    g.v = NULL;
    long cap = 16, used = 0;
    g.ci = (int *)xmalloc((size_t)cap * sizeof(int));
    for (int j = 0; j < n1; ++j) mark[j] = -1;
    for (int i = 0; i < n; ++i) {
        int ii = c1[i];
        if (ii < 0) continue;
        int cnt = 0;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            if (!strong[p]) continue;
            int k = a->ci[p];
            int kk = c1[k];
            if (kk >= 0 && kk != ii && mark[kk] != ii) { mark[kk] = ii; list[cnt++] = kk; }
            for (int q = a->rp[k]; q < a->rp[k + 1]; ++q) {
                if (!strong[q]) continue;
                int jj = c1[a->ci[q]];
                if (jj >= 0 && jj != ii && mark[jj] != ii) { mark[jj] = ii; list[cnt++] = jj; }
            }
        }
        /* ascending columns (insertion sort: rows are short) */
        for (int t = 1; t < cnt; ++t) {
            int v = list[t], u = t - 1;
            while (u >= 0 && list[u] > v) { list[u + 1] = list[u]; u--; }
            list[u + 1] = v;
        }
        if (used + cnt > cap) {
            while (used + cnt > cap) cap *= 2;
            g.ci = (int *)realloc(g.ci, (size_t)cap * sizeof(int));
            if (!g.ci) { fprintf(stderr, "oracle: out of memory\n"); abort(); }
        }
        memcpy(g.ci + used, list, (size_t)cnt * sizeof(int));
        used += cnt;
        g.rp[ii + 1] = (int)used;
    }
    unsigned char *all = (unsigned char *)xmalloc((size_t)(used > 0 ? used : 1));
    memset(all, 1, (size_t)(used > 0 ? used : 1));
    int *cf2 = (int *)xmalloc((size_t)(n1 > 0 ? n1 : 1) * sizeof(int));
    amg_pmis(&g, all, seed, level + 64, cf2);
    for (int i = 0; i < n; ++i)
        if (c1[i] >= 0 && cf2[c1[i]] != 1) cf[i] = -1;
    free(cf2); free(all); free(g.rp); free(g.ci); free(list); free(mark); free(c1);
}

/* Extended+i interpolation (De Sterck, Falgout, Nolting, Yang, Numer. Linear
 * Algebra Appl. 15 (2008), the distance-two interpolation paired with PMIS-type
 * coarsening).  For an F-point i with strong C- and F-neighbours C_i^s, F_i^s
 * (S_i, as in the strength definition) and other same-label neighbours
 * (weak), the interpolatory set is
 *   Chat_i = C_i^s  union  (union over k in F_i^s of C_k^s),
 * abar_kl = a_kl where a_kl < 0 (opposite in sign to the positive a_kk), else 0,
 * d_k = sum over l in Chat_i + {i} of abar_kl (row k left to right), and
 *   atilde_ii = a_ii + sum_{weak n not in Chat_i} a_in
 *               + sum_{k in F_i^s} a_ik abar_ki / d_k,
 *   w_ij = -(a_ij + sum_{k in F_i^s} a_ik abar_kj / d_k) / atilde_ii   (j in Chat_i),
 * with a_ij = 0 when j is not a neighbour of i.  A strong F-neighbour with
 * d_k = 0 is lumped into the diagonal (atilde_ii += a_ik).  Order: the weak
 * terms follow a_ii in row order, then the k terms in row order; each w_ij
 * numerator starts from a_ij and adds its k terms in row order; each term is
 * (a_ik * abar_kl) / d_k.  Columns of P ascend.  C-rows are unit rows; F-rows
 * with an empty Chat_i are zero.  With labels only same-label couplings are
 * used. */
static int amg_ext_interp(const Csr *a, const unsigned char *strong, const int *cf, const int *label, Csr *pout) {
    int n = a->nr;
    int *cidx = (int *)xmalloc((size_t)n * sizeof(int));
    int nc = 0;
    for (int i = 0; i < n; ++i) cidx[i] = (cf[i] == 1) ? nc++ : -1;
    int *mark = (int *)xmalloc((size_t)n * sizeof(int));       /* mark[j] == i + 1: j in Chat_i */
    int *slot = (int *)xmalloc((size_t)n * sizeof(int));       /* position of j in the sorted Chat_i */
    for (int i = 0; i < n; ++i) mark[i] = 0;
    int *rp = (int *)xcalloc((size_t)n + 1, sizeof(int));
    int *list = (int *)xmalloc((size_t)n * sizeof(int));
    /* symbolic pass: |Chat_i| */
    for (int i = 0; i < n; ++i) {
        int cnt = 0;
        if (cf[i] == 1) cnt = 1;
        else
            for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
                if (!strong[p]) continue;
                int k = a->ci[p];
                if (cf[k] == 1) { if (mark[k] != i + 1) { mark[k] = i + 1; cnt++; } continue; }
                for (int q = a->rp[k]; q < a->rp[k + 1]; ++q) {
                    int l = a->ci[q];
                    if (strong[q] && cf[l] == 1 && mark[l] != i + 1) { mark[l] = i + 1; cnt++; }
                }
            }
        rp[i + 1] = rp[i] + cnt;
    }
    Csr pm;
    pm.nr = n; pm.nc = nc; pm.rp = rp;
    pm.ci = (int *)xmalloc((size_t)(rp[n] > 0 ? rp[n] : 1) * sizeof(int));
    pm.v = (double *)xmalloc((size_t)(rp[n] > 0 ? rp[n] : 1) * sizeof(double));
    double *num = (double *)xmalloc((size_t)n * sizeof(double));
    for (int i = 0; i < n; ++i) mark[i] = 0;
    int status = ORC_OK;
    for (int i = 0; i < n; ++i) {
        int o = rp[i];
        if (cf[i] == 1) { pm.ci[o] = cidx[i]; pm.v[o] = 1.0; continue; }
        int m = rp[i + 1] - rp[i];
        if (m == 0) continue;
        /* Chat_i in ascending order */
        int c = 0;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            if (!strong[p]) continue;
            int k = a->ci[p];
            if (cf[k] == 1) { if (mark[k] != i + 1) { mark[k] = i + 1; list[c++] = k; } continue; }
            for (int q = a->rp[k]; q < a->rp[k + 1]; ++q) {
                int l = a->ci[q];
                if (strong[q] && cf[l] == 1 && mark[l] != i + 1) { mark[l] = i + 1; list[c++] = l; }
            }
        }
        qsort(list, (size_t)c, sizeof(int), cmp_int);
        for (int t = 0; t < c; ++t) { slot[list[t]] = t; num[t] = 0.0; }
        /* a_ii, a_ij (j in Chat_i) and the weak terms */
        double aii = 0.0, atil;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p)
            if (a->ci[p] == i) aii = a->v[p];
        atil = aii;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            int j = a->ci[p];
            if (j == i || (label && label[j] != label[i])) continue;
            if (mark[j] == i + 1) num[slot[j]] = a->v[p];
            else if (!strong[p]) atil += a->v[p];
        }
        /* the strong F-neighbours, in row order */
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
            int k = a->ci[p];
            if (!strong[p] || cf[k] == 1) continue;
            double aik = a->v[p], d = 0.0;
            for (int q = a->rp[k]; q < a->rp[k + 1]; ++q) {
                int l = a->ci[q];
                if (a->v[q] < 0.0 && l != k && (l == i || mark[l] == i + 1)) d += a->v[q];
            }
            if (d == 0.0) { atil += aik; continue; }
            for (int q = a->rp[k]; q < a->rp[k + 1]; ++q) {
                int l = a->ci[q];
                if (!(a->v[q] < 0.0) || l == k) continue;
                if (l == i) atil += (aik * a->v[q]) / d;
                else if (mark[l] == i + 1) num[slot[l]] += (aik * a->v[q]) / d;
            }
        }
        if (!(atil > 0.0)) status = ORC_ERR_UNSUPPORTED;
        for (int t = 0; t < c; ++t) {
            pm.ci[o + t] = cidx[list[t]];
            pm.v[o + t] = -num[t] / atil;
        }
    }
    free(cidx); free(mark); free(slot); free(list); free(num);
    *pout = pm;
    return status;
}

typedef struct {
    double theta;
    int max_levels, max_coarse, nu_pre, nu_post, unknown_based;
    int interp;             /* AMG_INTERP_DIRECT or AMG_INTERP_EXT_I */
    int smoother;           /* AMG_SMOOTH_L1_JACOBI or AMG_SMOOTH_HYBRID_GS */
    int chunk;              /* rows per chunk of the hybrid Gauss-Seidel smoother */
    int agg_levels;         /* the first agg_levels levels coarsen aggressively */
    uint64_t seed;
} AmgOpts;

typedef struct {
    int nlev;                         /* levels including the coarsest        */
    Csr A[MAX_AMG_LEVELS], AT[MAX_AMG_LEVELS];
    Csr P[MAX_AMG_LEVELS], R[MAX_AMG_LEVELS];
    int *cf[MAX_AMG_LEVELS];
    int *label[MAX_AMG_LEVELS];
    double *dl1[MAX_AMG_LEVELS];      /* L1 diagonal a_ii + sum_{j!=i} |a_ij|   */
    double *dgs[MAX_AMG_LEVELS];      /* hybrid GS diagonal a_ii + sum_{j outside i's chunk} |a_ij| */
    int smoother, chunk;
    int nu_pre, nu_post;
    int nc;                           /* coarsest size                         */
    double *lu;
    int *piv;
    double **wb, **wx, **wr;          /* per-level work vectors               */
} Amg;

static void amg_free(Amg *h) {
    if (!h) return;
    for (int k = 0; k < h->nlev; ++k) {
        csr_free(&h->A[k]); csr_free(&h->AT[k]);
        if (k < h->nlev - 1) {
            csr_free(&h->P[k]); csr_free(&h->R[k]); free(h->cf[k]); free(h->dl1[k]); free(h->dgs[k]);
        }
        free(h->label[k]);
        free(h->wb[k]); free(h->wx[k]); free(h->wr[k]);
    }
    free(h->wb); free(h->wx); free(h->wr);
    free(h->lu); free(h->piv);
    free(h);
}

static int amg_finish(Amg *h, int k, int status);
static int amg_l1_diag(Amg *h, int k);

/* Setup of the AMG hierarchy: strength, PMIS, direct interpolation, Galerkin
 * product A_{k+1} = P^T (A_k P) (both SpGEMMs in Gustavson order), until the
 * level is small (<= max_coarse), the level cap is reached, or coarsening
 * stalls (n_{k+1} > 0.9 n_k or no C-point); the last level is factored. */
static int amg_setup(const Csr *a0, const int *label0, const AmgOpts *o, Amg **out) {
    Amg *h = (Amg *)xcalloc(1, sizeof(Amg));
    h->nu_pre = o->nu_pre; h->nu_post = o->nu_post;
    h->smoother = o->smoother; h->chunk = o->chunk;
    h->A[0] = csr_copy(a0);
    if (o->unknown_based && label0) {
        h->label[0] = (int *)xmalloc((size_t)a0->nr * sizeof(int));
        memcpy(h->label[0], label0, (size_t)a0->nr * sizeof(int));
    }
    int k = 0, status = ORC_OK;
    for (;;) {
        const Csr *a = &h->A[k];
        int n = a->nr;
        if (n <= o->max_coarse || k + 1 >= o->max_levels) break;
        unsigned char *strong = (unsigned char *)xmalloc((size_t)(csr_nnz(a) > 0 ? csr_nnz(a) : 1));
        amg_strength(a, o->theta, h->label[k], strong);
        int *cf = (int *)xmalloc((size_t)n * sizeof(int));
        const int aggressive = k < o->agg_levels;
        if (aggressive) amg_aggressive_split(a, strong, o->seed, k, cf);
        else amg_pmis(a, strong, o->seed, k, cf);
        int nc = 0;
        for (int i = 0; i < n; ++i) nc += (cf[i] == 1);
        if (nc == 0 || (double)nc > 0.9 * (double)n) { free(strong); free(cf); break; }
        Csr p;
        int st = aggressive ? amg_multipass_interp(a, strong, cf, h->label[k], &p)
                 : o->interp == AMG_INTERP_EXT_I ? amg_ext_interp(a, strong, cf, h->label[k], &p)
                                                 : amg_direct_interp(a, strong, cf, h->label[k], &p);
        free(strong);
        if (st != ORC_OK) { free(cf); csr_free(&p); status = st; break; }
        h->cf[k] = cf;
        h->P[k] = p;
        h->R[k] = csr_transpose(&p);
        Csr ap = csr_spgemm(a, &p);
        h->A[k + 1] = csr_spgemm(&h->R[k], &ap);
        csr_free(&ap);
        if (h->label[k]) {
            h->label[k + 1] = (int *)xmalloc((size_t)nc * sizeof(int));
            for (int i = 0, c = 0; i < n; ++i) if (cf[i] == 1) h->label[k + 1][c++] = h->label[k][i];
        }
        int sl = amg_l1_diag(h, k);
        if (sl != ORC_OK) status = sl;
        k++;
    }
    *out = h;
    return amg_finish(h, k, status);
}

/* Transposes, work vectors and the LU factors of the coarsest level k. */
static int amg_finish(Amg *h, int k, int status) {
    h->nlev = k + 1;
    for (int l = 0; l < h->nlev; ++l) h->AT[l] = csr_transpose(&h->A[l]);
    int nc = h->A[k].nr;
    h->nc = nc;
    h->wb = (double **)xcalloc((size_t)h->nlev, sizeof(double *));
    h->wx = (double **)xcalloc((size_t)h->nlev, sizeof(double *));
    h->wr = (double **)xcalloc((size_t)h->nlev, sizeof(double *));
    for (int l = 0; l < h->nlev; ++l) {
        h->wb[l] = (double *)xcalloc((size_t)h->A[l].nr, sizeof(double));
        h->wx[l] = (double *)xcalloc((size_t)h->A[l].nr, sizeof(double));
        h->wr[l] = (double *)xcalloc((size_t)h->A[l].nr, sizeof(double));
    }
    if (status == ORC_OK) {
        if (nc > MAX_DENSE) status = ORC_ERR_UNSUPPORTED;
        else {
            h->lu = (double *)xcalloc((size_t)nc * nc, sizeof(double));
            h->piv = (int *)xcalloc((size_t)nc, sizeof(int));
            const Csr *c = &h->A[k];
            for (int i = 0; i < nc; ++i)
                for (int p = c->rp[i]; p < c->rp[i + 1]; ++p) h->lu[(long)i * nc + c->ci[p]] = c->v[p];
            status = lu_factor(nc, h->lu, h->piv);
        }
    }
    return status;
}

/* L1 diagonal of level k (a_ii + sum_{j != i} |a_ij|); status if not positive. */
static int amg_l1_diag(Amg *h, int k) {
    const Csr *a = &h->A[k];
    int n = a->nr, status = ORC_OK;
    h->dl1[k] = (double *)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(double));
    for (int i = 0; i < n; ++i) {
        double s = 0.0, aii = 0.0;
        for (int q = a->rp[i]; q < a->rp[i + 1]; ++q) {
            if (a->ci[q] == i) aii = a->v[q];
            else s += fabs(a->v[q]);
        }
        h->dl1[k][i] = aii + s;
        if (!(h->dl1[k][i] > 0.0)) status = ORC_ERR_UNSUPPORTED;
    }
    if (h->smoother == AMG_SMOOTH_HYBRID_GS) {
        /* the hybrid smoother's l1 term covers only the entries outside the row's chunk */
        h->dgs[k] = (double *)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(double));
        for (int i = 0; i < n; ++i) {
            int c0 = i / h->chunk * h->chunk, c1 = c0 + h->chunk;
            double s = 0.0, aii = 0.0;
            for (int q = a->rp[i]; q < a->rp[i + 1]; ++q) {
                int j = a->ci[q];
                if (j == i) aii = a->v[q];
                else if (j < c0 || j >= c1) s += fabs(a->v[q]);
            }
            h->dgs[k][i] = aii + s;
            if (!(h->dgs[k][i] > 0.0)) status = ORC_ERR_UNSUPPORTED;
        }
    }
    return status;
}

/* Setup reuse across value updates of one sparsity pattern: the C/F splits,
 * labels and interpolation operators of `old` are kept; every Galerkin product
 * A_{k+1} = P^T (A_k P), L1 diagonal and the coarsest factorisation are formed
 * again from the new level-0 matrix a0. */
static int amg_reuse(const Csr *a0, const Amg *old, Amg **out) {
    Amg *h = (Amg *)xcalloc(1, sizeof(Amg));
    h->nu_pre = old->nu_pre; h->nu_post = old->nu_post;
    h->smoother = old->smoother; h->chunk = old->chunk;
    h->A[0] = csr_copy(a0);
    int status = ORC_OK, k = 0;
    if (old->label[0]) {
        h->label[0] = (int *)xmalloc((size_t)a0->nr * sizeof(int));
        memcpy(h->label[0], old->label[0], (size_t)a0->nr * sizeof(int));
    }
    if (a0->nr != old->A[0].nr) status = ORC_ERR_ARG;
    for (; status == ORC_OK && k + 1 < old->nlev; ++k) {
        int n = h->A[k].nr, nc = old->P[k].nc;
        h->cf[k] = (int *)xmalloc((size_t)n * sizeof(int));
        memcpy(h->cf[k], old->cf[k], (size_t)n * sizeof(int));
        h->P[k] = csr_copy(&old->P[k]);
        h->R[k] = csr_copy(&old->R[k]);
        Csr ap = csr_spgemm(&h->A[k], &h->P[k]);
        h->A[k + 1] = csr_spgemm(&h->R[k], &ap);
        csr_free(&ap);
        if (old->label[k + 1]) {
            h->label[k + 1] = (int *)xmalloc((size_t)nc * sizeof(int));
            memcpy(h->label[k + 1], old->label[k + 1], (size_t)nc * sizeof(int));
        }
        int st = amg_l1_diag(h, k);
        if (st != ORC_OK) status = st;
    }
    *out = h;
    return amg_finish(h, k, status);
}

/* An independent copy of a whole hierarchy (kept as is when its matrix does
 * not change). */
static Amg *amg_clone(const Amg *old) {
    Amg *h = (Amg *)xcalloc(1, sizeof(Amg));
    h->nu_pre = old->nu_pre; h->nu_post = old->nu_post;
    h->smoother = old->smoother; h->chunk = old->chunk;
    h->nlev = old->nlev; h->nc = old->nc;
    for (int k = 0; k < old->nlev; ++k) {
        int n = old->A[k].nr;
        h->A[k] = csr_copy(&old->A[k]);
        h->AT[k] = csr_copy(&old->AT[k]);
        if (old->label[k]) {
            h->label[k] = (int *)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(int));
            memcpy(h->label[k], old->label[k], (size_t)n * sizeof(int));
        }
        if (k + 1 < old->nlev) {
            h->P[k] = csr_copy(&old->P[k]);
            h->R[k] = csr_copy(&old->R[k]);
            h->cf[k] = (int *)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(int));
            memcpy(h->cf[k], old->cf[k], (size_t)n * sizeof(int));
            h->dl1[k] = (double *)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(double));
            memcpy(h->dl1[k], old->dl1[k], (size_t)n * sizeof(double));
            if (old->dgs[k]) {
                h->dgs[k] = (double *)xmalloc((size_t)(n > 0 ? n : 1) * sizeof(double));
                memcpy(h->dgs[k], old->dgs[k], (size_t)n * sizeof(double));
            }
        }
    }
    h->wb = (double **)xcalloc((size_t)h->nlev, sizeof(double *));
    h->wx = (double **)xcalloc((size_t)h->nlev, sizeof(double *));
    h->wr = (double **)xcalloc((size_t)h->nlev, sizeof(double *));
    for (int l = 0; l < h->nlev; ++l) {
        h->wb[l] = (double *)xcalloc((size_t)h->A[l].nr + 1, sizeof(double));
        h->wx[l] = (double *)xcalloc((size_t)h->A[l].nr + 1, sizeof(double));
        h->wr[l] = (double *)xcalloc((size_t)h->A[l].nr + 1, sizeof(double));
    }
    if (old->lu) {
        h->lu = (double *)xmalloc((size_t)old->nc * old->nc * sizeof(double));
        memcpy(h->lu, old->lu, (size_t)old->nc * old->nc * sizeof(double));
        h->piv = (int *)xmalloc((size_t)old->nc * sizeof(int));
        memcpy(h->piv, old->piv, (size_t)old->nc * sizeof(int));
    }
    return h;
}

/* One L1-Jacobi sweep x <- x + D_l1^{-1} (b - A x) (Baker et al. 2011); the
 * transposed cycle uses A^T but the same row-based D_l1. */
static void l1_sweep(const Csr *a, const double *d, const double *b, double *x, double *r) {
    csr_residual(a, b, x, r);
    #pragma omp parallel for schedule(static) if (PAR_OK(a->nr))
    for (int i = 0; i < a->nr; ++i) x[i] += r[i] / d[i];
}

/* One sweep of hybrid L1 Gauss-Seidel (Baker, Falgout, Kolev, Yang, SIAM J.
 * Sci. Comput. 33 (2011)), the smoother of the paper's AMG settings (Sec. 4.1),
 * with chunks of `chunk` consecutive rows in place of the processors' row
 * blocks: inside a chunk the rows are relaxed one after another, in increasing
 * order (forward) or decreasing order (backward), each with the values this
 * sweep already gave the chunk's earlier rows and the previous values of every
 * other unknown; the diagonal d_i is a_ii plus the l1 norm of row i's entries
 * outside its chunk.  With chunk = 1 this is the L1-Jacobi sweep; with one
 * chunk, sequential Gauss-Seidel.  xold: scratch of n entries. */
static void hgs_sweep(const Csr *a, const double *d, int chunk, const double *b, double *x, double *xold,
                      int backward) {
    int n = a->nr;
    memcpy(xold, x, (size_t)n * sizeof(double));
    int nch = (n + chunk - 1) / chunk;
    #pragma omp parallel for schedule(static) if (PAR_OK(n))
    for (int c = 0; c < nch; ++c) {
        int c0 = c * chunk, c1 = c0 + chunk < n ? c0 + chunk : n;
        for (int t = 0; t < c1 - c0; ++t) {
            int i = backward ? c1 - 1 - t : c0 + t;
            double s = 0.0;
            for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) {
                int j = a->ci[p];
                int fresh = backward ? (j > i && j < c1) : (j >= c0 && j < i);
                s += a->v[p] * (fresh ? x[j] : xold[j]);
            }
            x[i] = xold[i] + (b[i] - s) / d[i];
        }
    }
}

/* Pre-smoothing (post = 0: L1-Jacobi, or forward hybrid Gauss-Seidel) and
 * post-smoothing (post = 1: L1-Jacobi, or backward hybrid Gauss-Seidel) on
 * level k; the transposed cycle passes A^T with the same row-based diagonals
 * and the same directions (the transpose of a backward sweep on A is a forward
 * sweep on A^T). */
static void amg_smooth(const Amg *h, int k, const Csr *a, const double *b, double *x, double *r, int post) {
    if (h->smoother == AMG_SMOOTH_HYBRID_GS) hgs_sweep(a, h->dgs[k], h->chunk, b, x, r, post);
    else l1_sweep(a, h->dl1[k], b, x, r);
}

/* V(nu_pre, nu_post) cycle from a zero initial guess.  trans = 1 applies the
 * exact transpose: A^T on every level, sweep counts swapped, coarse LU^T. */
static void amg_vcycle(Amg *h, int k, const double *b, double *x, int trans) {
    const Csr *a = trans ? &h->AT[k] : &h->A[k];
    int n = a->nr;
    if (k == h->nlev - 1) { lu_solve(n, h->lu, h->piv, b, x, trans); return; }
    int npre = trans ? h->nu_post : h->nu_pre, npost = trans ? h->nu_pre : h->nu_post;
    double *r = h->wr[k];
    #pragma omp parallel for schedule(static) if (PAR_OK(n))
    for (int i = 0; i < n; ++i) x[i] = 0.0;
    for (int s = 0; s < npre; ++s) amg_smooth(h, k, a, b, x, r, 0);
    csr_residual(a, b, x, r);
    double *bc = h->wb[k + 1], *xc = h->wx[k + 1];
    csr_matvec(&h->R[k], r, bc);
    amg_vcycle(h, k + 1, bc, xc, trans);
    const Csr *p = &h->P[k];
    #pragma omp parallel for schedule(static) if (PAR_OK(n))
    for (int i = 0; i < n; ++i) {
        double s = 0.0;
        for (int q = p->rp[i]; q < p->rp[i + 1]; ++q) s += p->v[q] * xc[p->ci[q]];
        x[i] += s;
    }
    for (int s = 0; s < npost; ++s) amg_smooth(h, k, a, b, x, r, 1);
}

/* ------------------------------------------------------------------------- */
/* MGR hierarchy (Sec. 2) and its application (Algorithm 1).                  */
/* ------------------------------------------------------------------------- */
typedef struct {
    int n, nF, nC;
    int *isF, *fmap, *cmap, *lmap;   /* lmap: global -> local F or C index    */
    int *field;                      /* field label of each point             */
    Csr A, AT;                       /* level operator and its transpose      */
    Csr AFF, AFC, ACF, ACC;
    Csr MF;                          /* F-relaxation operator M_FF^{-1} as CSR (Jacobi / block-Jacobi) */
    Csr PF, RF;                      /* P = [PF; I], R = [RF, I] (RF empty for injection) */
    Csr PFT, RFT, AFFT, ACFT, MFT;   /* explicit transposes for the transposed apply */
    int frelax, sweeps, restrict_type;
    double omega;
    Amg *famg;                       /* F-relaxation by one AMG V-cycle       */
    double *ilu;                     /* ILU(0) factors on the pattern of A_FF  */
    int *ilu_diag;
} MgrLevel;

typedef struct {
    int nlev;                        /* number of MGR reduction levels        */
    int b, nbr;                      /* block layout of the input             */
    MgrLevel L[MAX_MGR_LEVELS];
    Amg *camg;                       /* AMG on the final coarse system        */
    Csr Acoarse;                     /* final coarse operator                 */
    int *coarse_field;
    double **wv, **wz, **wr, **wt;   /* per-level work vectors               */
} Mgr;

/* ILU(0) on the pattern of A_FF (Saad, Iterative Methods, Alg. 10.4), in the
 * natural row order; values stored on A_FF's pattern. */
static int ilu0_factor(const Csr *a, double **lu_out, int **diag_out) {
    int n = a->nr;
    long nnz = csr_nnz(a);
    double *lu = (double *)xmalloc((size_t)(nnz > 0 ? nnz : 1) * sizeof(double));
    memcpy(lu, a->v, (size_t)nnz * sizeof(double));
    int *diag = (int *)xmalloc((size_t)n * sizeof(int));
    int *pos = (int *)xmalloc((size_t)n * sizeof(int));
    for (int j = 0; j < n; ++j) pos[j] = -1;
    int status = ORC_OK;
    for (int i = 0; i < n; ++i) {
        diag[i] = -1;
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) { pos[a->ci[p]] = p; if (a->ci[p] == i) diag[i] = p; }
        if (diag[i] < 0) { status = ORC_ERR_ZERO_PIVOT; }
        for (int p = a->rp[i]; p < a->rp[i + 1] && a->ci[p] < i; ++p) {
            int k = a->ci[p];
            if (diag[k] < 0 || lu[diag[k]] == 0.0) { status = ORC_ERR_ZERO_PIVOT; continue; }
            double l = lu[p] / lu[diag[k]];
            lu[p] = l;
            for (int q = diag[k] + 1; q < a->rp[k + 1]; ++q) {
                int j = a->ci[q];
                if (pos[j] >= 0) lu[pos[j]] -= l * lu[q];
            }
        }
        for (int p = a->rp[i]; p < a->rp[i + 1]; ++p) pos[a->ci[p]] = -1;
        if (diag[i] >= 0 && (lu[diag[i]] == 0.0 || !isfinite(lu[diag[i]]))) status = ORC_ERR_ZERO_PIVOT;
    }
    free(pos);
    *lu_out = lu; *diag_out = diag;
    return status;
}

/* z = (LU)^{-1} r, or (LU)^{-T} r when trans. */
static void ilu0_solve(const Csr *a, const double *lu, const int *diag, const double *r, double *z, int trans) {
    int n = a->nr;
    if (!trans) {
        for (int i = 0; i < n; ++i) {
            double s = r[i];
            for (int p = a->rp[i]; p < diag[i]; ++p) s -= lu[p] * z[a->ci[p]];
            z[i] = s;
        }
        for (int i = n - 1; i >= 0; --i) {
            double s = z[i];
            for (int p = diag[i] + 1; p < a->rp[i + 1]; ++p) s -= lu[p] * z[a->ci[p]];
            z[i] = s / lu[diag[i]];
        }
    } else {
        /* (LU)^T = U^T L^T: solve U^T y = r (column sweep), then L^T z = y. */
        for (int i = 0; i < n; ++i) z[i] = r[i];
        for (int i = 0; i < n; ++i) {
            z[i] = z[i] / lu[diag[i]];
            for (int p = diag[i] + 1; p < a->rp[i + 1]; ++p) z[a->ci[p]] -= lu[p] * z[i];
        }
        for (int i = n - 1; i >= 0; --i)
            for (int p = a->rp[i]; p < diag[i]; ++p) z[a->ci[p]] -= lu[p] * z[i];
    }
}

static void mgr_level_free(MgrLevel *l) {
    free(l->isF); free(l->fmap); free(l->cmap); free(l->lmap); free(l->field);
    csr_free(&l->A); csr_free(&l->AT);
    csr_free(&l->AFF); csr_free(&l->AFC); csr_free(&l->ACF); csr_free(&l->ACC);
    csr_free(&l->MF); csr_free(&l->PF); csr_free(&l->RF);
    csr_free(&l->PFT); csr_free(&l->RFT); csr_free(&l->AFFT); csr_free(&l->ACFT); csr_free(&l->MFT);
    amg_free(l->famg);
    free(l->ilu); free(l->ilu_diag);
}

static void mgr_free(Mgr *m) {
    if (!m) return;
    for (int l = 0; l < m->nlev; ++l) mgr_level_free(&m->L[l]);
    amg_free(m->camg);
    csr_free(&m->Acoarse);
    free(m->coarse_field);
    if (m->wv) for (int l = 0; l <= m->nlev; ++l) { free(m->wv[l]); free(m->wz[l]); free(m->wr[l]); free(m->wt[l]); }
    free(m->wv); free(m->wz); free(m->wr); free(m->wt);
    free(m);
}

/* The F-relaxation operator as a CSR on the F-local numbering:
 *  Jacobi: diag(A_FF)^{-1};  block-Jacobi: inverse of each diagonal block of
 *  A_FF formed by the F-points that share one block row of the input layout. */
static int build_frelax_operator(MgrLevel *l, int bsize, const int *global_block) {
    int nF = l->nF;
    Csr *a = &l->AFF;
    if (l->frelax == FRELAX_JACOBI) {
        l->MF = csr_alloc(nF, nF, nF);
        for (int k = 0; k < nF; ++k) {
            double d = 0.0;
            for (int p = a->rp[k]; p < a->rp[k + 1]; ++p) if (a->ci[p] == k) d = a->v[p];
            if (d == 0.0 || !isfinite(d)) return ORC_ERR_ZERO_PIVOT;
            l->MF.rp[k + 1] = k + 1;
            l->MF.ci[k] = k;
            l->MF.v[k] = 1.0 / d;
        }
        return ORC_OK;
    }
    if (l->frelax == FRELAX_BLOCK_JACOBI) {
        /* blocks = maximal runs of consecutive F-points with equal block id */
        int *bstart = (int *)xmalloc((size_t)(nF + 1) * sizeof(int));
        int nb = 0;
        for (int k = 0; k < nF; ++k)
            if (k == 0 || global_block[l->fmap[k]] != global_block[l->fmap[k - 1]]) bstart[nb++] = k;
        bstart[nb] = nF;
        long nnz = 0;
        for (int t = 0; t < nb; ++t) { long s = bstart[t + 1] - bstart[t]; nnz += s * s; }
        l->MF = csr_alloc(nF, nF, nnz);
        long o = 0;
        int status = ORC_OK;
        (void)bsize;
        for (int t = 0; t < nb; ++t) {
            int s0 = bstart[t], bs = bstart[t + 1] - bstart[t];
            if (bs > 4) { status = ORC_ERR_UNSUPPORTED; break; }
            double blk[16], inv[16];
            for (int r = 0; r < bs; ++r)
                for (int c = 0; c < bs; ++c) {
                    double v = 0.0;
                    for (int p = a->rp[s0 + r]; p < a->rp[s0 + r + 1]; ++p) if (a->ci[p] == s0 + c) v = a->v[p];
                    blk[r * bs + c] = v;
                }
            int st = small_inverse(bs, blk, inv);
            if (st != ORC_OK) { status = st; break; }
            for (int r = 0; r < bs; ++r) {
                for (int c = 0; c < bs; ++c) { l->MF.ci[o] = s0 + c; l->MF.v[o] = inv[r * bs + c]; o++; }
                l->MF.rp[s0 + r + 1] = (int)o;
            }
        }
        free(bstart);
        return status;
    }
    return ORC_OK;
}

typedef struct {
    int frelax, sweeps, restrict_type, amg_unknown_based, amg_agg_levels;
    double omega;
    unsigned fmask;
} LevelOpts;

/* One MGR reduction level (Sec. 2): split by field, extract blocks, F-operator,
 * P = [-M A_FC; I] (eq. (4); with M = D^{-1} it is Jacobi interpolation and it
 * equals the ideal P of eq. (3) whenever A_FF is diagonal), R = [0 I] or
 * [-A_CF M, I] (eq. (5)), and the Petrov-Galerkin coarse operator
 *   A_c = R A P = A_CC + A_CF P_F + R_F A_FC + R_F (A_FF P_F),
 * summed in that order. */
static int mgr_setup_level(MgrLevel *l, const Csr *a, const int *field, const LevelOpts *lo, int bsize,
                           const int *global_block, const AmgOpts *ao, uint64_t amg_seed, const Amg *famg_old,
                           int keep_famg) {
    int n = a->nr;
    l->n = n;
    l->A = csr_copy(a);
    l->AT = csr_transpose(a);
    l->field = (int *)xmalloc((size_t)n * sizeof(int));
    memcpy(l->field, field, (size_t)n * sizeof(int));
    l->frelax = lo->frelax; l->sweeps = lo->sweeps; l->omega = lo->omega; l->restrict_type = lo->restrict_type;
    l->isF = (int *)xmalloc((size_t)n * sizeof(int));
    l->lmap = (int *)xmalloc((size_t)n * sizeof(int));
    int nF = 0, nC = 0;
    for (int i = 0; i < n; ++i) {
        if (field[i] < 0 || field[i] >= 32) return ORC_ERR_BAD_LABELS;
        l->isF[i] = (int)((lo->fmask >> field[i]) & 1u);
        if (l->isF[i]) l->lmap[i] = nF++; else l->lmap[i] = nC++;
    }
    if (nF == 0 || nC == 0) return ORC_ERR_BAD_LABELS;
    l->nF = nF; l->nC = nC;
    l->fmap = (int *)xmalloc((size_t)nF * sizeof(int));
    l->cmap = (int *)xmalloc((size_t)nC * sizeof(int));
    int *fcol = (int *)xmalloc((size_t)n * sizeof(int));
    int *ccol = (int *)xmalloc((size_t)n * sizeof(int));
    for (int i = 0; i < n; ++i) {
        if (l->isF[i]) { l->fmap[l->lmap[i]] = i; fcol[i] = l->lmap[i]; ccol[i] = -1; }
        else { l->cmap[l->lmap[i]] = i; ccol[i] = l->lmap[i]; fcol[i] = -1; }
    }
    l->AFF = csr_extract(a, l->fmap, nF, fcol, nF);
    l->AFC = csr_extract(a, l->fmap, nF, ccol, nC);
    l->ACF = csr_extract(a, l->cmap, nC, fcol, nF);
    l->ACC = csr_extract(a, l->cmap, nC, ccol, nC);
    free(fcol); free(ccol);

    int status = ORC_OK;
    if (l->frelax == FRELAX_JACOBI || l->frelax == FRELAX_BLOCK_JACOBI) {
        status = build_frelax_operator(l, bsize, global_block);
        if (status != ORC_OK) return status;
    } else {
        /* ILU(0) and AMG F-relaxation still use Jacobi interpolation (eq. (4)) */
        MgrLevel tmp = *l;
        tmp.frelax = FRELAX_JACOBI;
        status = build_frelax_operator(&tmp, bsize, global_block);
        l->MF = tmp.MF;
        if (status != ORC_OK) return status;
        if (l->frelax == FRELAX_ILU0) {
            status = ilu0_factor(&l->AFF, &l->ilu, &l->ilu_diag);
            if (status != ORC_OK) return status;
        } else if (l->frelax == FRELAX_AMG) {
            int *flab = (int *)xmalloc((size_t)nF * sizeof(int));
            for (int k = 0; k < nF; ++k) flab[k] = field[l->fmap[k]];
            /* the AMG operator: A_FF, or its separate-component approximation
             * (amg_unknown_based == 2: the couplings between unknowns of
             * different fields dropped, Sec. 4.4) */
            Csr aop = lo->amg_unknown_based == 2 ? csr_same_label(&l->AFF, flab) : csr_copy(&l->AFF);
            if (famg_old && keep_famg) {
                /* A_FF unchanged (the mechanics block between Newton solves, Sec. 3.3) */
                l->famg = amg_clone(famg_old);
            } else if (famg_old) {
                status = amg_reuse(&aop, famg_old, &l->famg);
            } else {
                AmgOpts fo = *ao;
                fo.unknown_based = lo->amg_unknown_based != 0;
                fo.agg_levels = lo->amg_agg_levels;
                fo.seed = amg_seed;
                status = amg_setup(&aop, flab, &fo, &l->famg);
            }
            csr_free(&aop);
            free(flab);
            if (status != ORC_OK) return status;
        } else {
            return ORC_ERR_ARG;
        }
    }
    l->PF = csr_spgemm(&l->MF, &l->AFC);
    csr_negate(&l->PF);
    if (l->restrict_type == RESTRICT_JACOBI) {
        l->RF = csr_spgemm(&l->ACF, &l->MF);
        csr_negate(&l->RF);
    }
    l->PFT = csr_transpose(&l->PF);
    l->AFFT = csr_transpose(&l->AFF);
    l->ACFT = csr_transpose(&l->ACF);
    l->MFT = csr_transpose(&l->MF);
    if (l->restrict_type == RESTRICT_JACOBI) l->RFT = csr_transpose(&l->RF);
    return ORC_OK;
}

static void mgr_coarse_product(const MgrLevel *l, Csr *out) {
    Csr t1 = csr_spgemm(&l->ACF, &l->PF);
    Csr ac = csr_add(&l->ACC, &t1);
    csr_free(&t1);
    if (l->restrict_type == RESTRICT_JACOBI) {
        Csr t2 = csr_spgemm(&l->RF, &l->AFC);
        Csr s2 = csr_add(&ac, &t2);
        csr_free(&ac); csr_free(&t2);
        Csr ffp = csr_spgemm(&l->AFF, &l->PF);
        Csr t3 = csr_spgemm(&l->RF, &ffp);
        csr_free(&ffp);
        ac = csr_add(&s2, &t3);
        csr_free(&s2); csr_free(&t3);
    }
    *out = ac;
}

/* z_F = M_FF^{-1} r_F for the level's F-relaxation (trans: M_FF^{-T}). */
static void frelax_solve(MgrLevel *l, const double *rF, double *zF, int trans) {
    if (l->frelax == FRELAX_JACOBI || l->frelax == FRELAX_BLOCK_JACOBI) {
        csr_matvec(trans ? &l->MFT : &l->MF, rF, zF);
    } else if (l->frelax == FRELAX_ILU0) {
        ilu0_solve(&l->AFF, l->ilu, l->ilu_diag, rF, zF, trans);
    } else {
        amg_vcycle(l->famg, 0, rF, zF, trans);
    }
}

/* Algorithm 1 from z = 0 with no global relaxation (the paper needs none):
 *   repeat nu times: z <- z + Q^T (omega M_FF^{-1}) Q (v - A z)      (F-relaxation)
 *   r_c = R (v - A z)                                              (restriction)
 *   e_c = next level, or the AMG V-cycle on the last coarse system  (recursion)
 *   z <- z + P e_c                                                 (interpolation + correction) */
static void mgr_vcycle(Mgr *m, int lev, const double *v, double *z) {
    if (lev == m->nlev) { amg_vcycle(m->camg, 0, v, z, 0); return; }
    MgrLevel *l = &m->L[lev];
    int n = l->n, nF = l->nF, nC = l->nC;
    double *r = m->wr[lev], *t = m->wt[lev];
    double *rF = t, *zF = t + nF;  /* scratch split: rF[nF], zF[nF] */
    #pragma omp parallel for schedule(static) if (PAR_OK(n))
    for (int i = 0; i < n; ++i) z[i] = 0.0;
    for (int s = 0; s < l->sweeps; ++s) {
        csr_residual(&l->A, v, z, r);
        #pragma omp parallel for schedule(static) if (PAR_OK(nF))
        for (int k = 0; k < nF; ++k) rF[k] = r[l->fmap[k]];
        frelax_solve(l, rF, zF, 0);
        #pragma omp parallel for schedule(static) if (PAR_OK(nF))
        for (int k = 0; k < nF; ++k) z[l->fmap[k]] += l->omega * zF[k];
    }
    csr_residual(&l->A, v, z, r);
    double *rc = m->wv[lev + 1], *ec = m->wz[lev + 1];
    #pragma omp parallel for schedule(static) if (PAR_OK(nC))
    for (int i = 0; i < nC; ++i) rc[i] = r[l->cmap[i]];
    if (l->restrict_type == RESTRICT_JACOBI) {
        #pragma omp parallel for schedule(static) if (PAR_OK(nF))
        for (int k = 0; k < nF; ++k) rF[k] = r[l->fmap[k]];
        #pragma omp parallel for schedule(static) if (PAR_OK(nC))
        for (int i = 0; i < nC; ++i) {
            double s = 0.0;
            for (int p = l->RF.rp[i]; p < l->RF.rp[i + 1]; ++p) s += l->RF.v[p] * rF[l->RF.ci[p]];
            rc[i] += s;
        }
    }
    mgr_vcycle(m, lev + 1, rc, ec);
    #pragma omp parallel for schedule(static) if (PAR_OK(nF))
    for (int k = 0; k < nF; ++k) {
        double s = 0.0;
        for (int p = l->PF.rp[k]; p < l->PF.rp[k + 1]; ++p) s += l->PF.v[p] * ec[l->PF.ci[p]];
        z[l->fmap[k]] += s;
    }
    #pragma omp parallel for schedule(static) if (PAR_OK(nC))
    for (int i = 0; i < nC; ++i) z[l->cmap[i]] += ec[i];
}

/* Exact transpose of the one-sweep cycle above.  With M_F = omega M_FF^{-1},
 *   M^{-1} = Q^T M_F Q + P C R (I - A Q^T M_F Q), hence
 *   M^{-T} v:  u_c = P^T v;  e = C^T u_c;  y = R^T e;
 *              z_F = y_F + M_F^T (v_F - (A^T y)_F);  z_C = e. */
static void mgr_vcycle_t(Mgr *m, int lev, const double *v, double *z) {
    if (lev == m->nlev) { amg_vcycle(m->camg, 0, v, z, 1); return; }
    MgrLevel *l = &m->L[lev];
    int nF = l->nF, nC = l->nC;
    double *t = m->wt[lev];
    double *tF = t, *zF = t + nF;
    double *uc = m->wv[lev + 1], *ec = m->wz[lev + 1];
    #pragma omp parallel for schedule(static) if (PAR_OK(nC))
    for (int i = 0; i < nC; ++i) {
        double s = 0.0;
        for (int p = l->PFT.rp[i]; p < l->PFT.rp[i + 1]; ++p) s += l->PFT.v[p] * v[l->fmap[l->PFT.ci[p]]];
        uc[i] = v[l->cmap[i]] + s;
    }
    mgr_vcycle_t(m, lev + 1, uc, ec);
    double *yF = m->wr[lev];  /* y_F = R_F^T e (zero for injection) */
    #pragma omp parallel for schedule(static) if (PAR_OK(nF))
    for (int k = 0; k < nF; ++k) {
        double s = 0.0;
        if (l->restrict_type == RESTRICT_JACOBI)
            for (int p = l->RFT.rp[k]; p < l->RFT.rp[k + 1]; ++p) s += l->RFT.v[p] * ec[l->RFT.ci[p]];
        yF[k] = s;
    }
    #pragma omp parallel for schedule(static) if (PAR_OK(nF))
    for (int k = 0; k < nF; ++k) {
        double s = 0.0;
        for (int p = l->AFFT.rp[k]; p < l->AFFT.rp[k + 1]; ++p) s += l->AFFT.v[p] * yF[l->AFFT.ci[p]];
        for (int p = l->ACFT.rp[k]; p < l->ACFT.rp[k + 1]; ++p) s += l->ACFT.v[p] * ec[l->ACFT.ci[p]];
        tF[k] = v[l->fmap[k]] - s;
    }
    frelax_solve(l, tF, zF, 1);
    #pragma omp parallel for schedule(static) if (PAR_OK(nF))
    for (int k = 0; k < nF; ++k) z[l->fmap[k]] = yF[k] + l->omega * zF[k];
    #pragma omp parallel for schedule(static) if (PAR_OK(nC))
    for (int i = 0; i < nC; ++i) z[l->cmap[i]] = ec[i];
}

/* ------------------------------------------------------------------------- */
/* Flexible GMRES(m) with right preconditioning (Saad, SISC 14 (1993)).        */
/* ------------------------------------------------------------------------- */
typedef void (*op_fn)(void *ctx, const double *x, double *y);

typedef struct {
    int iterations, restarts, status;
    double rel_res_est, rel_res_true;
} SolveInfo;

static void fgmres(int n, op_fn matvec, op_fn prec, void *ctx, const double *b, double *x, int m, int maxiter,
                   double rtol, int mgs, SolveInfo *info) {
    memset(info, 0, sizeof(*info));
    #pragma omp parallel for schedule(static) if (PAR_OK(n))
    for (int i = 0; i < n; ++i) x[i] = 0.0;
    double bnorm = nrm2(n, b);
    if (bnorm == 0.0) { info->status = ORC_OK; return; }
    double *V = (double *)xmalloc((size_t)(m + 1) * n * sizeof(double));
    double *Z = (double *)xmalloc((size_t)m * n * sizeof(double));
    double *w = (double *)xmalloc((size_t)n * sizeof(double));
    double *H = (double *)xcalloc((size_t)(m + 1) * m, sizeof(double));   /* H[i*m + j] */
    double *cs = (double *)xcalloc((size_t)m, sizeof(double));
    double *sn = (double *)xcalloc((size_t)m, sizeof(double));
    double *g = (double *)xcalloc((size_t)m + 1, sizeof(double));
    double *y = (double *)xcalloc((size_t)m, sizeof(double));
    double *hp = (double *)xcalloc((size_t)m + 1, sizeof(double));
    int iters = 0, converged = 0;
    double est = 1.0, truer = 1.0;
    for (int cycle = 0;; ++cycle) {
        /* r = b - A x */
        matvec(ctx, x, w);
        #pragma omp parallel for schedule(static) if (PAR_OK(n))
        for (int i = 0; i < n; ++i) V[i] = b[i] - w[i];
        double beta = nrm2(n, V);
        if (beta <= rtol * bnorm) { converged = 1; est = beta / bnorm; truer = est; break; }
        if (cycle > 0) info->restarts++;
        #pragma omp parallel for schedule(static) if (PAR_OK(n))
        for (int i = 0; i < n; ++i) V[i] /= beta;
        memset(g, 0, (size_t)(m + 1) * sizeof(double));
        memset(H, 0, (size_t)(m + 1) * m * sizeof(double));
        g[0] = beta;
        int k = 0;
        for (int j = 0; j < m; ++j) {
            double *vj = V + (size_t)j * n, *zj = Z + (size_t)j * n;
            prec(ctx, vj, zj);
            matvec(ctx, zj, w);
            for (int i = 0; i <= j; ++i) H[i * m + j] = 0.0;
            if (mgs) {
                for (int i = 0; i <= j; ++i) {
                    double h = dot(n, V + (size_t)i * n, w);
                    H[i * m + j] += h;
                    #pragma omp parallel for schedule(static) if (PAR_OK(n))
                    for (int q = 0; q < n; ++q) w[q] -= h * V[(size_t)i * n + q];
                }
            } else {
                for (int pass = 0; pass < 2; ++pass) {           /* classical Gram-Schmidt, twice */
                    for (int i = 0; i <= j; ++i) hp[i] = dot(n, V + (size_t)i * n, w);
                    #pragma omp parallel for schedule(static) if (PAR_OK(n))
                    for (int q = 0; q < n; ++q) {
                        double s = 0.0;
                        for (int i = 0; i <= j; ++i) s += hp[i] * V[(size_t)i * n + q];
                        w[q] -= s;
                    }
                    for (int i = 0; i <= j; ++i) H[i * m + j] += hp[i];
                }
            }
            double hn = nrm2(n, w);
            H[(j + 1) * m + j] = hn;
            for (int i = 0; i < j; ++i) {                        /* previous rotations */
                double a0 = H[i * m + j], a1 = H[(i + 1) * m + j];
                H[i * m + j] = cs[i] * a0 + sn[i] * a1;
                H[(i + 1) * m + j] = -sn[i] * a0 + cs[i] * a1;
            }
            double a0 = H[j * m + j], a1 = H[(j + 1) * m + j];
            double den = sqrt(a0 * a0 + a1 * a1);
            if (den == 0.0) { cs[j] = 1.0; sn[j] = 0.0; }
            else { cs[j] = a0 / den; sn[j] = a1 / den; }
            H[j * m + j] = cs[j] * a0 + sn[j] * a1;
            H[(j + 1) * m + j] = 0.0;
            g[j + 1] = -sn[j] * g[j];
            g[j] = cs[j] * g[j];
            iters++;
            k = j + 1;
            est = fabs(g[j + 1]) / bnorm;
            if (hn == 0.0) break;                                /* lucky breakdown */
            double *vn = V + (size_t)(j + 1) * n;
            #pragma omp parallel for schedule(static) if (PAR_OK(n))
            for (int q = 0; q < n; ++q) vn[q] = w[q] / hn;
            if (fabs(g[j + 1]) <= rtol * bnorm || iters >= maxiter) break;
        }
        for (int i = k - 1; i >= 0; --i) {                       /* H y = g */
            double s = g[i];
            for (int q = i + 1; q < k; ++q) s -= H[i * m + q] * y[q];
            y[i] = s / H[i * m + i];
        }
        #pragma omp parallel for schedule(static) if (PAR_OK(n))
        for (int q = 0; q < n; ++q)
            for (int i = 0; i < k; ++i) x[q] += y[i] * Z[(size_t)i * n + q];
        matvec(ctx, x, w);
        #pragma omp parallel for schedule(static) if (PAR_OK(n))
        for (int q = 0; q < n; ++q) w[q] = b[q] - w[q];
        truer = nrm2(n, w) / bnorm;
        if (truer <= rtol) { converged = 1; break; }
        if (iters >= maxiter) break;
    }
    info->iterations = iters;
    info->rel_res_est = est;
    info->rel_res_true = truer;
    info->status = converged ? ORC_OK : ORC_NOT_CONVERGED;
    free(V); free(Z); free(w); free(H); free(cs); free(sn); free(g); free(y); free(hp);
}

/* ------------------------------------------------------------------------- */
/* Exported interface (used through ctypes by the tests).                      */
/* ------------------------------------------------------------------------- */
typedef struct {
    Mgr *mgr;
    Csr A0, A0T;          /* input operator (scalar) and transpose */
    int b, nbr;
    int trans_mode;
    int ortho;
} Handle;

static void h_matvec(void *ctx, const double *x, double *y) {
    Handle *h = (Handle *)ctx;
    csr_matvec(h->trans_mode ? &h->A0T : &h->A0, x, y);
}
static void h_prec(void *ctx, const double *x, double *y) {
    Handle *h = (Handle *)ctx;
    if (h->trans_mode) mgr_vcycle_t(h->mgr, 0, x, y);
    else mgr_vcycle(h->mgr, 0, x, y);
}

/* Build the oracle's MGR hierarchy.  Inputs: block-CSR (b = 1 is plain CSR),
 * the field label of every scalar unknown, per-level F-field bitmasks and
 * options, and the AMG options for the final coarse system. */
static void *setup_impl(int b, int nbr, const int *rp, const int *ci, const double *val, const int *field,
                        int nlevels, const unsigned *fmask, const int *frelax, const int *sweeps,
                        const double *omega, const int *restrict_type, const int *amg_unknown_based_lvl, const int *amg_agg_lvl,
                        double theta, int max_levels, int max_coarse, int nu_pre, int nu_post,
                        int coarse_unknown_based, int coarse_agg_levels, int interp, int smoother, int chunk, unsigned long long seed, const int *block_of_dof,
                        const void *reuse_from, int keep_famg, int *status);

void *orc_setup(int b, int nbr, const int *rp, const int *ci, const double *val, const int *field, int nlevels,
                const unsigned *fmask, const int *frelax, const int *sweeps, const double *omega,
                const int *restrict_type, const int *amg_unknown_based_lvl, const int *amg_agg_lvl, double theta, int max_levels,
                int max_coarse, int nu_pre, int nu_post, int coarse_unknown_based, int coarse_agg_levels, int interp, int smoother, int chunk, unsigned long long seed,
                const int *block_of_dof, int *status) {
    return setup_impl(b, nbr, rp, ci, val, field, nlevels, fmask, frelax, sweeps, omega, restrict_type,
                      amg_unknown_based_lvl, amg_agg_lvl, theta, max_levels, max_coarse, nu_pre, nu_post,
                      coarse_unknown_based, coarse_agg_levels,
                      interp, smoother, chunk, seed, block_of_dof, NULL, 0, status);
}

/* Setup reuse for new values on the same pattern (the AMG data reuse between
 * Newton solves of Sec. 3.3 and Sec. 4.4): the MGR levels are formed again; every AMG
 * hierarchy (the coarse one and those used as F-relaxation) keeps the C/F
 * splits and interpolation of `old` and forms its Galerkin products anew, or,
 * with keep_famg, the F-relaxation hierarchies are kept whole (their A_FF is
 * unchanged).  The other arguments must be those `old` was set up with. */
void *orc_update(const void *old, int b, int nbr, const int *rp, const int *ci, const double *val, const int *field,
                 int nlevels, const unsigned *fmask, const int *frelax, const int *sweeps, const double *omega,
                 const int *restrict_type, const int *amg_unknown_based_lvl, const int *amg_agg_lvl, double theta, int max_levels,
                 int max_coarse, int nu_pre, int nu_post, int coarse_unknown_based, int coarse_agg_levels, int interp, int smoother,
                 int chunk, unsigned long long seed, const int *block_of_dof, int keep_famg, int *status) {
    return setup_impl(b, nbr, rp, ci, val, field, nlevels, fmask, frelax, sweeps, omega, restrict_type,
                      amg_unknown_based_lvl, amg_agg_lvl, theta, max_levels, max_coarse, nu_pre, nu_post,
                      coarse_unknown_based, coarse_agg_levels,
                      interp, smoother, chunk, seed, block_of_dof, old, keep_famg, status);
}

static void *setup_impl(int b, int nbr, const int *rp, const int *ci, const double *val, const int *field,
                        int nlevels, const unsigned *fmask, const int *frelax, const int *sweeps,
                        const double *omega, const int *restrict_type, const int *amg_unknown_based_lvl, const int *amg_agg_lvl,
                        double theta, int max_levels, int max_coarse, int nu_pre, int nu_post,
                        int coarse_unknown_based, int coarse_agg_levels, int interp, int smoother, int chunk, unsigned long long seed, const int *block_of_dof,
                        const void *reuse_from, int keep_famg, int *status) {
    const Handle *old = (const Handle *)reuse_from;
    Handle *h = (Handle *)xcalloc(1, sizeof(Handle));
    h->b = b; h->nbr = nbr;
    h->A0 = bsr_expand(b, nbr, nbr, rp, ci, val);
    h->A0T = csr_transpose(&h->A0);
    int n = h->A0.nr;
    Mgr *m = (Mgr *)xcalloc(1, sizeof(Mgr));
    h->mgr = m;
    m->b = b; m->nbr = nbr;
    *status = ORC_OK;
    if (nlevels < 0 || nlevels > MAX_MGR_LEVELS) { *status = ORC_ERR_ARG; return h; }
    if (smoother != AMG_SMOOTH_L1_JACOBI && smoother != AMG_SMOOTH_HYBRID_GS) { *status = ORC_ERR_ARG; return h; }
    if (chunk < 1) { *status = ORC_ERR_ARG; return h; }
    if (coarse_agg_levels < 0) { *status = ORC_ERR_ARG; return h; }
    AmgOpts ao = {theta, max_levels, max_coarse, nu_pre, nu_post, coarse_unknown_based, interp, smoother, chunk,
                  coarse_agg_levels, (uint64_t)seed};
    /* block-Jacobi groups: the caller's group id of every unknown, else its block row */
    int *gblock = (int *)xmalloc((size_t)n * sizeof(int));
    for (int i = 0; i < n; ++i) gblock[i] = block_of_dof ? block_of_dof[i] : i / b;
    Csr cur = csr_copy(&h->A0);
    int *cfield = (int *)xmalloc((size_t)n * sizeof(int));
    memcpy(cfield, field, (size_t)n * sizeof(int));
    int *cblock = gblock;
    for (int lev = 0; lev < nlevels; ++lev) {
        LevelOpts lo = {frelax[lev], sweeps[lev], restrict_type[lev], amg_unknown_based_lvl[lev], amg_agg_lvl[lev],
                        omega[lev],
                        fmask[lev]};
        MgrLevel *l = &m->L[lev];
        m->nlev = lev + 1;
        const Amg *fold = (old && lev < old->mgr->nlev) ? old->mgr->L[lev].famg : NULL;
        int st = mgr_setup_level(l, &cur, cfield, &lo, b, cblock, &ao,
                                 (uint64_t)seed + 0x1000193ULL * (uint64_t)(lev + 1), fold, keep_famg);
        if (st != ORC_OK) { *status = st; break; }
        Csr ac;
        mgr_coarse_product(l, &ac);
        csr_free(&cur);
        cur = ac;
        int *nf = (int *)xmalloc((size_t)l->nC * sizeof(int));
        int *nb = (int *)xmalloc((size_t)l->nC * sizeof(int));
        for (int i = 0; i < l->nC; ++i) { nf[i] = cfield[l->cmap[i]]; nb[i] = cblock[l->cmap[i]]; }
        free(cfield);
        if (cblock != gblock) free(cblock);
        cfield = nf; cblock = nb;
    }
    if (cblock != gblock) free(cblock);
    free(gblock);
    m->Acoarse = cur;
    m->coarse_field = cfield;
    if (*status == ORC_OK) {
        int st = (old && old->mgr->camg) ? amg_reuse(&m->Acoarse, old->mgr->camg, &m->camg)
                                         : amg_setup(&m->Acoarse, cfield, &ao, &m->camg);
        if (st != ORC_OK) *status = st;
    }
    m->wv = (double **)xcalloc((size_t)m->nlev + 1, sizeof(double *));
    m->wz = (double **)xcalloc((size_t)m->nlev + 1, sizeof(double *));
    m->wr = (double **)xcalloc((size_t)m->nlev + 1, sizeof(double *));
    m->wt = (double **)xcalloc((size_t)m->nlev + 1, sizeof(double *));
    for (int l = 0; l <= m->nlev; ++l) {
        int sz = (l < m->nlev) ? m->L[l].n : m->Acoarse.nr;
        if (sz <= 0) sz = 1;
        m->wv[l] = (double *)xcalloc((size_t)sz, sizeof(double));
        m->wz[l] = (double *)xcalloc((size_t)sz, sizeof(double));
        m->wr[l] = (double *)xcalloc((size_t)sz, sizeof(double));
        m->wt[l] = (double *)xcalloc((size_t)2 * sz, sizeof(double));
    }
    return h;
}

void orc_free(void *hp) {
    Handle *h = (Handle *)hp;
    if (!h) return;
    mgr_free(h->mgr);
    csr_free(&h->A0); csr_free(&h->A0T);
    free(h);
}

int orc_apply(void *hp, const double *v, double *z, int trans) {
    Handle *h = (Handle *)hp;
    if (trans) {
        for (int l = 0; l < h->mgr->nlev; ++l)
            if (h->mgr->L[l].sweeps != 1) return ORC_ERR_UNSUPPORTED;
        mgr_vcycle_t(h->mgr, 0, v, z);
    } else {
        mgr_vcycle(h->mgr, 0, v, z);
    }
    return ORC_OK;
}

int orc_matvec(void *hp, const double *x, double *y, int trans) {
    Handle *h = (Handle *)hp;
    csr_matvec(trans ? &h->A0T : &h->A0, x, y);
    return ORC_OK;
}

int orc_solve(void *hp, int trans, const double *b, double *x, int restart, int maxiter, double rtol, int mgs,
              int *iterations, int *restarts, double *est, double *truer) {
    Handle *h = (Handle *)hp;
    if (trans)
        for (int l = 0; l < h->mgr->nlev; ++l)
            if (h->mgr->L[l].sweeps != 1) return ORC_ERR_UNSUPPORTED;
    h->trans_mode = trans;
    SolveInfo info;
    fgmres(h->A0.nr, h_matvec, h_prec, h, b, x, restart, maxiter, rtol, mgs, &info);
    h->trans_mode = 0;
    *iterations = info.iterations; *restarts = info.restarts;
    *est = info.rel_res_est; *truer = info.rel_res_true;
    return info.status;
}

/* dL/dA on the block pattern (adjoint identity): for each stored value
 * (block p = (I,J), entry (r,c)) the gradient is -sum_k lam_k[I b + r] x_k[J b + c]. */
void orc_grad_values(int b, int nbr, const int *rp, const int *ci, int nrhs, const double *lam,
                     const double *x, double *dval) {
    long n = (long)nbr * b;
    for (int I = 0; I < nbr; ++I)
        for (int p = rp[I]; p < rp[I + 1]; ++p)
            for (int r = 0; r < b; ++r)
                for (int c = 0; c < b; ++c) {
                    double s = 0.0;
                    for (int k = 0; k < nrhs; ++k) s += lam[k * n + (long)I * b + r] * x[k * n + (long)ci[p] * b + c];
                    dval[(long)p * b * b + r * b + c] = -s;
                }
}

/* Hierarchy sizes: out[0] = MGR levels, out[1] = AMG levels, then for each MGR
 * level (n, nF, nC, nnz(A_c)), then for each AMG level (n, nnz). */
int orc_info(void *hp, long long *out, int cap) {
    Handle *h = (Handle *)hp;
    Mgr *m = h->mgr;
    int o = 0;
    if (cap < 2) return ORC_ERR_ARG;
    out[o++] = m->nlev;
    out[o++] = m->camg ? m->camg->nlev : 0;
    for (int l = 0; l < m->nlev && o + 4 <= cap; ++l) {
        out[o++] = m->L[l].n; out[o++] = m->L[l].nF; out[o++] = m->L[l].nC;
        const Csr *ac = (l + 1 < m->nlev) ? &m->L[l + 1].A : &m->Acoarse;
        out[o++] = csr_nnz(ac);
    }
    if (m->camg)
        for (int k = 0; k < m->camg->nlev && o + 2 <= cap; ++k) {
            out[o++] = m->camg->A[k].nr;
            out[o++] = csr_nnz(&m->camg->A[k]);
        }
    return o;
}

/* Export pieces of the hierarchy.
 * kind 0 (MGR level `level`): what 0 = C/F flags (int32, 1 = C), 1 = coarse
 *   operator A_{l+1}, 2 = P_F, 3 = R_F, 4 = A_FF, 5 = F-relaxation operator M.
 * kind 1 (AMG on the final coarse system, level `level`): what 0 = C/F (+1/-1),
 *   1 = A_k, 2 = P_k.
 * kind 2 (F-relaxation AMG of MGR level `sub`, AMG level `level`): as kind 1.
 * sizes[0..2] = rows, cols, nnz (or vector length in sizes[0]). */
static const Csr *export_csr(Handle *h, int kind, int level, int what, int sub) {
    Mgr *m = h->mgr;
    if (kind == 0) {
        if (level < 0 || level >= m->nlev) return NULL;
        MgrLevel *l = &m->L[level];
        if (what == 1) return (level + 1 < m->nlev) ? &m->L[level + 1].A : &m->Acoarse;
        if (what == 2) return &l->PF;
        if (what == 3) return &l->RF;
        if (what == 4) return &l->AFF;
        if (what == 5) return &l->MF;
        return NULL;
    }
    Amg *a = (kind == 1) ? m->camg : ((sub >= 0 && sub < m->nlev) ? m->L[sub].famg : NULL);
    if (!a || level < 0 || level >= a->nlev) return NULL;
    if (what == 1) return &a->A[level];
    if (what == 2) return (level < a->nlev - 1) ? &a->P[level] : NULL;
    return NULL;
}

int orc_export(void *hp, int kind, int level, int what, int sub, long long *sizes, int *b0, int *b1, double *b2) {
    Handle *h = (Handle *)hp;
    Mgr *m = h->mgr;
    if (what == 0) {
        const int *src = NULL;
        int n = 0;
        int conv = 0;
        if (kind == 0) {
            if (level < 0 || level >= m->nlev) return ORC_ERR_ARG;
            src = m->L[level].isF; n = m->L[level].n; conv = 1;
        } else {
            Amg *a = (kind == 1) ? m->camg : ((sub >= 0 && sub < m->nlev) ? m->L[sub].famg : NULL);
            if (!a || level < 0 || level >= a->nlev - 1) return ORC_ERR_ARG;
            src = a->cf[level]; n = a->A[level].nr;
        }
        sizes[0] = n; sizes[1] = 0; sizes[2] = 0;
        if (b0)
            for (int i = 0; i < n; ++i) b0[i] = conv ? (src[i] ? 0 : 1) : src[i];
        return ORC_OK;
    }
    const Csr *c = export_csr(h, kind, level, what, sub);
    if (!c) return ORC_ERR_ARG;
    sizes[0] = c->nr; sizes[1] = c->nc; sizes[2] = c->rp ? csr_nnz(c) : 0;
    if (b0 && c->rp) memcpy(b0, c->rp, ((size_t)c->nr + 1) * sizeof(int));
    if (b1 && c->rp) memcpy(b1, c->ci, (size_t)csr_nnz(c) * sizeof(int));
    if (b2 && c->rp) memcpy(b2, c->v, (size_t)csr_nnz(c) * sizeof(double));
    return ORC_OK;
}

/* ---- standalone building blocks, exposed so tests can pin each one ---- */
typedef struct { Csr c; } CsrBox;

static Csr wrap(int nr, int nc, const int *rp, const int *ci, const double *v) {
    Csr a;
    a.nr = nr; a.nc = nc;
    a.rp = (int *)rp; a.ci = (int *)ci; a.v = (double *)v;
    return a;
}

void *orc_csr_spgemm(int anr, int anc, const int *arp, const int *aci, const double *av, int bnr, int bnc,
                     const int *brp, const int *bci, const double *bv) {
    (void)anc; (void)bnr;
    Csr a = wrap(anr, anc, arp, aci, av), b = wrap(bnr, bnc, brp, bci, bv);
    CsrBox *box = (CsrBox *)xcalloc(1, sizeof(CsrBox));
    box->c = csr_spgemm(&a, &b);
    return box;
}
void *orc_csr_add(int nr, int nc, const int *arp, const int *aci, const double *av, const int *brp,
                  const int *bci, const double *bv) {
    Csr a = wrap(nr, nc, arp, aci, av), b = wrap(nr, nc, brp, bci, bv);
    CsrBox *box = (CsrBox *)xcalloc(1, sizeof(CsrBox));
    box->c = csr_add(&a, &b);
    return box;
}
void *orc_csr_transpose(int nr, int nc, const int *rp, const int *ci, const double *v) {
    Csr a = wrap(nr, nc, rp, ci, v);
    CsrBox *box = (CsrBox *)xcalloc(1, sizeof(CsrBox));
    box->c = csr_transpose(&a);
    return box;
}
void orc_box_sizes(void *bp, long long *sizes) {
    CsrBox *b = (CsrBox *)bp;
    sizes[0] = b->c.nr; sizes[1] = b->c.nc; sizes[2] = csr_nnz(&b->c);
}
void orc_box_copy(void *bp, int *rp, int *ci, double *v) {
    CsrBox *b = (CsrBox *)bp;
    memcpy(rp, b->c.rp, ((size_t)b->c.nr + 1) * sizeof(int));
    memcpy(ci, b->c.ci, (size_t)csr_nnz(&b->c) * sizeof(int));
    memcpy(v, b->c.v, (size_t)csr_nnz(&b->c) * sizeof(double));
}
void orc_box_free(void *bp) {
    CsrBox *b = (CsrBox *)bp;
    if (!b) return;
    csr_free(&b->c);
    free(b);
}
void orc_strength(int n, const int *rp, const int *ci, const double *v, double theta, const int *label,
                  unsigned char *strong) {
    Csr a = wrap(n, n, rp, ci, v);
    amg_strength(&a, theta, label, strong);
}
int orc_pmis(int n, const int *rp, const int *ci, const unsigned char *strong, unsigned long long seed, int level,
             int *cf) {
    Csr a = wrap(n, n, rp, ci, NULL);
    return amg_pmis(&a, strong, (uint64_t)seed, level, cf);
}
double orc_pmis_uniform(unsigned long long seed, int level, int i) { return pmis_uniform((uint64_t)seed, level, i); }
void *orc_direct_interp(int n, const int *rp, const int *ci, const double *v, const unsigned char *strong,
                        const int *cf, const int *label, int *status) {
    Csr a = wrap(n, n, rp, ci, v);
    CsrBox *box = (CsrBox *)xcalloc(1, sizeof(CsrBox));
    *status = amg_direct_interp(&a, strong, cf, label, &box->c);
    return box;
}
void orc_aggressive_split(int n, const int *rp, const int *ci, const unsigned char *strong, unsigned long long seed,
                          int level, int *cf) {
    Csr a = wrap(n, n, rp, ci, NULL);
    amg_aggressive_split(&a, strong, (uint64_t)seed, level, cf);
}
void *orc_multipass_interp(int n, const int *rp, const int *ci, const double *v, const unsigned char *strong,
                           const int *cf, const int *label, int *status) {
    Csr a = wrap(n, n, rp, ci, v);
    CsrBox *box = (CsrBox *)xcalloc(1, sizeof(CsrBox));
    *status = amg_multipass_interp(&a, strong, cf, label, &box->c);
    return box;
}
void *orc_ext_interp(int n, const int *rp, const int *ci, const double *v, const unsigned char *strong,
                     const int *cf, const int *label, int *status) {
    Csr a = wrap(n, n, rp, ci, v);
    CsrBox *box = (CsrBox *)xcalloc(1, sizeof(CsrBox));
    *status = amg_ext_interp(&a, strong, cf, label, &box->c);
    return box;
}
int orc_lu_solve(int n, const double *dense, const double *b, double *x, int trans) {
    double *m = (double *)xmalloc((size_t)n * n * sizeof(double));
    int *piv = (int *)xmalloc((size_t)n * sizeof(int));
    memcpy(m, dense, (size_t)n * n * sizeof(double));
    int st = lu_factor(n, m, piv);
    if (st == ORC_OK) lu_solve(n, m, piv, b, x, trans);
    free(m); free(piv);
    return st;
}
int orc_small_inverse(int bs, const double *blk, double *inv) { return small_inverse(bs, blk, inv); }
/* ILU(0) factor of a square CSR matrix on its own pattern (lu: nnz values,
 * diag: n positions of the diagonal entries) and the solves with it. */
int orc_ilu0(int n, const int *rp, const int *ci, const double *v, double *lu, int *diag) {
    Csr a = wrap(n, n, rp, ci, v);
    double *f = NULL;
    int *d = NULL;
    int st = ilu0_factor(&a, &f, &d);
    memcpy(lu, f, (size_t)csr_nnz(&a) * sizeof(double));
    memcpy(diag, d, (size_t)n * sizeof(int));
    free(f); free(d);
    return st;
}
void orc_ilu0_solve(int n, const int *rp, const int *ci, const double *lu, const int *diag, const double *r,
                    double *z, int trans) {
    Csr a = wrap(n, n, rp, ci, NULL);
    ilu0_solve(&a, lu, diag, r, z, trans);
}

/* Threads used by the solve phase (OpenMP); 0 or less leaves the default. */
int orc_set_threads(int nthreads) {
#ifdef _OPENMP
    if (nthreads > 0) omp_set_num_threads(nthreads);
    return omp_get_max_threads();
#else
    (void)nthreads;
    return 1;
#endif
}
