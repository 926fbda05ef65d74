// apply.hpp -- launchers of the solve-phase kernels (k_apply.hip).
#pragma once

#include "common.hpp"

namespace mgr {

// Number of per-block partial sums used by the Krylov reductions (a fixed grid
// so that every reduction is formed in the same order on every call).
constexpr int KRYLOV_PARTS = 2048;
// CSR-stream SpMV: nominal nonzeros per row block, and the LDS stage size.
constexpr int SPMV_CHUNK = 1024;
constexpr int SPMV_LDS = 2048;
// a row counts as 1/SPMV_ROW_COST of a nonzero when rows are cut into blocks,
// so a block never holds more than SPMV_CHUNK * SPMV_ROW_COST rows (matrices
// with many empty rows, such as an interpolation onto a few wells)
constexpr int SPMV_ROW_COST = 4;

// Read-only view of a CSR operator in value type T with its SpMV group size
// (lanes per row, chosen from the average row length).
template <typename T>
struct SpOp {
    int nr = 0, nc = 0;
    long nnz = 0;
    const int* rp = nullptr;
    const int* ci = nullptr;
    const T* v = nullptr;
    const int* blk = nullptr;  // row-block boundaries (nblk + 1)
    const int* bpos = nullptr; // their entry offsets
    int nblk = 0;
    const int* eci = nullptr;  // sliced ELL copy, if any (see DCsr)
    const int* esw = nullptr;
    const T* ev = nullptr;
    int ew = 0;
};

// number of row blocks of an operator with nnz entries, and their boundaries
int rowblock_count(int nr, long nnz);
void rowblocks(int nr, long nnz, const int* rp, int* blk, int* bpos, hipStream_t s);

template <typename T>
inline SpOp<T> view(const DCsr& A);
// Sliced ELL copies for operators of at least ELL_MIN_ROWS rows whose longest
// row (at most ELL_MAX_W) is within 1/0.7 of the mean: one thread per row then
// reads its slots with coalesced loads and no row pointers or LDS stage, and
// each workgroup's slice is only as wide as its own longest row.  Whether the
// copy pays is decided once per operator, on its first use, from the slice
// widths (read back with a synchronisation): its slots may exceed the stored
// entries by 15% at most (rows of very different lengths mixed within slices
// would make the copy longer than the CSR stream it replaces).
constexpr int ELL_MAX_W = 16;
constexpr int ELL_MIN_ROWS = 32768;
constexpr int ELL_SLICE = 256;   // rows per slice = threads per workgroup of the kernel
inline bool ell_ok(const DCsr& A) {
    return A.nc >= 1 && A.nr >= ELL_MIN_ROWS && A.max_row >= 1 && A.max_row <= ELL_MAX_W &&
           7L * A.max_row * A.nr <= 10L * A.nnz;
}
// the copy pays when its slots (sum of the slice widths times ELL_SLICE)
// exceed the stored entries by at most 15%
inline bool ell_pays(long slots, long nnz) { return 20 * slots <= 23 * nnz; }
// slice widths (esw, one per ELL_SLICE rows), then the slices (with eci = nullptr
// only the values: the columns are there already)
void ell_widths(int nr, const int* rp, int* esw, hipStream_t s);
long ell_total_width(const int* esw, int nsl, hipStream_t s);   // sum of esw (synchronises)
void to_ell(int nr, int nc, int w, const int* esw, const int* rp, const int* ci, const double* v, int* eci,
            double* ev, hipStream_t s);
void to_ell(int nr, int nc, int w, const int* esw, const int* rp, const int* ci, const float* v, int* eci,
            float* ev, hipStream_t s);

// The row-block partition of an operator (and its ELL copy, where one pays) is
// made on its first use by an SpMV (on the operator's stream), so setup
// temporaries never pay for one.
inline void ensure_ell(const DCsr& A, bool fp32) {
    if (A.ell_state < 0) return;
    DCsr& M = const_cast<DCsr&>(A);
    const size_t nsl = (size_t)(M.nr + ELL_SLICE - 1) / ELL_SLICE;
    const size_t slots = (size_t)M.max_row * ELL_SLICE * nsl;
    if (M.ell_state == 0) {
        if (!ell_ok(M)) {
            M.ell_state = -1;
            return;
        }
        M.esw.alloc(nsl, M.rp.s);
        ell_widths(M.nr, M.rp.p, M.esw.p, M.rp.s);
        const long used = ell_total_width(M.esw.p, (int)nsl, M.rp.s) * ELL_SLICE;
        if (!ell_pays(used, M.nnz)) {
            M.esw.reset();
            M.ell_state = -1;
            return;
        }
        M.ell_state = 1;
    }
    if (!fp32 && !M.ev.p) {
        M.ev.alloc(slots, M.rp.s);
        const bool need_ci = !M.eci.p;
        if (need_ci) M.eci.alloc(slots, M.rp.s);
        to_ell(M.nr, M.nc, M.max_row, M.esw.p, M.rp.p, M.ci.p, M.v.p, need_ci ? M.eci.p : nullptr, M.ev.p,
               M.rp.s);
    }
    if (fp32 && !M.evf.p && M.vf.p) {
        M.evf.alloc(slots, M.rp.s);
        const bool need_ci = !M.eci.p;
        if (need_ci) M.eci.alloc(slots, M.rp.s);
        to_ell(M.nr, M.nc, M.max_row, M.esw.p, M.rp.p, M.ci.p, M.vf.p, need_ci ? M.eci.p : nullptr, M.evf.p,
               M.rp.s);
    }
    M.ew = M.max_row;
}
inline void ensure_rowblocks(const DCsr& A) {
    if (A.blk.p || A.nr <= 0) return;
    DCsr& M = const_cast<DCsr&>(A);
    M.nblk = rowblock_count(M.nr, M.nnz);
    M.blk.alloc((size_t)M.nblk + 1, M.rp.s);
    M.bpos.alloc((size_t)M.nblk + 1, M.rp.s);
    rowblocks(M.nr, M.nnz, M.rp.p, M.blk.p, M.bpos.p, M.rp.s);
}

template <>
inline SpOp<double> view<double>(const DCsr& A) {
    ensure_rowblocks(A);
    SpOp<double> o;
    o.nr = A.nr; o.nc = A.nc; o.nnz = A.nnz; o.rp = A.rp.p; o.ci = A.ci.p; o.v = A.v.p;
    o.blk = A.blk.p; o.bpos = A.bpos.p; o.nblk = A.nblk;
    ensure_ell(A, false);
    if (A.ev.p) { o.eci = A.eci.p; o.esw = A.esw.p; o.ev = A.ev.p; o.ew = A.ew; }
    return o;
}
template <>
inline SpOp<float> view<float>(const DCsr& A) {
    ensure_rowblocks(A);
    SpOp<float> o;
    o.nr = A.nr; o.nc = A.nc; o.nnz = A.nnz; o.rp = A.rp.p; o.ci = A.ci.p; o.v = A.vf.p;
    o.blk = A.blk.p; o.bpos = A.bpos.p; o.nblk = A.nblk;
    ensure_ell(A, true);
    if (A.evf.p) { o.eci = A.eci.p; o.esw = A.esw.p; o.ev = A.evf.p; o.ew = A.ew; }
    return o;
}

// y = alpha * A [x | x2] + beta * w: columns >= split read x2[c - split];
// pass x2 = nullptr and split = INT_MAX for a single source, w = nullptr for beta = 0.
// tag = 1 selects a separately named kernel instance (the FGMRES matvec), so that
// profiles report it on its own.
template <typename MT, typename XT, typename X2T, typename YT, typename WT>
void spmv(const SpOp<MT>& A, const XT* x, const X2T* x2, int split, const WT* w, YT* y, MT alpha, MT beta,
          hipStream_t s, int tag = 0);
// y = x + dinv .* (b - A x)  (out of place)
template <typename T>
void jacobi_sweep(const SpOp<T>& A, const T* dinv, const T* b, const T* x, T* y, hipStream_t s);
// x = dinv .* b ; r = b - A x
template <typename T>
void presmooth(const SpOp<T>& A, const T* dinv, const T* b, T* x, T* r, hipStream_t s);
// the same with bd = dinv .* b formed beforehand (one gathered vector per entry)
template <typename T>
void presmooth_scaled(const SpOp<T>& A, const T* bd, const T* b, T* x, T* r, hipStream_t s);
// y = A x and yd = dsc .* y (a restriction that also forms the next level's D^-1 b)
template <typename T, typename XT>
void restrict_scaled(const SpOp<T>& A, const XT* x, const T* dsc, T* y, T* yd, hipStream_t s);
// block-CSR y = alpha A x + beta w (FP64)
void bsr_spmv(int bsize, int nbr, const int* rp, const int* ci, const double* v, long nnzb, const double* x,
              const double* w, double* y, double alpha, double beta, hipStream_t s);
template <typename T, typename XT>
void dense_gemv(int n, const T* m, const XT* x, T* y, hipStream_t s);
template <typename S, typename D>
void gather(int n, const int* map, const S* src, D* dst, hipStream_t s);
template <typename S, typename D>
void scatter(int n, const int* map, const S* src, D* dst, hipStream_t s);
template <typename T>
void axpby(long n, T a, const T* x, T b, T* y, hipStream_t s);
template <typename T>
void mul(long n, const T* d, const T* x, T* y, T w, hipStream_t s);
template <typename T>
void addmul(long n, const T* d, const T* x, T* y, T w, hipStream_t s);
template <typename S, typename D>
void copy(long n, const S* src, D* dst, hipStream_t s);
template <typename T>
void set(long n, T* dst, T v, hipStream_t s);
void scale(long n, double a, double* x, hipStream_t s);
// x /= sqrt(*norm2), norm2 in device memory
void scale_by_norm(long n, const double* norm2, double* x, hipStream_t s);

int krylov_parts(long n);
// out[i] = <V_i, w> for i < nvec (V column-major with leading dimension ldv);
// part needs nvec * KRYLOV_PARTS doubles.
void mdot(long n, const double* V, long ldv, int nvec, const double* w, double* part, double* out, hipStream_t s);
// Arnoldi step with delayed reorthogonalisation (two passes over the basis).
// arnoldi_dots: out[0..nvec) = V_i . V_{nvec-1}, out[nvec..2 nvec) = V_i . w
// (part needs 2 nvec KRYLOV_PARTS doubles).  arnoldi_update: from those dots,
// V_{nvec-1} gets its second Gram-Schmidt pass and normalisation, w is
// orthogonalised once against the final V_0..V_{nvec-1}; coef[0..nvec) = w's
// coefficients, coef[64] = the normalisation; *norm2_out = ||w||^2, after
// which csrc[0..ncopy) is stored to the host-mapped cdst and then 1.0 to
// cdst[ncopy] (the ready flag).
void arnoldi_dots(long n, const double* V, long ldv, int nvec, const double* w, double* part, double* out,
                  hipStream_t s);
void arnoldi_update(long n, double* V, long ldv, int nvec, const double* sh, double* w, double* part,
                    double* norm2_out, double* coef, const double* csrc, double* cdst, int ncopy, hipStream_t s);
// w -= hscale * sum_i h[i] V_i; if norm2_out, *norm2_out = ||w_new||^2.
void maxpy(long n, const double* V, long ldv, int nvec, const double* h, double hscale, double* w, double* part,
           double* norm2_out, hipStream_t s);
// Hybrid L1 Gauss-Seidel, second pass of a sweep: chunks of `chunk`
// consecutive rows (1..HGS_CHUNK_MAX), each relaxed in order by one thread;
// r = b - A x of the old x (or b when the sweep starts from zero, which then
// overwrites x).  The in-chunk entries of the sweep's direction come from the
// slot tables of hgs_tri_fill (width w, nchp chunks, a multiple of 64), dT =
// the reciprocal chunked L1 diagonal in the same chunk-position layout.
constexpr int HGS_CHUNK_MAX = 128;
template <typename T>
void hgs_tri(int n, int chunk, int w, int nchp, const unsigned char* lc, const T* lv, const T* dT, const T* r, T* x,
             bool backward, bool from_zero, hipStream_t s);
// rows[0..cnt) of one level of a triangular solve with matrix A: x_i = (b_i - sum_{j!=i} a_ij x_j) / a_ii
// (unit: diagonal 1 and not stored).  b may alias x.
template <typename T>
void trsv_level(int cnt, const int* rows, const SpOp<T>& A, const T* b, T* x, bool unit, hipStream_t s);
void grad_values(int b, int nbr, const int* rp, const int* ci, long nnzb, int nrhs, const double* lam,
                 const double* x, double* dv, hipStream_t s);

}  // namespace mgr
