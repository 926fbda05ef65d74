// kernels.hpp -- host-side launchers of the gfx950 kernels.  Setup kernels
// live in k_setup.hip (built with -ffp-contract=off so that every coarse value
// is rounded exactly as the sums are written); apply / Krylov kernels live in
// k_apply.hip.  All launchers are asynchronous on the given stream unless they
// return a host value.
#pragma once

#include "common.hpp"

namespace mgr {

// ---------------------------------------------------------------- setup
// out[0..n] = exclusive prefix sum of in[0..n), out[n] = total (clamped to
// int32; scan_async reports the exact total), asynchronous.
void scan_exclusive_async(const int* in, int* out, int n, hipStream_t s);
// Asynchronous scan that also stores {total, max input} into slot[0..1] (device).
void scan_async(const int* in, int* out, int n, long long* slot, hipStream_t s);
void fill_ll(long long* p, long long v, int n, hipStream_t s);
int read_int(const int* dptr, hipStream_t s);

// Scalar CSR of the block-CSR input without exact zeros inside blocks (the
// diagonal is always kept): row lengths, then (rows allocated from their scan)
// the entries.
void bsr_count(int b, int nbr, long nnzb, const int* brp, const int* bci, const double* bv, int* cnt,
               hipStream_t s);
void bsr_fill(int b, int nbr, long nnzb, const int* brp, const int* bci, const double* bv, DCsr& A, hipStream_t s);
void bsr_transpose_blocks(int b, int nbr, const int* rp, const int* ci, const double* v, int* trp, int* tci,
                          double* tv, hipStream_t s);

// hist[f] = number of labels equal to f (32 bins); *flag = 5 for a label
// outside [0, 32).
void field_hist(int n, const int* field, int* hist, int* flag, hipStream_t s);
// isF[i] = bit field[i] of mask; flag set to 1 if a label is outside [0,32).
void cf_flags(int n, const int* field, uint32_t mask, int* isF, int* flag, hipStream_t s);
// fpos = exclusive scan of isF; lmap[i] = local index in F or C; fmap / cmap.
void cf_maps(int n, const int* isF, const int* fpos, int* lmap, int* fmap, int* cmap, hipStream_t s);
void iota_div(int n, int b, int* out, hipStream_t s);
void gather_int(int n, const int* map, const int* src, int* dst, hipStream_t s);
// row counts of the four blocks A_FF, A_FC (F rows), A_CF, A_CC (C rows), then
// their entries; fblk (F-relaxation block of each F-point, or null) keeps in
// A_FF only each F row's own block; null counts / outputs are skipped.  The
// bsr_ variants read the block-CSR input directly (exact zeros inside blocks
// off the diagonal are not entries).
void extract_count(const DCsr& A, const int* isF, const int* lmap, const int* fblk, int* cFF, int* cFC, int* cCF,
                   int* cCC, hipStream_t s);
void extract_fill(const DCsr& A, const int* isF, const int* lmap, const int* fblk, DCsr* FF, DCsr* FC, DCsr* CF,
                  DCsr* CC, hipStream_t s);
void bsr_extract_count(int b, int nbr, long nnzb, const int* brp, const int* bci, const double* bv, const int* isF,
                       const int* lmap, const int* fblk, int* cFF, int* cFC, int* cCF, int* cCC, hipStream_t s);
// With vcopy (nnzb b^2 values), the block values are also copied there.
void bsr_extract_fill(int b, int nbr, long nnzb, const int* brp, const int* bci, const double* bv, const int* isF,
                      const int* lmap, const int* fblk, DCsr* FF, DCsr* FC, DCsr* CF, DCsr* CC, double* vcopy,
                      hipStream_t s);

// F-relaxation operator: blocks = runs of consecutive F-points with equal block id
// (Jacobi: every point its own block).  bstart gets nb+1 entries.
void frelax_block_flags(int nF, const int* bid, int* flagk, hipStream_t s);
void frelax_block_starts(int nF, const int* flagk, const int* excl, int* bstart, int* bnum, hipStream_t s);
void frelax_row_len(int nF, const int* bnum, const int* bstart, int* len, int* flag, hipStream_t s);
void frelax_fill(int nb, const int* bstart, const DCsr& AFF, DCsr& M, int* flag, hipStream_t s);

// C = A B counts; rows of A longer than the variant chosen by max_row get a zero
// count and set *flag (an int in device memory) to 1.
// Right factors with at most SPGEMM_DENSE_COLS columns (and few enough rows x
// columns) use a dense-row accumulator per output row instead of the merge.
// With `loose`, products whose rows may exceed 256 columns (up to a bound of
// SPGEMM_HASH_LOOSE) are counted in hash tables of 512 slots; a full table
// sets *flag to 2, and the count must then be made again without `loose`.
constexpr int SPGEMM_DENSE_COLS = 4096;
constexpr long SPGEMM_HASH_LOOSE = 2048;
void spgemm_count(const DCsr& A, const DCsr& B, int max_row, int* cnt, int* flag, hipStream_t s, bool loose = false);
// C's row pointers and max_row come from the counts; a failure of the hashed
// variant (a full table) sets *flag (an int in device memory).  With neg,
// C = -A B (each value the negated sum).
void spgemm_fill(const DCsr& A, const DCsr& B, int max_row, DCsr& C, int* flag, hipStream_t s, bool neg = false);
// C = D + A B in one hashed product (D has A's rows and B's columns), when
// every row of C is bounded by maxrow(A) maxrow(B) + maxrow(D) <= 256; the
// values are those of the product followed by a separate sparse add.
bool spgemm_add_fusable(const DCsr& A, const DCsr& B, const DCsr& D);
// With `loose`, the rows are counted in tables of at most the larger of
// SPGEMM_ADD_LOOSE_CAP slots and twice D's longest row (the bound maxrow(A)
// maxrow(B) + maxrow(D) is far above the rows of a Galerkin product of stencil
// operators); a full table sets *flag to 2, and the count must then be made
// again without `loose`.
constexpr int SPGEMM_ADD_LOOSE_CAP = 64;
// With brep (one int per row of B), rows of B with equal brep must have equal
// patterns (the rows of P_F = -M A_FC of one F-relaxation block): the count
// then inserts the pattern of a run of such rows selected by consecutive
// entries of a row of A once, and the numeric pass finds such a row's slots
// where the previous entry put them.
void spgemm_add_count(const DCsr& A, const DCsr& B, const DCsr& D, int* cnt, int* flag, hipStream_t s,
                      bool loose = false, const int* brep = nullptr);
void spgemm_add_fill(const DCsr& A, const DCsr& B, const DCsr& D, DCsr& C, int* flag, hipStream_t s,
                     const int* brep = nullptr);
// Products with the block-diagonal F-relaxation operator M (blocks of at most
// four rows over [bstart[t], bstart[t+1]), each row storing its block's
// columns; a failed larger block one diagonal entry per row), with the
// pattern (and values) of the general product.  Left: the row counts of M B
// (B's rows of at most 16 entries).  Right: C = A M (A's rows of at most 32
// entries, columns ascending).  A violated bound sets *flag to 1.
bool bdiag_left_ok(const DCsr& M, const DCsr& B);
bool bdiag_right_ok(const DCsr& A, const DCsr& M);
void bdiag_left_count(int nb, const int* bstart, const DCsr& B, int* cnt, int* flag, hipStream_t s);
void bdiag_right_count(const DCsr& A, const DCsr& M, int* cnt, int* flag, hipStream_t s);
void bdiag_right_fill(const DCsr& A, const DCsr& M, DCsr& C, int* flag, hipStream_t s);
void add_count(const DCsr& A, const DCsr& B, int* cnt, hipStream_t s);
void add_fill(const DCsr& A, const DCsr& B, DCsr& C, hipStream_t s);
void negate(double* v, long n, hipStream_t s);
void transpose_count(const DCsr& A, int* cnt, hipStream_t s);
// T's row pointers must be the exclusive scan of cnt (the column counts of A);
// cnt is consumed (decremented to zero).
void transpose_fill(const DCsr& A, DCsr& T, int* cnt, hipStream_t s);

// AMG setup
// strength flags per entry, the number of strong entries per row (scnt) and
// per column (lam, incremented: it must start at zero); with dinv, also the
// L1 Jacobi diagonal exactly as l1_dinv forms it (*flag set where it is not
// positive)
void amg_strength(const DCsr& A, double theta, const int* label, unsigned char* strong, int* scnt, int* lam,
                  double* dinv, int* flag, hipStream_t s);
void strength_compact_fill(const DCsr& A, const unsigned char* strong, const int* srp, int* sci, hipStream_t s);
void pmis_init(int n, const int* lam, uint64_t seed, int level, double* w, int* cf, hipStream_t s);
// PMIS rounds (lane groups sized to avg_row, the mean strong-row length):
// select marks the beaten undecided points (beaten must start at zero);
// update moves the state cf -> cf_next and clears beaten_next.
void pmis_select(int n, const int* srp, const int* sci, const double* w, const int* cf, unsigned char* beaten,
                 int avg_row, hipStream_t s);
void pmis_update(int n, const int* srp, const int* sci, const int* cf, const unsigned char* beaten, int* cf_next,
                 unsigned char* beaten_next, int* undecided, int avg_row, hipStream_t s);
void cf_is_c(int n, const int* cf, int* isC, hipStream_t s);
void interp_count(const DCsr& A, const unsigned char* strong, const int* cf, int* cnt, hipStream_t s);
// needs A's CSR-stream row blocks (one workgroup each)
void interp_fill(const DCsr& A, const unsigned char* strong, const int* cf, const int* cidx, const int* label,
                 DCsr& P, int* flag, hipStream_t s);
// Extended+i interpolation: the row counts of P (the size of each F-point's
// interpolatory set; *flag set where one exceeds the table), then the weights
// (P's row pointers and max_row from the counts; max_row <= 256)
void interp_ext_count(const DCsr& A, const unsigned char* strong, const int* cf, int* cnt, int* flag, hipStream_t s);
void interp_ext_fill(const DCsr& A, const unsigned char* strong, const int* cf, const int* cidx, const int* label,
                     DCsr& P, int* flag, hipStream_t s);
void l1_dinv(const DCsr& A, double* dinv, int* flag, hipStream_t s);
// aggressive coarsening: the factors of the second-order strength graph on the
// first C-points (C1 flags isC1, C1 index e1, C1 points pts), its diagonal
// dropped, column counts, the final split; multi-pass interpolation's
// interpolated-so-far flags and the count of points the next pass reaches
void agg_rt_count(int n, const int* srp, const int* sci, const int* isC1, int* cnt, hipStream_t s);
void agg_rt_fill(int n, const int* srp, const int* sci, const int* isC1, const int* e1, DCsr& Rt, hipStream_t s);
void agg_l_count(int n1, const int* pts, const int* srp, int* cnt, hipStream_t s);
void agg_l_fill(int n1, const int* pts, const int* srp, const int* sci, DCsr& L, hipStream_t s);
void nodiag_count(const DCsr& A, int* cnt, hipStream_t s);
void nodiag_fill(const DCsr& A, DCsr& B, hipStream_t s);
void col_count(long nnz, const int* ci, int* lam, hipStream_t s);
void agg_final(int n, const int* isC1, const int* e1, const int* cf2, int* cf, hipStream_t s);
void mp_assigned(int n, const int* cf, const int* prp, int* cfm, hipStream_t s);
void mp_reach(int n, const int* cfm, const int* wcnt, long long* reach, hipStream_t s);
// diagonal of the hybrid L1 Gauss-Seidel smoother: a_ii + sum of |a_ij| over the
// entries of row i outside its chunk of `chunk` consecutive rows
void hgs_diag(const DCsr& A, int chunk, double* d, int* flag, hipStream_t s);
// B = the entries a_ij of A with label[i] == label[j] (the separate-component
// approximation), in A's order: row counts, then (B's rows allocated) the fill.
void label_filter_count(const DCsr& A, const int* label, int* cnt, hipStream_t s);
void label_filter_fill(const DCsr& A, const int* label, DCsr& B, hipStream_t s);
// In-chunk triangles of the hybrid Gauss-Seidel sweep (columns sorted, dpos =
// each row's diagonal position): w[0], w[1] = the most entries of a row below
// and above its diagonal inside its chunk (w zeroed beforehand); the fill
// writes slot tables of widths wl and wu for nchp >= ceil(n / chunk) chunks
// (slot k of position t of chunk c at (t W + k) nchp + c: local column, value;
// padding has value 0) and dT[t nchp + c] = 1 / d of row c chunk + t (1 past n).
void hgs_tri_count(const DCsr& A, const int* dpos, int chunk, int* w, hipStream_t s);
void hgs_tri_fill(const DCsr& A, const int* dpos, const double* d, int chunk, int nchp, int wl, unsigned char* lc,
                  double* lv, int wu, unsigned char* uc, double* uv, double* dT, hipStream_t s);
// Composed operators of one L1-Jacobi V(1,1) level (b_c = G b, x = W b + Q x_c):
// w = 2 D^-1 - D^-1 A D^-1 on A's pattern; out = X - S Y on Y's pattern with
// S = diag(rs) on the left or diag(cs) on the right; C = [A | B].  *bad is set
// when a row of A stores no diagonal or X is not contained in Y.
void compose_w(const DCsr& A, const double* dinv, double* w, int* bad, hipStream_t s);
void compose_sub(const DCsr& X, const DCsr& Y, const double* rs, const double* cs, double* out, int* bad,
                 hipStream_t s);
void concat_rows(const DCsr& A, const DCsr& B, DCsr& C, hipStream_t s);
// dense row-major copy of A (nr x nc)
void densify(const DCsr& A, double* dense, hipStream_t s);
// small dense helpers for the coarse tail of the AMG cycle: C = A B (m x k
// times k x n), T += Q X (Q sparse, X with rows of n), T = A^T (n x n)
void dense_gemm(int m, int k, int n, const double* a, const double* b, double* c, hipStream_t s);
void sparse_dense_add(const DCsr& Q, const double* x, int n, double* t, hipStream_t s);
void dense_transpose(int n, const double* a, double* t, hipStream_t s);
void dense_inverse(int n, double* a, double* inv, int* flag, hipStream_t s);

// ILU(0): level analysis (fwd: dependencies on columns < i; else > i), bucketing
// of rows by level, factorization of one level, split into L (strict lower) and
// U (diagonal + upper)
void level_sweep(const DCsr& A, bool fwd, int* lev, int* changed, hipStream_t s);
void level_max(int n, const int* lev, int* out, hipStream_t s);
void level_bucket(int n, const int* lev, int* cnt, int* cursor, int* order, hipStream_t s, bool scatter);
void diag_pos(const DCsr& A, int* dpos, int* flag, hipStream_t s);
void ilu_level(int cnt, const int* rows, DCsr& LU, const int* dpos, int* flag, hipStream_t s);
void split_count(const DCsr& A, int* nl, int* nu, hipStream_t s);
void split_fill(const DCsr& A, DCsr& L, DCsr& U, hipStream_t s);

// MGR apply operators of the fused one-sweep path (the fills also write the
// FP32 copy of the values when R.vf / P.vf is allocated)
void rj_count(int nC, const DCsr& X, int* len, hipStream_t s);
void rj_fill(int nC, const DCsr& X, double scale, const int* fmap, const int* cmap, DCsr& R, hipStream_t s);
void pj_count(int n, const int* isF, const int* lmap, const DCsr& Y, const DCsr& M, int* len, hipStream_t s);
void pj_fill(int n, int nC, const int* isF, const int* lmap, const DCsr& Y, double yscale, const DCsr& M,
             double mscale, const int* fmap, DCsr& P, hipStream_t s);

void to_float(const double* src, float* dst, long n, hipStream_t s);
// k (at most F32_SEGS) conversions dst[q][i] = (float)src[q][i], i < n[q], in
// one launch (segments with n[q] <= 0 take no blocks)
constexpr int F32_SEGS = 32;
struct F32Segs {
    const double* src[F32_SEGS];
    float* dst[F32_SEGS];
    long n[F32_SEGS];
    int boff[F32_SEGS + 1];
    int k;
};
void to_float_batch(int k, const double* const* src, float* const* dst, const long* n, hipStream_t s);
void fill_int(int* p, int v, long n, hipStream_t s);
void fill_bytes(unsigned char* p, unsigned char v, long n, hipStream_t s);

}  // namespace mgr
