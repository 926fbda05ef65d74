// mgr.hip -- host orchestration of the MGR + FGMRES library and its C-ABI.
//
// Method: Bui et al., arXiv 2101.11649.  Setup builds, per MGR level, the C/F
// split by field, the F-relaxation operator M, the Jacobi interpolation
// P = [-M A_FC; I] (Sec. 2, eq. (4)), the restriction (injection, eq. (4), or
// Jacobi, eq. (5)) and the Petrov-Galerkin coarse operator R A P, then a
// classical AMG hierarchy on the last coarse system (Sec. 4.1).  The apply is
// Algorithm 1 from z = 0 without global relaxation; FGMRES uses it as a right
// preconditioner (Sec. 4.1).  Every numeric step runs in the kernels of
// k_setup.hip / k_apply.hip; this file only sequences launches and sizes.
#include <atomic>
#include <climits>
#include <cmath>
#include <cstring>
#include <functional>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <type_traits>
#include <vector>

#include "apply.hpp"
#include "kernels.hpp"
#include "mgr.h"

namespace mgr {

// ====================================================================== sparse helpers
// Device-produced values the host needs during setup (prefix-sum totals,
// longest rows, counters, error flags) land in a small slot array that is read
// back with ONE pinned copy per sync point, so a whole setup needs a few tens of
// host synchronisations instead of one per scan.  The slots of one sync period
// form a region; each sync moves on to the next region, zeroed in advance
// with all the others, instead of clearing the region it read with a kernel of
// its own (a launch per sync saved).
struct Slots {
    static constexpr int N = 64;           // slots per region
    static constexpr int FLAG = N - 1;     // int error flag kept in the last slot
    static constexpr int REGIONS = 64;     // regions zeroed together
    DArr<long long> d;
    long long* h = nullptr;
    long long* cur = nullptr;    // the region slots are taken from
    long long* read = nullptr;   // the region the last sync read into h
    int region = 0;
    int next = 0;
    hipStream_t s = nullptr;
    void init(hipStream_t st) {
        s = st;
        d.alloc((size_t)N * REGIONS, s);
        fill_ll(d.p, 0, (long)N * REGIONS, s);
        cur = read = d.p;
        region = 0;
        MGR_HIP(hipHostMalloc(reinterpret_cast<void**>(&h), sizeof(long long) * N, hipHostMallocDefault));
        std::memset(h, 0, sizeof(long long) * N);
    }
    ~Slots() {
        if (h) (void)hipHostFree(h);
    }
    long long* take(int k) {
        if (next + k > FLAG) throw Error(MGR_ERR_ARG, "internal: too many pending setup values");
        long long* p = cur + next;
        next += k;
        return p;
    }
    int* flag() { return reinterpret_cast<int*>(cur + FLAG); }
    // called by the AMG setup at the start of each level with its size (work
    // held back for the small levels, whose kernels leave the GPU mostly idle)
    std::function<void(int)> level_hook;
    // Reads the region back; slots taken afterwards come from the next region
    // (zero).  When the regions run out they are all zeroed again, on the
    // stream, which the sync has just drained.
    void sync(const char* what) {
        MGR_HIP(hipMemcpyAsync(h, cur, sizeof(long long) * N, hipMemcpyDeviceToHost, s));
        MGR_HIP(hipStreamSynchronize(s));
        read = cur;
        if (++region == REGIONS) {
            fill_ll(d.p, 0, (long)N * REGIONS, s);
            region = 0;
        }
        cur = d.p + (long)region * N;
        next = 0;
        int f = (int)(h[FLAG] & 0xffffffffLL);
        if (f != 0) {
            std::string m = std::string(what) + ": ";
            if (f == 3) throw Error(MGR_ERR_ZERO_PIVOT, m + "zero or non-finite pivot");
            if (f == 5) throw Error(MGR_ERR_BAD_LABELS, m + "field label outside [0, 32)");
            throw Error(MGR_ERR_UNSUPPORTED,
                        m + "unsupported input (row too long, block larger than 4, or a_ii <= 0)");
        }
    }
    // a slot's value, read back by the sync after it was taken (a slot read
    // after a later sync is an error in the caller's sequencing)
    long long val(const long long* p) const {
        const long i = p - read;
        if (i < 0 || i >= N) throw Error(MGR_ERR_ARG, "internal: setup value read after a later sync");
        return h[i];
    }
};

// Two-phase construction from row counts: begin() scans asynchronously, the
// caller syncs the slots, finish() allocates the entries.
struct Pend {
    DCsr* C = nullptr;
    long long* slot = nullptr;
};

static Pend csr_begin(DCsr& C, int nr, int nc, const int* counts, Slots& S) {
    C = DCsr();
    C.nr = nr;
    C.nc = nc;
    C.rp.alloc((size_t)nr + 1, S.s);
    Pend p{&C, S.take(2)};
    scan_async(counts, C.rp.p, nr, p.slot, S.s);
    return p;
}

static void csr_finish(const Pend& p, Slots& S) {
    DCsr& C = *p.C;
    long long nnz = S.val(p.slot);
    if (nnz > INT_MAX) throw Error(MGR_ERR_UNSUPPORTED, "operator exceeds the int32 index range");
    C.nnz = (long)nnz;
    C.max_row = (int)S.val(p.slot + 1);
    C.ci.alloc((size_t)(C.nnz > 0 ? C.nnz : 1), S.s);
    C.v.alloc((size_t)(C.nnz > 0 ? C.nnz : 1), S.s);
}

static DCsr csr_from_counts(int nr, int nc, const int* counts, Slots& S, const char* what) {
    DCsr C;
    Pend p = csr_begin(C, nr, nc, counts, S);
    S.sync(what);
    csr_finish(p, S);
    return C;
}

// C = A B in two phases around a sync point (symbolic count, then numeric fill).
struct Spgemm {
    const DCsr* A = nullptr;
    const DCsr* B = nullptr;
    const DCsr* D = nullptr;  // C = D + A B when set
    DCsr* C = nullptr;
    int bdiag = 0;            // symbolic pass by the block kernels: 1 for M B, 2 for A M
    bool neg = false;         // C = -A B
    const int* brep = nullptr;   // rows of B with equal brep share a pattern (C = D + A B)
    DArr<int> cnt;
    long long* lr = nullptr;
    Pend pend;
};

static void spgemm_begin(Spgemm& j, const DCsr& A, const DCsr& B, DCsr& C, Slots& S) {
    if (A.nc != B.nr) throw Error(MGR_ERR_ARG, "spgemm: inner dimensions differ");
    if (A.max_row < 0) throw Error(MGR_ERR_ARG, "internal: spgemm left factor without a known row length");
    j.A = &A;
    j.B = &B;
    j.C = &C;
    j.cnt.alloc((size_t)A.nr + 1, S.s);
    j.lr = S.take(1);
    spgemm_count(A, B, A.max_row, j.cnt.p, reinterpret_cast<int*>(j.lr), S.s, true);
    j.pend = csr_begin(C, A.nr, B.nc, j.cnt.p, S);
}

// A row overflowed its hash table in the symbolic pass: count again with
// tables sized for the bound (or the merging kernels) and size C from a read
// of its own (not through the slots, whose other pending values the caller
// has yet to use).
static void spgemm_recount(Spgemm& j, hipStream_t s) {
    DCsr& C = *j.C;
    DArr<long long> t(3, s);
    fill_ll(t.p, 0, 3, s);
    if (j.D) spgemm_add_count(*j.A, *j.B, *j.D, j.cnt.p, reinterpret_cast<int*>(t.p), s, false);
    else spgemm_count(*j.A, *j.B, j.A->max_row, j.cnt.p, reinterpret_cast<int*>(t.p), s, false);
    C = DCsr();
    C.nr = j.A->nr;
    C.nc = j.B->nc;
    C.rp.alloc((size_t)C.nr + 1, s);
    scan_async(j.cnt.p, C.rp.p, C.nr, t.p + 1, s);
    long long h[3] = {0, 0, 0};
    MGR_HIP(hipMemcpyAsync(h, t.p, sizeof(h), hipMemcpyDeviceToHost, s));
    MGR_HIP(hipStreamSynchronize(s));
    if (h[0] != 0) throw Error(MGR_ERR_ARG, "internal: spgemm row longer than its recorded length");
    if (h[1] > INT_MAX) throw Error(MGR_ERR_UNSUPPORTED, "operator exceeds the int32 index range");
    C.nnz = (long)h[1];
    C.max_row = (int)h[2];
    C.ci.alloc((size_t)(C.nnz > 0 ? C.nnz : 1), s);
    C.v.alloc((size_t)(C.nnz > 0 ? C.nnz : 1), s);
}

// C = D + A B in one hashed product (requires spgemm_add_fusable(A, B, D));
// brep as for spgemm_add_count.
static void spgemm_add_begin(Spgemm& j, const DCsr& A, const DCsr& B, const DCsr& D, DCsr& C, Slots& S,
                             const int* brep = nullptr) {
    if (A.nc != B.nr) throw Error(MGR_ERR_ARG, "spgemm: inner dimensions differ");
    j.A = &A;
    j.B = &B;
    j.D = &D;
    j.C = &C;
    j.cnt.alloc((size_t)A.nr + 1, S.s);
    j.lr = S.take(1);
    j.brep = brep;
    spgemm_add_count(A, B, D, j.cnt.p, reinterpret_cast<int*>(j.lr), S.s, true, brep);
    j.pend = csr_begin(C, A.nr, B.nc, j.cnt.p, S);
}

// The transfer products with the block-diagonal M (side 1: M A_FC, counted by
// blocks and filled by the hashed kernel; side 2: A_CF M, by rows and runs).
static void bdiag_begin(Spgemm& j, int side, const DCsr& A, const DCsr& B, DCsr& C, int nb, const int* bstart,
                        Slots& S) {
    if (A.nc != B.nr) throw Error(MGR_ERR_ARG, "spgemm: inner dimensions differ");
    j.A = &A;
    j.B = &B;
    j.C = &C;
    j.bdiag = side;
    j.cnt.alloc((size_t)A.nr + 1, S.s);
    j.lr = S.take(1);
    if (side == 1) bdiag_left_count(nb, bstart, B, j.cnt.p, reinterpret_cast<int*>(j.lr), S.s);
    else bdiag_right_count(A, B, j.cnt.p, reinterpret_cast<int*>(j.lr), S.s);
    j.pend = csr_begin(C, A.nr, B.nc, j.cnt.p, S);
}

// After the sync that read the job's slot: C's row pointers and arrays
// (spgemm_alloc), then the numeric pass on stream st (spgemm_fillpass), which
// may be another stream than the slots' when C is read only there.
static void spgemm_alloc(Spgemm& j, Slots& S) {
    const long long v = S.val(j.lr);
    if (j.bdiag) {
        if (v != 0) throw Error(MGR_ERR_ARG, "internal: block-diagonal product outside its row bounds");
        csr_finish(j.pend, S);
    } else if (v == 2) {
        spgemm_recount(j, S.s);
    } else {
        if (v != 0) throw Error(MGR_ERR_ARG, "internal: spgemm row longer than its recorded length");
        csr_finish(j.pend, S);
    }
    j.cnt.reset();
}

struct FillPass {
    const DCsr* A = nullptr;
    const DCsr* B = nullptr;
    const DCsr* D = nullptr;
    DCsr* C = nullptr;
    int bdiag = 0;
    bool neg = false;
    const int* brep = nullptr;
    void run(int* flag, hipStream_t st) const {
        if (bdiag == 2) bdiag_right_fill(*A, *B, *C, flag, st);
        else if (D) spgemm_add_fill(*A, *B, *D, *C, flag, st, brep);
        else spgemm_fill(*A, *B, A->max_row, *C, flag, st, neg);
    }
};
static FillPass fill_pass(const Spgemm& j) { return FillPass{j.A, j.B, j.D, j.C, j.bdiag, j.neg, j.brep}; }

static void spgemm_fillpass(const Spgemm& j, Slots& S, hipStream_t st) { fill_pass(j).run(S.flag(), st); }

static void spgemm_finish(Spgemm& j, Slots& S) {
    spgemm_alloc(j, S);
    spgemm_fillpass(j, S, S.s);
}

static DCsr spgemm(const DCsr& A, const DCsr& B, Slots& S) {
    DCsr C;
    Spgemm j;
    spgemm_begin(j, A, B, C, S);
    S.sync("SpGEMM");
    spgemm_finish(j, S);
    return C;
}

static DCsr csr_add(const DCsr& A, const DCsr& B, Slots& S) {
    DArr<int> cnt((size_t)A.nr + 1, S.s);
    add_count(A, B, cnt.p, S.s);
    DCsr C = csr_from_counts(A.nr, A.nc, cnt.p, S, "sparse add");
    add_fill(A, B, C, S.s);
    return C;
}

// Transpose: the entry count is known, so no sync is needed; the longest row of
// the result is recorded in a slot (read at the caller's next sync point).
struct Transp {
    DCsr* T = nullptr;
    long long* slot = nullptr;
};

static Transp csr_transpose_begin(const DCsr& A, DCsr& T, Slots& S) {
    hipStream_t s = S.s;
    DArr<int> cnt((size_t)A.nc + 1, s);
    fill_int(cnt.p, 0, A.nc + 1, s);
    transpose_count(A, cnt.p, s);
    T = DCsr();
    T.nr = A.nc;
    T.nc = A.nr;
    T.nnz = A.nnz;
    T.rp.alloc((size_t)A.nc + 1, s);
    Transp t{&T, S.take(2)};
    scan_async(cnt.p, T.rp.p, A.nc, t.slot, s);
    T.ci.alloc((size_t)(A.nnz > 0 ? A.nnz : 1), s);
    T.v.alloc((size_t)(A.nnz > 0 ? A.nnz : 1), s);
    transpose_fill(A, T, cnt.p, s);   // consumes the column counts
    return t;
}

static void csr_transpose_finish(const Transp& t, Slots& S) { t.T->max_row = (int)S.val(t.slot + 1); }

static DCsr csr_transpose(const DCsr& A, Slots& S) {
    DCsr T;
    Transp t = csr_transpose_begin(A, T, S);
    S.sync("transpose");
    csr_transpose_finish(t, S);
    return T;
}

static DCsr csr_copy(const DCsr& A, hipStream_t s) {
    DCsr C;
    C.alloc(A.nr, A.nc, A.nnz, s);
    MGR_HIP(hipMemcpyAsync(C.rp.p, A.rp.p, sizeof(int) * ((size_t)A.nr + 1), hipMemcpyDeviceToDevice, s));
    if (A.nnz > 0) {
        MGR_HIP(hipMemcpyAsync(C.ci.p, A.ci.p, sizeof(int) * A.nnz, hipMemcpyDeviceToDevice, s));
        MGR_HIP(hipMemcpyAsync(C.v.p, A.v.p, sizeof(double) * A.nnz, hipMemcpyDeviceToDevice, s));
    }
    C.max_row = A.max_row;
    return C;
}

static void make_float(DCsr& A, hipStream_t s) {
    if (A.vf.p || A.nr == 0) return;
    A.vf.alloc((size_t)(A.nnz > 0 ? A.nnz : 1), s);
    to_float(A.v.p, A.vf.p, A.nnz, s);
}

// FP32 conversions gathered and issued F32_SEGS arrays per launch (a
// hierarchy's small operators would each cost a dependent launch otherwise);
// the destinations are taken on the owning stream, flush converts on `run`.
struct F32Batch {
    std::vector<const double*> src;
    std::vector<float*> dst;
    std::vector<long> n;
    void add(const double* a, float* b, long k) {
        if (k <= 0) return;
        src.push_back(a);
        dst.push_back(b);
        n.push_back(k);
    }
    void flush(hipStream_t run) {
        for (size_t i = 0; i < src.size(); i += F32_SEGS) {
            const int k = (int)std::min(src.size() - i, (size_t)F32_SEGS);
            to_float_batch(k, src.data() + i, dst.data() + i, n.data() + i, run);
        }
        src.clear();
        dst.clear();
        n.clear();
    }
};

static void make_float_on(DCsr& A, hipStream_t s, F32Batch& fb) {
    if (A.vf.p || A.nr == 0) return;
    A.vf.alloc((size_t)(A.nnz > 0 ? A.nnz : 1), s);
    fb.add(A.v.p, A.vf.p, A.nnz);
}

// ====================================================================== AMG
// Slot tables of the in-chunk entries of a hybrid Gauss-Seidel operator on one
// side of the diagonal (see hgs_tri_fill): w slots per row.
struct HgsTri {
    int w = 0;
    DArr<unsigned char> c;
    DArr<double> v;
    DArr<float> vf;
    void reset() {
        w = 0;
        c.reset();
        v.reset();
        vf.reset();
    }
};

struct AmgLevel {
    int n = 0;
    DCsr A, P, R, AT;        // R = P^T; AT = A^T for the transposed cycle
    // composed form of a V(1,1) level: b_c = G b, x = [W | Q] [b; x_c]; the
    // transposed cycle uses b_c = Q^T b, x = [W^T | G^T] [b; x_c]
    bool composed = false;
    DCsr G, W, Q, WQ, Qt, WGt;
    DCsr AP, RA;             // setup temporaries of the composed form
    long long* bad = nullptr;
    DArr<int> cf, label;
    DArr<double> dinv;
    DArr<float> dinvf;
    DArr<double> rd, td, bd, xd, sd;   // sd = D^-1 b, formed by the restriction from the level above
    DArr<float> rf, tf, bf, xf, sf;
    // hybrid L1 Gauss-Seidel: chunked L1 diagonal (row order, and in the
    // chunk-position layout of the slot tables, nchp chunks), the diagonal's
    // position in each row of A and of A^T, and the in-chunk triangles of A
    // (lo: forward sweeps, up: backward sweeps) and of A^T; wslot, wslotT:
    // the pending table widths
    DArr<double> dgs, dT;
    DArr<float> dTf;
    DArr<int> dpos, dposT;
    HgsTri lo, up, loT, upT;
    int nchp = 0;
    long long* wslot = nullptr;
};

struct Amg {
    std::vector<AmgLevel> lv;
    DArr<double> cinv, cinvT;
    DArr<float> cinvf, cinvTf;
    // the level above the coarsest when composed: its whole cycle as one dense
    // n x n operator T = W + Q C^-1 G (tail = its index, -1 if none)
    int tail = -1;
    DArr<double> td, tdT;
    DArr<float> tdf, tdTf;
    int nc = 0, nu_pre = 1, nu_post = 1;
    int smoother = MGR_SMOOTH_L1_JACOBI, chunk = 1;
    bool have_float = false, have_trans = false;
};

// Levels whose matrix has at most this many entries (and at most
// SPGEMM_DENSE_COLS rows, so that R A is a cheap product) are applied in
// composed form: there a launch costs more than the extra entries the composed
// operators read.
constexpr long AMG_COMPOSE_NNZ = 1L << 20;

// Forms W, Q = P - D^-1 (A P) (in place over A P) and G = R - (R A) D^-1 (in
// place over R A) and [W | Q]; validity is read back at the next sync.
static void amg_compose_begin(AmgLevel& L, Slots& S) {
    hipStream_t s = S.s;
    L.bad = S.take(1);
    int* bad = reinterpret_cast<int*>(L.bad);
    L.W = csr_copy(L.A, s);
    compose_w(L.A, L.dinv.p, L.W.v.p, bad, s);
    compose_sub(L.P, L.AP, L.dinv.p, nullptr, L.AP.v.p, bad, s);
    L.Q = std::move(L.AP);
    compose_sub(L.R, L.RA, nullptr, L.dinv.p, L.RA.v.p, bad, s);
    L.G = std::move(L.RA);
    concat_rows(L.W, L.Q, L.WQ, s);
}

static void amg_compose_finish(AmgLevel& L, Slots& S) {
    if (S.val(L.bad) != 0) {
        // a row without a stored diagonal: keep the plain four-SpMV form
        L.composed = false;
        L.G = DCsr();
        L.W = DCsr();
        L.Q = DCsr();
        L.WQ = DCsr();
    }
    L.bad = nullptr;
}

// The cycle of the last level above the coarsest, when applied in composed
// form (b_c = G b, x_c = C^-1 b_c, x = W b + Q x_c), is the linear map
// T = W + Q C^-1 G; for small levels it is formed densely once and applied as
// one GEMV, so three dependent launches become one.
constexpr int AMG_TAIL_MAX = 1024;
static void amg_make_tail(Amg& H, hipStream_t s) {
    H.tail = -1;
    H.td.reset(); H.tdT.reset(); H.tdf.reset(); H.tdTf.reset();
    const int L = (int)H.lv.size() - 2;
    if (L < 0 || !H.lv[L].composed || H.lv[L].n > AMG_TAIL_MAX) return;
    AmgLevel& Lv = H.lv[L];
    const int n = Lv.n, nc = H.nc;
    DArr<double> gd((size_t)nc * n + 1, s), x((size_t)nc * n + 1, s);
    densify(Lv.G, gd.p, s);
    dense_gemm(nc, nc, n, H.cinv.p, gd.p, x.p, s);
    H.td.alloc((size_t)n * n + 1, s);
    densify(Lv.W, H.td.p, s);
    sparse_dense_add(Lv.Q, x.p, n, H.td.p, s);
    H.tail = L;
}

// Hybrid L1 Gauss-Seidel data of every level but the coarsest: the chunked L1
// diagonal (from the current values), the diagonal positions (validity read
// back at the next sync) and the widths of the in-chunk triangles (read at the
// next sync by amg_hgs_finish, which makes the slot tables).
static void amg_hgs_setup(Amg& H, Slots& S) {
    hipStream_t s = S.s;
    for (size_t l = 0; l + 1 < H.lv.size(); ++l) {
        AmgLevel& L = H.lv[l];
        L.dgs.alloc((size_t)L.n + 1, s);
        hgs_diag(L.A, H.chunk, L.dgs.p, S.flag(), s);
        if (!L.dpos.p) {
            L.dpos.alloc((size_t)L.n + 1, s);
            diag_pos(L.A, L.dpos.p, S.flag(), s);
        }
        L.lo.reset();
        L.up.reset();
        L.dT.reset();
        L.dTf.reset();
        L.wslot = S.take(1);
        hgs_tri_count(L.A, L.dpos.p, H.chunk, reinterpret_cast<int*>(L.wslot), s);
    }
}

static int hgs_nchp(int n, int chunk) { return (int)((((long)n + chunk - 1) / chunk + 63) / 64 * 64); }

// The slot tables of one operator (A, or A^T with its own diagonal positions)
// from the widths read back in the slot; dT is written when given.
static void hgs_make_tables(const DCsr& A, const int* dpos, const double* d, int chunk, int nchp, long long wv,
                            HgsTri& lo, HgsTri& up, double* dT, hipStream_t s) {
    lo.w = (int)(wv & 0xffffffffLL);
    up.w = (int)(wv >> 32);
    const size_t per = (size_t)chunk * nchp;
    lo.c.alloc(per * lo.w + 1, s);
    lo.v.alloc(per * lo.w + 1, s);
    up.c.alloc(per * up.w + 1, s);
    up.v.alloc(per * up.w + 1, s);
    hgs_tri_fill(A, dpos, d, chunk, nchp, lo.w, lo.c.p, lo.v.p, up.w, up.c.p, up.v.p, dT, s);
}

static void amg_hgs_finish(Amg& H, Slots& S) {
    hipStream_t s = S.s;
    for (size_t l = 0; l + 1 < H.lv.size(); ++l) {
        AmgLevel& L = H.lv[l];
        L.nchp = hgs_nchp(L.n, H.chunk);
        L.dT.alloc((size_t)H.chunk * L.nchp, s);
        hgs_make_tables(L.A, L.dpos.p, L.dgs.p, H.chunk, L.nchp, S.val(L.wslot), L.lo, L.up, L.dT.p, s);
        L.wslot = nullptr;
    }
}

constexpr int PMIS_SMALL_N = 8192;

// PMIS to completion on a strength graph (srp, sci) with measures lam and the
// random stream of `level`; cf gets +1 = C / -1 = F.  Host checks every four
// rounds, after a first batch of eight (four on levels of at most
// PMIS_SMALL_N points, which finish in about three rounds: rounds after the
// last undecided point is settled change nothing, so the split is the same).
static void pmis_run(int n, const int* srp, const int* sci, const int* lam, uint64_t seed, int level, DArr<int>& cf,
                     int avg_row, Slots& S) {
    hipStream_t s = S.s;
    DArr<double> w((size_t)n + 1, s);
    DArr<int> cf2((size_t)n + 1, s);
    DArr<unsigned char> bt((size_t)n + 1, s), bt2((size_t)n + 1, s);
    cf.alloc((size_t)n + 1, s);
    pmis_init(n, lam, seed, level, w.p, cf.p, s);
    fill_bytes(bt.p, 0, n, s);
    for (int total = 0, batch = n <= PMIS_SMALL_N ? 4 : 8;; total += batch, batch = 4) {
        if (total > 100000) throw Error(MGR_ERR_UNSUPPORTED, "PMIS did not terminate");
        long long* und = S.take(1);
        for (int r = 0; r < batch; ++r) {
            pmis_select(n, srp, sci, w.p, cf.p, bt.p, avg_row, s);
            pmis_update(n, srp, sci, cf.p, bt.p, cf2.p, bt2.p, r + 1 == batch ? reinterpret_cast<int*>(und) : nullptr,
                        avg_row, s);
            std::swap(cf, cf2);
            std::swap(bt, bt2);
        }
        S.sync("PMIS");
        if ((S.val(und) & 0xffffffffLL) == 0) break;
    }
}

// Aggressive coarsening of one level (Stueben 2001; the first level of the
// mechanics AMG, Sec. 4.1): PMIS on S gives C1; PMIS again on the graph of C1
// points one or two strong connections apart (random stream level + 64,
// indexed by the position in C1) keeps the final C-points; interpolation by
// multiple passes of direct interpolation, each pass substituting the
// interpolation of the points reached before (P_i = sum_j w_ij P_j, as the
// product W P).  Fills cf (+1 / -1), isC, cidx (C numbering) and P; returns
// the number of C-points (P is left empty when that is 0).
static long amg_aggressive_level(const DCsr& A, const unsigned char* strong, const int* srp, const int* sci,
                                 const int* lam, uint64_t seed, int k, const int* label, DArr<int>& cf,
                                 DArr<int>& isC, DArr<int>& cidx, DCsr& P, Slots& S) {
    hipStream_t s = S.s;
    const int n = A.nr;
    const int avg_row = (int)((A.nnz + 2L * n - 1) / (2L * n));
    DArr<int> cf1;
    pmis_run(n, srp, sci, lam, seed, k, cf1, avg_row, S);
    // C1 numbering
    DArr<int> isC1((size_t)n + 1, s), e1((size_t)n + 1, s);
    cf_is_c(n, cf1.p, isC1.p, s);
    long long* s1 = S.take(2);
    scan_async(isC1.p, e1.p, n, s1, s);
    DArr<int> rtc((size_t)n + 1, s);
    agg_rt_count(n, srp, sci, isC1.p, rtc.p, s);
    DCsr Rt;
    Pend prt = csr_begin(Rt, n, 0, rtc.p, S);
    S.sync("aggressive coarsening: first C-points");
    const int n1 = (int)S.val(s1);
    csr_finish(prt, S);
    Rt.nc = n1;
    DArr<int> cf2;
    if (n1 > 0) {
        agg_rt_fill(n, srp, sci, isC1.p, e1.p, Rt, s);
        // the C1 points in order, and the rows of L
        DArr<int> pts((size_t)n1 + 1, s), lmap((size_t)n + 1, s), rest((size_t)n + 1, s), lc((size_t)n1 + 1, s);
        cf_maps(n, isC1.p, e1.p, lmap.p, pts.p, rest.p, s);
        agg_l_count(n1, pts.p, srp, lc.p, s);
        DCsr Lr = csr_from_counts(n1, n, lc.p, S, "aggressive coarsening: strong rows of C1");
        agg_l_fill(n1, pts.p, srp, sci, Lr, s);
        DCsr G2 = spgemm(Lr, Rt, S);
        Lr = DCsr();
        Rt = DCsr();
        DArr<int> gc((size_t)n1 + 1, s);
        nodiag_count(G2, gc.p, s);
        DCsr S2 = csr_from_counts(n1, n1, gc.p, S, "aggressive coarsening: second-order strength");
        nodiag_fill(G2, S2, s);
        G2 = DCsr();
        DArr<int> lam2((size_t)n1 + 1, s);
        fill_int(lam2.p, 0, n1 + 1, s);
        col_count(S2.nnz, S2.ci.p, lam2.p, s);
        const int avg2 = (int)((S2.nnz + n1 - 1) / (n1 > 0 ? n1 : 1));
        pmis_run(n1, S2.rp.p, S2.ci.p, lam2.p, seed, k + 64, cf2, avg2, S);
    }
    cf.alloc((size_t)n + 1, s);
    if (n1 > 0) agg_final(n, isC1.p, e1.p, cf2.p, cf.p, s);
    else fill_int(cf.p, -1, n, s);
    // final C numbering, then multi-pass interpolation
    cf_is_c(n, cf.p, isC.p, s);
    long long* sc = S.take(2);
    scan_async(isC.p, cidx.p, n, sc, s);
    DArr<int> pcnt((size_t)n + 1, s);
    interp_count(A, strong, cf.p, pcnt.p, s);
    Pend pp = csr_begin(P, n, 0, pcnt.p, S);
    S.sync("aggressive coarsening: final C-points");
    const long nc = (long)S.val(sc);
    if (nc == 0 || (double)nc > 0.9 * (double)n) {
        P = DCsr();
        return nc;
    }
    P.nc = (int)nc;
    csr_finish(pp, S);
    ensure_rowblocks(A);
    interp_fill(A, strong, cf.p, cidx.p, label, P, S.flag(), s);
    DArr<int> cfm((size_t)n + 1, s), wcnt((size_t)n + 1, s), ident((size_t)n + 1, s);
    iota_div(n, 1, ident.p, s);
    for (int pass = 2;; ++pass) {
        if (pass > n + 1) throw Error(MGR_ERR_UNSUPPORTED, "multi-pass interpolation did not terminate");
        mp_assigned(n, cf.p, P.rp.p, cfm.p, s);
        interp_count(A, strong, cfm.p, wcnt.p, s);
        long long* reach = S.take(1);
        mp_reach(n, cfm.p, wcnt.p, reach, s);
        DCsr Wp;
        Pend pw = csr_begin(Wp, n, n, wcnt.p, S);
        S.sync("multi-pass interpolation");
        if (S.val(reach) == 0) break;
        csr_finish(pw, S);
        interp_fill(A, strong, cfm.p, ident.p, label, Wp, S.flag(), s);
        P = spgemm(Wp, P, S);
        P.nc = (int)nc;
    }
    return nc;
}

// Classical AMG setup (the coarse solver of Sec. 4.1, with PMIS coarsening,
// direct interpolation and L1-Jacobi smoothing; see the oracle for the
// definitions): stops at n <= max_coarse, at max_levels, or when coarsening
// stalls (no C-point or n_c > 0.9 n).  The coarsest matrix is inverted densely.
// Host synchronisation: about three sync points per level.
static void amg_setup(Amg& H, DCsr A0, const int* label0, const mgr_amg_opts& o, uint64_t seed, Slots& S) {
    hipStream_t s = S.s;
    H.lv.clear();
    H.nu_pre = o.nu_pre;
    H.nu_post = o.nu_post;
    H.smoother = o.smoother;
    H.chunk = o.gs_chunk;
    H.lv.emplace_back();
    int n0 = A0.nr;
    H.lv[0].A = std::move(A0);
    H.lv[0].n = n0;
    if (label0) {
        H.lv[0].label.alloc((size_t)n0, s);
        MGR_HIP(hipMemcpyAsync(H.lv[0].label.p, label0, sizeof(int) * n0, hipMemcpyDeviceToDevice, s));
    }
    int k = 0;
    for (;;) {
        AmgLevel& L = H.lv[k];
        const DCsr& A = L.A;
        int n = A.nr;
        if (S.level_hook) S.level_hook(n);
        if (n <= o.max_coarse || k + 1 >= o.max_levels) break;
        size_t nz = (size_t)(A.nnz > 0 ? A.nnz : 1);
        DArr<unsigned char> strong(nz, s);
        DArr<int> scnt((size_t)n + 1, s), srp((size_t)n + 1, s);
        DArr<int> lam((size_t)n + 1, s);
        fill_int(lam.p, 0, n + 1, s);
        L.dinv.alloc((size_t)n, s);
        amg_strength(A, o.theta, L.label.p, strong.p, scnt.p, lam.p, L.dinv.p, S.flag(), s);
        // strength graph S (row i lists S_i)
        DArr<int> sci(nz, s);
        scan_exclusive_async(scnt.p, srp.p, n, s);
        strength_compact_fill(A, strong.p, srp.p, sci.p, s);
        DArr<int> cf((size_t)n, s), isC((size_t)n + 1, s), cidx((size_t)n + 1, s);
        DCsr P;
        long nc = 0;
        if (k < o.agg_levels) {
            nc = amg_aggressive_level(A, strong.p, srp.p, sci.p, lam.p, seed, k, L.label.p, cf, isC, cidx, P, S);
            if (nc == 0 || (double)nc > 0.9 * (double)n) break;
        } else {
        // PMIS rounds, run in batches between checks of the undecided count;
        // the state (cf, beaten) alternates between two buffers
        DArr<double> w((size_t)n, s);
        DArr<int> cf2((size_t)n, s), pcnt((size_t)n + 1, s);
        DArr<unsigned char> bt((size_t)n, s), bt2((size_t)n, s);
        pmis_init(n, lam.p, seed, k, w.p, cf.p, s);
        fill_bytes(bt.p, 0, n, s);
        Pend pp;
        long long* sc = nullptr;
        // seven rounds usually decide every point: a first batch of eight rarely
        // needs a second (each batch costs a sync and a speculative P count);
        // levels of at most PMIS_SMALL_N points take about three, so four
        int batch = n <= PMIS_SMALL_N ? 4 : 8;
        // strong rows hold about half of a row of A
        const int avg_row = (int)((A.nnz + 2L * n - 1) / (2L * n));
        for (int total = 0;; total += batch, batch = 4) {
            if (total > 100000) throw Error(MGR_ERR_UNSUPPORTED, "PMIS did not terminate");
            long long* und = S.take(1);
            for (int r = 0; r < batch; ++r) {
                pmis_select(n, srp.p, sci.p, w.p, cf.p, bt.p, avg_row, s);
                // the undecided points are counted after the last round of the batch
                pmis_update(n, srp.p, sci.p, cf.p, bt.p, cf2.p, bt2.p,
                            r + 1 == batch ? reinterpret_cast<int*>(und) : nullptr, avg_row, s);
                std::swap(cf, cf2);
                std::swap(bt, bt2);
            }
            // speculative: C numbering and interpolation row counts for this state
            cf_is_c(n, cf.p, isC.p, s);
            sc = S.take(2);
            scan_async(isC.p, cidx.p, n, sc, s);
            if (o.interp == MGR_INTERP_EXT_I) interp_ext_count(A, strong.p, cf.p, pcnt.p, S.flag(), s);
            else interp_count(A, strong.p, cf.p, pcnt.p, s);
            pp = csr_begin(P, n, 0, pcnt.p, S);
            S.sync("PMIS");
            if ((S.val(und) & 0xffffffffLL) == 0) break;
        }
        nc = (long)S.val(sc);
        if (nc == 0 || (double)nc > 0.9 * (double)n) break;
        P.nc = (int)nc;
        csr_finish(pp, S);
        ensure_rowblocks(A);
        if (o.interp == MGR_INTERP_EXT_I) interp_ext_fill(A, strong.p, cf.p, cidx.p, L.label.p, P, S.flag(), s);
        else interp_fill(A, strong.p, cf.p, cidx.p, L.label.p, P, S.flag(), s);
        }
        // R = P^T and A P, then P^T (A P)
        DCsr R, AP, Ac;
        Transp tr = csr_transpose_begin(P, R, S);
        Spgemm j1;
        spgemm_begin(j1, A, P, AP, S);
        S.sync("AMG interpolation");
        csr_transpose_finish(tr, S);
        spgemm_finish(j1, S);
        Spgemm j2, j3;
        spgemm_begin(j2, R, AP, Ac, S);
        // small V(1,1) L1-Jacobi levels are applied in composed form (two SpMVs instead of four)
        L.composed = H.smoother == MGR_SMOOTH_L1_JACOBI && H.nu_pre == 1 && H.nu_post == 1 &&
                     A.nnz <= AMG_COMPOSE_NNZ && n <= SPGEMM_DENSE_COLS;
        if (L.composed) spgemm_begin(j3, R, A, L.RA, S);
        S.sync("AMG Galerkin product");
        spgemm_finish(j2, S);
        if (L.composed) {
            spgemm_finish(j3, S);
            L.AP = std::move(AP);
        }
        AP = DCsr();
        L.P = std::move(P);
        L.R = std::move(R);
        L.cf = std::move(cf);
        AmgLevel next;
        next.n = (int)nc;
        next.A = std::move(Ac);
        if (L.label.p) {
            DArr<int> lmap((size_t)n, s), cmap((size_t)nc, s), dummy((size_t)n, s);
            cf_maps(n, isC.p, cidx.p, lmap.p, cmap.p, dummy.p, s);
            next.label.alloc((size_t)nc, s);
            gather_int((int)nc, cmap.p, L.label.p, next.label.p, s);
        }
        H.lv.push_back(std::move(next));
        ++k;
    }
    H.lv.back().composed = false;
    for (size_t l = 0; l + 1 < H.lv.size(); ++l)
        if (H.lv[l].composed) amg_compose_begin(H.lv[l], S);
    if (H.smoother == MGR_SMOOTH_HYBRID_GS) amg_hgs_setup(H, S);
    AmgLevel& Lc = H.lv.back();
    H.nc = Lc.n;
    if (H.nc > 2048) throw Error(MGR_ERR_UNSUPPORTED, "AMG: coarsest level has more than 2048 unknowns");
    int nc = H.nc;
    DArr<double> dense((size_t)nc * nc + 1, s);
    H.cinv.alloc((size_t)nc * nc + 1, s);
    densify(Lc.A, dense.p, s);
    dense_inverse(nc, dense.p, H.cinv.p, S.flag(), s);
    // work vectors
    for (size_t l = 0; l < H.lv.size(); ++l) {
        AmgLevel& L = H.lv[l];
        L.rd.alloc((size_t)L.n + 1, s);
        L.td.alloc((size_t)L.n + 1, s);
        L.sd.alloc((size_t)L.n + 1, s);
        if (l > 0) {
            L.bd.alloc((size_t)L.n + 1, s);
            L.xd.alloc((size_t)L.n + 1, s);
        }
    }
    S.sync("AMG coarsest inverse");
    for (size_t l = 0; l + 1 < H.lv.size(); ++l)
        if (H.lv[l].composed) amg_compose_finish(H.lv[l], S);
    if (H.smoother == MGR_SMOOTH_HYBRID_GS) amg_hgs_finish(H, S);
    amg_make_tail(H, s);
    H.have_float = false;
    H.have_trans = false;
}

// Setup reuse for new values of the level-0 matrix: C/F splits, labels,
// interpolation P and R = P^T of every level are kept; the Galerkin products
// A_{k+1} = P^T (A_k P), L1 diagonals, composed operators and the coarsest
// inverse are formed again (same products and order as amg_setup).
static void amg_refresh(Amg& H, DCsr A0, Slots& S) {
    hipStream_t s = S.s;
    if (H.lv.empty() || A0.nr != H.lv[0].n) throw Error(MGR_ERR_ARG, "AMG reuse: level-0 size changed");
    H.lv[0].A = std::move(A0);
    const int nl = (int)H.lv.size();
    for (int k = 0; k + 1 < nl; ++k) {
        AmgLevel& L = H.lv[k];
        if (S.level_hook) S.level_hook(L.n);
        L.AT = DCsr();
        L.dposT.reset();
        L.loT.reset();
        L.upT.reset();
        L.G = DCsr(); L.W = DCsr(); L.Q = DCsr(); L.WQ = DCsr(); L.Qt = DCsr(); L.WGt = DCsr();
        L.dinvf.reset();
        DCsr AP, Ac;
        Spgemm j1;
        spgemm_begin(j1, L.A, L.P, AP, S);
        S.sync("AMG Galerkin product");
        spgemm_finish(j1, S);
        Spgemm j2, j3;
        spgemm_begin(j2, L.R, AP, Ac, S);
        if (L.composed) spgemm_begin(j3, L.R, L.A, L.RA, S);
        L.dinv.alloc((size_t)L.n, s);
        l1_dinv(L.A, L.dinv.p, S.flag(), s);
        S.sync("AMG Galerkin product");
        spgemm_finish(j2, S);
        if (L.composed) {
            spgemm_finish(j3, S);
            L.AP = std::move(AP);
        }
        H.lv[k + 1].A = std::move(Ac);
    }
    H.lv.back().AT = DCsr();
    for (int k = 0; k + 1 < nl; ++k)
        if (H.lv[k].composed) amg_compose_begin(H.lv[k], S);
    if (H.smoother == MGR_SMOOTH_HYBRID_GS) amg_hgs_setup(H, S);
    int nc = H.nc;
    DArr<double> dense((size_t)nc * nc + 1, s);
    H.cinv.alloc((size_t)nc * nc + 1, s);
    densify(H.lv.back().A, dense.p, s);
    dense_inverse(nc, dense.p, H.cinv.p, S.flag(), s);
    S.sync("AMG coarsest inverse");
    for (int k = 0; k + 1 < nl; ++k)
        if (H.lv[k].composed) amg_compose_finish(H.lv[k], S);
    if (H.smoother == MGR_SMOOTH_HYBRID_GS) amg_hgs_finish(H, S);
    amg_make_tail(H, s);
    H.cinvT.reset();
    H.cinvf.reset();
    H.cinvTf.reset();
    H.have_float = false;
    H.have_trans = false;
}

// FP32 copies of the hierarchy: arrays taken on stream s, converted on run
// (s when null)
static void amg_make_float(Amg& H, hipStream_t s, F32Batch& fb) {
    if (H.have_float) return;
    for (size_t l = 0; l < H.lv.size(); ++l) {
        AmgLevel& L = H.lv[l];
        if (L.composed) {
            make_float_on(L.G, s, fb);
            make_float_on(L.WQ, s, fb);
            if (H.have_trans) {
                make_float_on(L.Qt, s, fb);
                make_float_on(L.WGt, s, fb);
            }
        } else {
            make_float_on(L.A, s, fb);
        }
        if (l + 1 < H.lv.size() && !L.composed) {
            make_float_on(L.P, s, fb);
            make_float_on(L.R, s, fb);
            L.dinvf.alloc((size_t)L.n, s);
            fb.add(L.dinv.p, L.dinvf.p, L.n);
            if (L.dT.p) {
                const long per = (long)H.chunk * L.nchp;
                L.dTf.alloc((size_t)per, s);
                fb.add(L.dT.p, L.dTf.p, per);
                for (HgsTri* t : {&L.lo, &L.up, &L.loT, &L.upT}) {
                    if (!t->v.p) continue;
                    t->vf.alloc(t->v.n, s);
                    fb.add(t->v.p, t->vf.p, per * t->w);
                }
            }
        }
        if (H.have_trans && L.AT.nr && !L.composed) make_float_on(L.AT, s, fb);
        L.rf.alloc((size_t)L.n + 1, s);
        L.tf.alloc((size_t)L.n + 1, s);
        L.sf.alloc((size_t)L.n + 1, s);
        if (l > 0) {
            L.bf.alloc((size_t)L.n + 1, s);
            L.xf.alloc((size_t)L.n + 1, s);
        }
    }
    long nn = (long)H.nc * H.nc;
    H.cinvf.alloc((size_t)nn + 1, s);
    fb.add(H.cinv.p, H.cinvf.p, nn);
    if (H.have_trans) {
        H.cinvTf.alloc((size_t)nn + 1, s);
        fb.add(H.cinvT.p, H.cinvTf.p, nn);
    }
    if (H.tail >= 0) {
        const long tn = (long)H.lv[H.tail].n * H.lv[H.tail].n;
        H.tdf.alloc((size_t)tn + 1, s);
        fb.add(H.td.p, H.tdf.p, tn);
        if (H.have_trans) {
            H.tdTf.alloc((size_t)tn + 1, s);
            fb.add(H.tdT.p, H.tdTf.p, tn);
        }
    }
    H.have_float = true;
}

static void amg_make_trans(Amg& H, Slots& S) {
    hipStream_t s = S.s;
    if (H.have_trans) return;
    for (size_t l = 0; l + 1 < H.lv.size(); ++l) {
        AmgLevel& L = H.lv[l];
        if (L.composed) {
            DCsr Wt, Gt;
            Transp t1 = csr_transpose_begin(L.Q, L.Qt, S);
            Transp t2 = csr_transpose_begin(L.W, Wt, S);
            Transp t3 = csr_transpose_begin(L.G, Gt, S);
            S.sync("transpose of a composed level");
            csr_transpose_finish(t1, S);
            csr_transpose_finish(t2, S);
            csr_transpose_finish(t3, S);
            concat_rows(Wt, Gt, L.WGt, s);
            if (H.have_float) {
                make_float(L.Qt, s);
                make_float(L.WGt, s);
            }
            continue;
        }
        L.AT = csr_transpose(L.A, S);
        if (H.have_float) make_float(L.AT, s);
    }
    if (H.smoother == MGR_SMOOTH_HYBRID_GS) {
        // the widths of every level counted after the last transpose's sync,
        // so that one sync reads them all
        for (size_t l = 0; l + 1 < H.lv.size(); ++l) {
            AmgLevel& L = H.lv[l];
            if (L.composed) continue;
            // A^T keeps every diagonal entry of A
            L.dposT.alloc((size_t)L.n + 1, s);
            diag_pos(L.AT, L.dposT.p, S.flag(), s);
            L.wslot = S.take(1);
            hgs_tri_count(L.AT, L.dposT.p, H.chunk, reinterpret_cast<int*>(L.wslot), s);
        }
        // the transposed sweeps use A's diagonal d, so dT is shared
        S.sync("hybrid Gauss-Seidel tables of A^T");
        for (size_t l = 0; l + 1 < H.lv.size(); ++l) {
            AmgLevel& L = H.lv[l];
            if (!L.wslot) continue;
            hgs_make_tables(L.AT, L.dposT.p, L.dgs.p, H.chunk, L.nchp, S.val(L.wslot), L.loT, L.upT, nullptr, s);
            L.wslot = nullptr;
            if (H.have_float) {
                const long per = (long)H.chunk * L.nchp;
                for (HgsTri* t : {&L.loT, &L.upT}) {
                    t->vf.alloc(t->v.n, s);
                    to_float(t->v.p, t->vf.p, per * t->w, s);
                }
            }
        }
    }
    int nc = H.nc;
    std::vector<double> h((size_t)nc * nc), t((size_t)nc * nc);
    MGR_HIP(hipMemcpyAsync(h.data(), H.cinv.p, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s));
    MGR_HIP(hipStreamSynchronize(s));
    for (int i = 0; i < nc; ++i)
        for (int j = 0; j < nc; ++j) t[(size_t)j * nc + i] = h[(size_t)i * nc + j];
    H.cinvT.alloc((size_t)nc * nc + 1, s);
    MGR_HIP(hipMemcpyAsync(H.cinvT.p, t.data(), sizeof(double) * t.size(), hipMemcpyHostToDevice, s));
    if (H.have_float) {
        H.cinvTf.alloc((size_t)nc * nc + 1, s);
        to_float(H.cinvT.p, H.cinvTf.p, (long)nc * nc, s);
    }
    if (H.tail >= 0) {
        const int tn = H.lv[H.tail].n;
        H.tdT.alloc((size_t)tn * tn + 1, s);
        dense_transpose(tn, H.td.p, H.tdT.p, s);
        if (H.have_float) {
            H.tdTf.alloc((size_t)tn * tn + 1, s);
            to_float(H.tdT.p, H.tdTf.p, (long)tn * tn, s);
        }
    }
    MGR_HIP(hipStreamSynchronize(s));
    H.have_trans = true;
}

template <typename T> struct Prec;
template <> struct Prec<double> {
    static double* r(AmgLevel& L) { return L.rd.p; }
    static double* t(AmgLevel& L) { return L.td.p; }
    static double* b(AmgLevel& L) { return L.bd.p; }
    static double* x(AmgLevel& L) { return L.xd.p; }
    static double* sb(AmgLevel& L) { return L.sd.p; }
    static const double* dinv(AmgLevel& L) { return L.dinv.p; }
    static const double* dT(AmgLevel& L) { return L.dT.p; }
    static const double* tv(const HgsTri& t) { return t.v.p; }
    static const double* cinv(Amg& H, bool tr) { return tr ? H.cinvT.p : H.cinv.p; }
    static const double* tail(Amg& H, bool tr) { return tr ? H.tdT.p : H.td.p; }
};
template <> struct Prec<float> {
    static float* r(AmgLevel& L) { return L.rf.p; }
    static float* t(AmgLevel& L) { return L.tf.p; }
    static float* b(AmgLevel& L) { return L.bf.p; }
    static float* x(AmgLevel& L) { return L.xf.p; }
    static float* sb(AmgLevel& L) { return L.sf.p; }
    static const float* dinv(AmgLevel& L) { return L.dinvf.p; }
    static const float* dT(AmgLevel& L) { return L.dTf.p; }
    static const float* tv(const HgsTri& t) { return t.vf.p; }
    static const float* cinv(Amg& H, bool tr) { return tr ? H.cinvTf.p : H.cinvf.p; }
    static const float* tail(Amg& H, bool tr) { return tr ? H.tdTf.p : H.tdf.p; }
};

// V(nu_pre, nu_post) cycle from x = 0 with L1-Jacobi smoothing; the transposed
// cycle uses A^T on every level, swaps the sweep counts and applies the
// transposed coarsest inverse (the exact adjoint of the forward cycle).  bd,
// when given, is D^-1 b of this level (formed by the restriction above it).
template <typename T>
static void amg_vcycle(Amg& H, int k, const T* b, T* x, bool tr, hipStream_t s, const T* bd = nullptr) {
    AmgLevel& L = H.lv[k];
    int n = L.n;
    if (k + 1 == (int)H.lv.size()) {
        dense_gemv<T, T>(n, Prec<T>::cinv(H, tr), b, x, s);
        return;
    }
    if (k == H.tail) {
        dense_gemv<T, T>(n, Prec<T>::tail(H, tr), b, x, s);
        return;
    }
    if (L.composed) {
        AmgLevel& Lc = H.lv[k + 1];
        T* bc = Prec<T>::b(Lc);
        T* xc = Prec<T>::x(Lc);
        spmv<T, T, T, T, T>(view<T>(tr ? L.Qt : L.G), b, (const T*)nullptr, INT_MAX, (const T*)nullptr, bc, T(1),
                            T(0), s);
        amg_vcycle<T>(H, k + 1, bc, xc, tr, s);
        spmv<T, T, T, T, T>(view<T>(tr ? L.WGt : L.WQ), b, xc, n, (const T*)nullptr, x, T(1), T(0), s);
        return;
    }
    SpOp<T> A = view<T>(tr ? L.AT : L.A);
    const T* dinv = Prec<T>::dinv(L);
    T* r = Prec<T>::r(L);
    T* t = Prec<T>::t(L);
    int npre = tr ? H.nu_post : H.nu_pre, npost = tr ? H.nu_pre : H.nu_post;
    if (H.smoother == MGR_SMOOTH_HYBRID_GS) {
        // forward sweeps down, backward sweeps up; the transposed cycle runs the
        // same directions on A^T (the transpose of a backward sweep on A is a
        // forward sweep on A^T) with A's row-based diagonal
        const T* dT = Prec<T>::dT(L);
        const HgsTri& fw = tr ? L.loT : L.lo;
        const HgsTri& bw = tr ? L.upT : L.up;
        if (npre >= 1) {
            hgs_tri<T>(n, H.chunk, fw.w, L.nchp, fw.c.p, Prec<T>::tv(fw), dT, b, x, false, true, s);
            for (int q = 1; q < npre; ++q) {
                spmv<T, T, T, T, T>(A, x, (const T*)nullptr, INT_MAX, b, t, T(-1), T(1), s);
                hgs_tri<T>(n, H.chunk, fw.w, L.nchp, fw.c.p, Prec<T>::tv(fw), dT, t, x, false, false, s);
            }
            spmv<T, T, T, T, T>(A, x, (const T*)nullptr, INT_MAX, b, r, T(-1), T(1), s);
        } else {
            set<T>(n, x, T(0), s);
            copy<T, T>(n, b, r, s);
        }
        AmgLevel& Lc = H.lv[k + 1];
        T* bc = Prec<T>::b(Lc);
        T* xc = Prec<T>::x(Lc);
        spmv<T, T, T, T, T>(view<T>(L.R), r, (const T*)nullptr, INT_MAX, (const T*)nullptr, bc, T(1), T(0), s);
        amg_vcycle<T>(H, k + 1, bc, xc, tr, s);
        spmv<T, T, T, T, T>(view<T>(L.P), xc, (const T*)nullptr, INT_MAX, x, x, T(1), T(1), s);
        for (int q = 0; q < npost; ++q) {
            spmv<T, T, T, T, T>(A, x, (const T*)nullptr, INT_MAX, b, t, T(-1), T(1), s);
            hgs_tri<T>(n, H.chunk, bw.w, L.nchp, bw.c.p, Prec<T>::tv(bw), dT, t, x, true, false, s);
        }
        return;
    }
    if (npre >= 1) {
        if (bd) presmooth_scaled<T>(A, bd, b, x, r, s);
        else presmooth<T>(A, dinv, b, x, r, s);
        if (npre > 1) {
            for (int q = 1; q < npre; ++q) {
                jacobi_sweep<T>(A, dinv, b, x, t, s);
                copy<T, T>(n, t, x, s);
            }
            spmv<T, T, T, T, T>(A, x, (const T*)nullptr, INT_MAX, b, r, T(-1), T(1), s);
        }
    } else {
        set<T>(n, x, T(0), s);
        copy<T, T>(n, b, r, s);
    }
    AmgLevel& Lc = H.lv[k + 1];
    T* bc = Prec<T>::b(Lc);
    T* xc = Prec<T>::x(Lc);
    // a plain (not composed, not coarsest) next level gets D^-1 b_c from the restriction
    if (npre >= 1 && !Lc.composed && k + 2 < (int)H.lv.size()) {
        T* sc = Prec<T>::sb(Lc);
        restrict_scaled<T, T>(view<T>(L.R), r, Prec<T>::dinv(Lc), bc, sc, s);
        amg_vcycle<T>(H, k + 1, bc, xc, tr, s, sc);
    } else {
        spmv<T, T, T, T, T>(view<T>(L.R), r, (const T*)nullptr, INT_MAX, (const T*)nullptr, bc, T(1), T(0), s);
        amg_vcycle<T>(H, k + 1, bc, xc, tr, s);
    }
    SpOp<T> P = view<T>(L.P);
    if (npost == 0) {
        spmv<T, T, T, T, T>(P, xc, (const T*)nullptr, INT_MAX, x, x, T(1), T(1), s);
        return;
    }
    // prolongate into the buffer from which an odd/even number of out-of-place
    // sweeps ends in x
    T* src = (npost % 2 == 1) ? t : x;
    spmv<T, T, T, T, T>(P, xc, (const T*)nullptr, INT_MAX, x, src, T(1), T(1), s);
    T* other = (src == x) ? t : x;
    for (int q = 0; q < npost; ++q) {
        jacobi_sweep<T>(A, dinv, b, src, other, s);
        std::swap(src, other);
    }
}

// ====================================================================== triangular schedules
// Rows of a triangular matrix grouped by dependency level (rows of one level
// are independent once the earlier levels are solved).
struct Sched {
    DArr<int> order;           // rows, level by level
    std::vector<int> off;      // level offsets into order (host), nlev + 1
};

static Sched level_schedule(const DCsr& T, bool fwd, Slots& S) {
    hipStream_t s = S.s;
    int n = T.nr;
    Sched sc;
    DArr<int> lev((size_t)n + 1, s);
    fill_int(lev.p, 0, n + 1, s);
    for (int it = 0;; it += 8) {
        if (it > 8 * (n + 8)) throw Error(MGR_ERR_UNSUPPORTED, "level analysis did not converge");
        long long* ch = S.take(1);
        for (int q = 0; q < 8; ++q) level_sweep(T, fwd, lev.p, reinterpret_cast<int*>(ch), s);
        S.sync("level analysis");
        if (S.val(ch) == 0) break;
    }
    long long* mx = S.take(1);
    level_max(n, lev.p, reinterpret_cast<int*>(mx), s);
    S.sync("level analysis");
    int nlev = (int)(S.val(mx) & 0xffffffffLL) + 1;
    DArr<int> cnt((size_t)nlev + 1, s), off((size_t)nlev + 1, s), cursor((size_t)nlev + 1, s);
    fill_int(cnt.p, 0, nlev + 1, s);
    level_bucket(n, lev.p, cnt.p, nullptr, nullptr, s, false);
    scan_exclusive_async(cnt.p, off.p, nlev, s);
    MGR_HIP(hipMemcpyAsync(cursor.p, off.p, sizeof(int) * ((size_t)nlev + 1), hipMemcpyDeviceToDevice, s));
    sc.order.alloc((size_t)n + 1, s);
    level_bucket(n, lev.p, nullptr, cursor.p, sc.order.p, s, true);
    sc.off.resize((size_t)nlev + 1);
    MGR_HIP(hipMemcpyAsync(sc.off.data(), off.p, sizeof(int) * ((size_t)nlev + 1), hipMemcpyDeviceToHost, s));
    MGR_HIP(hipStreamSynchronize(s));
    return sc;
}

template <typename T>
static void trsv(const Sched& sc, const DCsr& A, const T* b, T* x, bool unit, hipStream_t s) {
    SpOp<T> op = view<T>(A);
    for (size_t k = 0; k + 1 < sc.off.size(); ++k)
        trsv_level<T>(sc.off[k + 1] - sc.off[k], sc.order.p + sc.off[k], op, b, x, unit, s);
}

// ====================================================================== MGR levels
struct MgrLevel {
    int n = 0, nF = 0, nC = 0;
    mgr_level_opts o{};
    bool fused = false;
    DArr<int> isF, lmap, fmap, cmap;
    DCsr AFF, AFC, ACF, ACC, M, PF, RF, W;   // W = A_CF M
    DCsr RJ, PJ, RJt, PJt;                   // operators of the fused one-sweep apply
    DCsr Aout;                               // coarse operator (input of the next level; the
                                             // last level's is owned by the coarse AMG)
    DCsr AFFt, ACFt, PFt, RFt, Mt;           // general transposed apply
    bool have_float = false, have_trans = false;
    bool aff_partial = false;                // AFF holds only the F-relaxation blocks
    std::unique_ptr<Amg> famg;
    // ILU(0) F-relaxation: L (unit, strict lower), U (diagonal + upper), their
    // transposes, and the level schedules of the four triangular solves
    DCsr iluL, iluU, iluLt, iluUt;
    Sched schL, schU, schLt, schUt;
    // level vectors: coarse input / output (the next level's v and z)
    DArr<double> rcd, ecd, vFd, vCd, zFd, rFd, tFd;
    DArr<float> rcf, ecf, vFf, vCf, zFf, rFf, tFf;
    DArr<float> vinf;   // FP32 apply, first fused level: the input v in FP32
};

struct Ctx {
    // declared first so that it is destroyed last, after every array has
    // returned its block
    BlockCache cache;
    hipStream_t s = nullptr;
    mgr_opts o{};
    std::string err;
    bool ready = false;
    int b = 1, nbr = 0, n = 0;
    long nnzb = 0;
    DArr<int> Arp, Aci, ATrp, ATci;
    DArr<double> Av, ATv;
    DCsr A0, A0t;      // scalar level-0 operator (b = 1: the CSR input)
    bool have_At = false;
    std::vector<MgrLevel> L;
    Amg camg;
    Slots slots;
    // setup inputs kept for mgr_update_values: field labels and level options,
    // and the labels' histogram (pinned; it sizes every level's F and C sets)
    DArr<int> field0, fhist;
    DArr<int> block0;   // block-Jacobi group of every unknown (empty: its block row)
    int* fhist_h = nullptr;
    std::vector<mgr_level_opts> lvl;
    // hierarchies handed from the previous setup to the one being formed
    std::vector<std::unique_ptr<Amg>> reuse_famg;
    std::unique_ptr<Amg> reuse_camg;
    bool reuse_keep_famg = false;
    // Krylov workspace
    int kr_m = 0;
    long kr_n = 0;
    DArr<double> V, Z, hbuf, part, yd;
    DArr<double> apply_tmp;
    // no-allocation apply: whether a forward / transposed apply has run on the
    // current hierarchy (every operator copy it reads then exists), this
    // device's scratch array, and room for the work-vector addresses it swaps
    bool warm[2] = {false, false};
    unsigned char* scratch = nullptr;
    std::vector<std::pair<DArr<double>*, double*>> saved_d;
    std::vector<std::pair<DArr<float>*, float*>> saved_f;
    // pinned copies of the Arnoldi coefficients, one row of HROW per
    // iteration, each ending in a ready flag that the kernel sets last
    static constexpr int HROW = 200;
    double* hpin = nullptr;
    double* hpin_dev = nullptr;  // the same rows as seen by kernels
    // auxiliary stream (default priority) for setup work off its critical
    // path -- the copy of the input values, the fused-apply operators R_J and
    // P_J -- forked from s and joined back into s before the setup returns
    // (also when it fails); Avin: the input values the setup reads meanwhile
    // (the caller's array, while the copy is in flight)
    hipStream_t aux = nullptr;
    hipEvent_t ev_fork = nullptr, ev_join = nullptr;
    bool aux_pending = false;
    const double* Avin = nullptr;
    // the copy of the input values is made by the first block extraction (a
    // block input with MGR levels) instead of a separate copy
    bool copy_in_extract = false;
    // setup work for the auxiliary stream held back until the coarse AMG
    // reaches its smaller levels, one piece per level (run_deferred)
    std::vector<std::function<void()>> deferred;
    size_t deferred_next = 0;
    ~Ctx() {
        if (aux) {
            (void)hipStreamSynchronize(aux);
            (void)hipStreamDestroy(aux);
        }
        if (ev_fork) (void)hipEventDestroy(ev_fork);
        if (ev_join) (void)hipEventDestroy(ev_join);
        if (hpin) (void)hipHostFree(hpin);
        if (fhist_h) (void)hipHostFree(fhist_h);
    }
};

// Work enqueued on c.aux after aux_fork runs after everything enqueued on
// c.s so far; after aux_join, work on c.s runs after everything on c.aux.
static void aux_fork(Ctx& c) {
    if (!c.aux) {
        MGR_HIP(hipStreamCreateWithFlags(&c.aux, hipStreamNonBlocking));
        MGR_HIP(hipEventCreateWithFlags(&c.ev_fork, hipEventDisableTiming));
        MGR_HIP(hipEventCreateWithFlags(&c.ev_join, hipEventDisableTiming));
    }
    MGR_HIP(hipEventRecord(c.ev_fork, c.s));
    MGR_HIP(hipStreamWaitEvent(c.aux, c.ev_fork, 0));
    c.aux_pending = true;
}

static void aux_join(Ctx& c) {
    if (!c.aux_pending) return;
    c.aux_pending = false;
    MGR_HIP(hipEventRecord(c.ev_join, c.aux));
    MGR_HIP(hipStreamWaitEvent(c.s, c.ev_join, 0));
}

// Joins the auxiliary stream at the end of a setup call, however it ends, so
// that no array of the handle is reused while work on c.aux may still touch it,
// and forgets the caller's input values.
struct AuxScope {
    Ctx& c;
    ~AuxScope() {
        if (c.aux_pending) {
            c.aux_pending = false;
            (void)hipEventRecord(c.ev_join, c.aux);
            (void)hipStreamWaitEvent(c.s, c.ev_join, 0);
        }
        c.Avin = nullptr;
        c.copy_in_extract = false;
        c.deferred.clear();
        c.deferred_next = 0;
        c.slots.level_hook = nullptr;
    }
};

// Held-back work, on the auxiliary stream after everything enqueued so far:
// the next `pieces` pieces (all with pieces < 0).  Spread over the AMG's
// smaller levels, whose own kernels are latency-bound, it slows them less
// than all at once.
static void run_deferred(Ctx& c, int pieces = -1) {
    if (c.deferred_next >= c.deferred.size()) return;
    aux_fork(c);
    for (; c.deferred_next < c.deferred.size() && pieces != 0; --pieces) c.deferred[c.deferred_next++]();
    if (c.deferred_next >= c.deferred.size()) {
        c.deferred.clear();
        c.deferred_next = 0;
    }
}

// the block values a setup step reads: the caller's while they are being copied
static const double* in_values(const Ctx& c) { return c.Avin ? c.Avin : c.Av.p; }

static bool fused_ok(const mgr_level_opts& o) {
    return o.sweeps == 1 && o.restrict_type == MGR_RESTRICT_INJECTION &&
           (o.frelax == MGR_FRELAX_JACOBI || o.frelax == MGR_FRELAX_BLOCK_JACOBI);
}

// One MGR level (Sec. 2): C/F split by field, blocks A_FF, A_FC, A_CF, A_CC,
// F-relaxation operator M, P_F = -M A_FC, R_F = -A_CF M (Jacobi restriction),
// coarse operator A_c = A_CC + A_CF P_F (+ R_F A_FC + R_F (A_FF P_F)).
// nF (the number of F-points, known from the label histogram) sizes the
// level's arrays without a sync; the scan's own count is checked at the first
// sync.
// The level's input is the scalar operator A, or, for the first level of a
// block input (A null), the block-CSR input itself.
static void level_extract_count(Ctx& c, const DCsr* A, const int* isF, const int* lmap, const int* fblk, int* cFF,
                                int* cFC, int* cCF, int* cCC) {
    if (A) extract_count(*A, isF, lmap, fblk, cFF, cFC, cCF, cCC, c.s);
    else bsr_extract_count(c.b, c.nbr, c.nnzb, c.Arp.p, c.Aci.p, in_values(c), isF, lmap, fblk, cFF, cFC, cCF, cCC,
                           c.s);
}
static void level_extract_fill(Ctx& c, const DCsr* A, const int* isF, const int* lmap, const int* fblk, DCsr* FF,
                               DCsr* FC, DCsr* CF, DCsr* CC) {
    if (A) {
        extract_fill(*A, isF, lmap, fblk, FF, FC, CF, CC, c.s);
        return;
    }
    // the first extraction of a setup also makes the library's copy of the
    // input values (every block is read here anyway); later steps read it
    double* vcopy = c.copy_in_extract ? c.Av.p : nullptr;
    bsr_extract_fill(c.b, c.nbr, c.nnzb, c.Arp.p, c.Aci.p, in_values(c), isF, lmap, fblk, FF, FC, CF, CC, vcopy, c.s);
    if (vcopy) {
        c.copy_in_extract = false;
        c.Avin = nullptr;
    }
}

// The whole of A_FF for a level that kept only its F-relaxation blocks (for
// export): extracted again from the level's input.
static void ensure_full_aff(Ctx& c, int lev) {
    MgrLevel& l = c.L[lev];
    if (!l.aff_partial) return;
    const DCsr* A = lev > 0 ? &c.L[lev - 1].Aout : (c.A0.nr ? &c.A0 : nullptr);
    DArr<int> cFF((size_t)l.n + 1, c.s);
    level_extract_count(c, A, l.isF.p, l.lmap.p, nullptr, cFF.p, nullptr, nullptr, nullptr);
    DCsr FF = csr_from_counts(l.nF, l.nF, cFF.p, c.slots, "A_FF");
    level_extract_fill(c, A, l.isF.p, l.lmap.p, nullptr, &FF, nullptr, nullptr, nullptr);
    l.AFF = std::move(FF);
    l.aff_partial = false;
}

static DCsr mgr_setup_level(Ctx& c, MgrLevel& l, const DCsr* A, const int* field, const int* block,
                            const mgr_level_opts& o, int lev, int nF) {
    hipStream_t s = c.s;
    Slots& S = c.slots;
    int n = A ? A->nr : c.n;
    l.n = n;
    l.o = o;
    l.isF.alloc((size_t)n + 1, s);
    l.lmap.alloc((size_t)n + 1, s);
    DArr<int> fpos((size_t)n + 1, s);
    l.nF = nF;
    l.nC = n - nF;
    if (l.nF == 0 || l.nC == 0)
        throw Error(MGR_ERR_BAD_LABELS, "MGR level " + std::to_string(lev) + ": empty F or C set");
    cf_flags(n, field, o.f_field_mask, l.isF.p, S.flag(), s);
    long long* sF = S.take(2);
    scan_async(l.isF.p, fpos.p, n, sF, s);
    // the maps and counts below are sized for n until the scan's count of F-points is read
    l.fmap.alloc((size_t)n, s);
    l.cmap.alloc((size_t)n, s);
    cf_maps(n, l.isF.p, fpos.p, l.lmap.p, l.fmap.p, l.cmap.p, s);
    // the F-relaxation block structure (Jacobi: 1x1 blocks; block-Jacobi: the
    // F-points of one group), then the block extraction
    DArr<int> bid, flagk((size_t)l.nF + 1, s), excl((size_t)l.nF + 1, s), bnum((size_t)l.nF + 1, s),
        len((size_t)l.nF + 1, s), bstart((size_t)l.nF + 1, s);
    const int* bidp = nullptr;
    if (o.frelax == MGR_FRELAX_BLOCK_JACOBI) {
        bid.alloc((size_t)l.nF, s);
        gather_int(l.nF, l.fmap.p, block, bid.p, s);
        bidp = bid.p;
    }
    frelax_block_flags(l.nF, bidp, flagk.p, s);
    long long* sB = S.take(2);
    scan_async(flagk.p, excl.p, l.nF, sB, s);
    frelax_block_starts(l.nF, flagk.p, excl.p, bstart.p, bnum.p, s);
    frelax_row_len(l.nF, bnum.p, bstart.p, len.p, S.flag(), s);
    Pend pM = csr_begin(l.M, l.nF, l.nF, len.p, S);
    // the one-sweep apply never reads A_FF: only the part M is formed from (each
    // F row's own block) is extracted; the rest follows on demand (export)
    l.aff_partial = fused_ok(o);
    const int* fblk = l.aff_partial ? bnum.p : nullptr;
    DArr<int> cFF((size_t)n + 1, s), cFC((size_t)n + 1, s), cCF((size_t)n + 1, s), cCC((size_t)n + 1, s);
    level_extract_count(c, A, l.isF.p, l.lmap.p, fblk, cFF.p, cFC.p, cCF.p, cCC.p);
    Pend pFF = csr_begin(l.AFF, l.nF, l.nF, cFF.p, S);
    Pend pFC = csr_begin(l.AFC, l.nF, l.nC, cFC.p, S);
    Pend pCF = csr_begin(l.ACF, l.nC, l.nF, cCF.p, S);
    Pend pCC = csr_begin(l.ACC, l.nC, l.nC, cCC.p, S);
    S.sync("block extraction");
    if (S.val(sF) != l.nF) throw Error(MGR_ERR_ARG, "internal: F-point count differs from the label histogram");
    csr_finish(pFF, S); csr_finish(pFC, S); csr_finish(pCF, S); csr_finish(pCC, S); csr_finish(pM, S);
    long nb = (long)S.val(sB);
    level_extract_fill(c, A, l.isF.p, l.lmap.p, fblk, &l.AFF, &l.AFC, &l.ACF, &l.ACC);
    // M's pivots are checked at the next sync (an invalid one sets the flag);
    // until then M is only an operand of products, never used for control
    frelax_fill((int)nb, bstart.p, l.AFF, l.M, S.flag(), s);
    if (o.frelax == MGR_FRELAX_ILU0) {
        // ILU(0) on the pattern of A_FF in the natural order, one level of rows at a time
        DCsr LU = csr_copy(l.AFF, s);
        DArr<int> dpos((size_t)l.nF + 1, s);
        diag_pos(LU, dpos.p, S.flag(), s);
        S.sync("ILU(0) diagonal");
        l.schL = level_schedule(LU, true, S);
        for (size_t k = 0; k + 1 < l.schL.off.size(); ++k)
            ilu_level(l.schL.off[k + 1] - l.schL.off[k], l.schL.order.p + l.schL.off[k], LU, dpos.p, S.flag(), s);
        DArr<int> nl((size_t)l.nF + 1, s), nu((size_t)l.nF + 1, s);
        split_count(LU, nl.p, nu.p, s);
        Pend pL = csr_begin(l.iluL, l.nF, l.nF, nl.p, S);
        Pend pU = csr_begin(l.iluU, l.nF, l.nF, nu.p, S);
        S.sync("ILU(0) factorization");
        csr_finish(pL, S);
        csr_finish(pU, S);
        split_fill(LU, l.iluL, l.iluU, s);
        l.schU = level_schedule(l.iluU, false, S);
    }
    if (o.frelax == MGR_FRELAX_AMG) {
        // the AMG operator: A_FF, or its separate-component approximation
        // (MGR_AMG_SEPARATE: the couplings between unknowns of different
        // fields dropped, Sec. 4.4)
        DArr<int> flab;
        if (o.amg_unknown_based) {
            flab.alloc((size_t)l.nF, s);
            gather_int(l.nF, l.fmap.p, field, flab.p, s);
        }
        auto amg_operator = [&]() {
            if (o.amg_unknown_based != MGR_AMG_SEPARATE) return csr_copy(l.AFF, s);
            DArr<int> cnt((size_t)l.nF + 1, s);
            label_filter_count(l.AFF, flab.p, cnt.p, s);
            DCsr B = csr_from_counts(l.nF, l.nF, cnt.p, S, "separate-component approximation");
            label_filter_fill(l.AFF, flab.p, B, s);
            return B;
        };
        if (lev < (int)c.reuse_famg.size() && c.reuse_famg[lev]) {
            // setup reuse: the previous hierarchy of this level, kept whole (A_FF
            // unchanged) or with new Galerkin products
            l.famg = std::move(c.reuse_famg[lev]);
            if (!c.reuse_keep_famg) amg_refresh(*l.famg, amg_operator(), S);
        } else {
            l.famg.reset(new Amg());
            mgr_amg_opts fo = c.o.amg;
            fo.unknown_based = o.amg_unknown_based != 0;
            fo.agg_levels = o.amg_agg_levels;
            amg_setup(*l.famg, amg_operator(), o.amg_unknown_based ? flab.p : nullptr, fo,
                      c.o.amg.seed + 0x1000193ULL * (uint64_t)(lev + 1), S);
        }
    }
    // transfer operators and the Petrov-Galerkin coarse operator R A P
    Spgemm jP, jW;
    const bool bdl = bdiag_left_ok(l.M, l.AFC), bdr = bdiag_right_ok(l.ACF, l.M);
    if (bdl) bdiag_begin(jP, 1, l.M, l.AFC, l.PF, (int)nb, bstart.p, S);
    else spgemm_begin(jP, l.M, l.AFC, l.PF, S);
    jP.neg = true;
    if (bdr) bdiag_begin(jW, 2, l.ACF, l.M, l.W, 0, nullptr, S);
    else spgemm_begin(jW, l.ACF, l.M, l.W, S);
    S.sync("MGR transfer operators");
    spgemm_finish(jP, S);
    // with the fused apply, W = A_CF M is read only by R_J's fill: its own
    // numeric pass goes to the auxiliary stream with it
    l.fused = fused_ok(o);
    spgemm_alloc(jW, S);
    if (!l.fused) spgemm_fillpass(jW, S, s);
    if (o.restrict_type == MGR_RESTRICT_JACOBI) {
        l.RF = csr_copy(l.W, s);
        negate(l.RF.v.p, l.RF.nnz, s);
    }
    // A_c = A_CC + A_CF P_F, as one hashed product when its rows are short
    const bool fuse_add = spgemm_add_fusable(l.ACF, l.PF, l.ACC);
    DCsr T1, Ac;
    Spgemm j1;
    // the rows of P_F of one F-relaxation block share their pattern (a failed
    // block has stopped the setup at the block extraction's sync)
    if (fuse_add) spgemm_add_begin(j1, l.ACF, l.PF, l.ACC, Ac, S, bnum.p);
    else spgemm_begin(j1, l.ACF, l.PF, T1, S);
    // fused one-sweep apply: r_c = [-omega A_CF M | I] v ; z = [P_F | omega M] [e_c ; v]
    DArr<int> lenR, lenP;
    Pend pR, pP;
    if (l.fused) {
        lenR.alloc((size_t)l.nC + 1, s);
        lenP.alloc((size_t)n + 1, s);
        rj_count(l.nC, l.W, lenR.p, s);
        pj_count(n, l.isF.p, l.lmap.p, l.PF, l.M, lenP.p, s);
        pR = csr_begin(l.RJ, l.nC, n, lenR.p, S);
        pP = csr_begin(l.PJ, n, l.nC + n, lenP.p, S);
    }
    S.sync("MGR coarse product");
    spgemm_finish(j1, S);
    if (l.fused) {
        csr_finish(pR, S);
        csr_finish(pP, S);
        // R_J and P_J (and W, read only by R_J's fill) are read only by the
        // apply: filled on the auxiliary stream once the coarse AMG reaches
        // its small levels (on the busy large levels the two streams would
        // only share the bandwidth), joined before the setup returns
        const FillPass wfill = fill_pass(jW);
        const double om = o.omega;
        const bool f32 = c.o.apply_precision == 32;
        c.deferred.push_back([&c, wfill]() { wfill.run(c.slots.flag(), c.aux); });
        // (with the FP32 apply, the fills write its FP32 copies too)
        c.deferred.push_back([&c, &l, om, f32]() {
            if (f32) l.RJ.vf.alloc((size_t)(l.RJ.nnz > 0 ? l.RJ.nnz : 1), c.s);
            rj_fill(l.nC, l.W, -om, l.fmap.p, l.cmap.p, l.RJ, c.aux);
        });
        c.deferred.push_back([&c, &l, om, n, f32]() {
            if (f32) l.PJ.vf.alloc((size_t)(l.PJ.nnz > 0 ? l.PJ.nnz : 1), c.s);
            pj_fill(n, l.nC, l.isF.p, l.lmap.p, l.PF, 1.0, l.M, om, l.fmap.p, l.PJ, c.aux);
        });
    }
    if (!fuse_add) {
        Ac = csr_add(l.ACC, T1, S);
        T1 = DCsr();
    }
    if (o.restrict_type == MGR_RESTRICT_JACOBI) {
        DCsr T2 = spgemm(l.RF, l.AFC, S);
        DCsr S2 = csr_add(Ac, T2, S);
        T2 = DCsr();
        DCsr FFP = spgemm(l.AFF, l.PF, S);
        DCsr T3 = spgemm(l.RF, FFP, S);
        FFP = DCsr();
        Ac = csr_add(S2, T3, S);
    }
    // level vectors
    l.rcd.alloc((size_t)l.nC + 1, s);
    l.ecd.alloc((size_t)l.nC + 1, s);
    if (!l.fused) {
        l.vFd.alloc((size_t)l.nF + 1, s); l.vCd.alloc((size_t)l.nC + 1, s);
        l.zFd.alloc((size_t)l.nF + 1, s); l.rFd.alloc((size_t)l.nF + 1, s); l.tFd.alloc((size_t)l.nF + 1, s);
    }
    return Ac;
}

static void mgr_level_make_trans(Ctx& c, MgrLevel& l) {
    if (l.have_trans) return;
    hipStream_t s = c.s;
    Slots& S = c.slots;
    if (l.o.sweeps != 1)
        throw Error(MGR_ERR_UNSUPPORTED, "transposed MGR apply needs one F-relaxation sweep per level");
    if (l.fused) {
        // r_c = [P_F^T | I] u ; z = [-omega W^T | omega M^T] [e ; u]
        DCsr PFt = csr_transpose(l.PF, S);
        DCsr Wt = csr_transpose(l.W, S);
        DCsr Mt = csr_transpose(l.M, S);
        DArr<int> len((size_t)l.n + 1, s);
        rj_count(l.nC, PFt, len.p, s);
        l.RJt = csr_from_counts(l.nC, l.n, len.p, S, "transposed restriction");
        rj_fill(l.nC, PFt, 1.0, l.fmap.p, l.cmap.p, l.RJt, s);
        pj_count(l.n, l.isF.p, l.lmap.p, Wt, Mt, len.p, s);
        l.PJt = csr_from_counts(l.n, l.nC + l.n, len.p, S, "transposed interpolation");
        pj_fill(l.n, l.nC, l.isF.p, l.lmap.p, Wt, -l.o.omega, Mt, l.o.omega, l.fmap.p, l.PJt, s);
        if (l.have_float) { make_float(l.RJt, s); make_float(l.PJt, s); }
    } else {
        l.AFFt = csr_transpose(l.AFF, S);
        l.ACFt = csr_transpose(l.ACF, S);
        l.PFt = csr_transpose(l.PF, S);
        l.Mt = csr_transpose(l.M, S);
        if (l.o.restrict_type == MGR_RESTRICT_JACOBI) l.RFt = csr_transpose(l.RF, S);
        if (l.o.frelax == MGR_FRELAX_ILU0) {
            l.iluLt = csr_transpose(l.iluL, S);
            l.iluUt = csr_transpose(l.iluU, S);
            l.schUt = level_schedule(l.iluUt, true, S);
            l.schLt = level_schedule(l.iluLt, false, S);
        }
        if (l.have_float) {
            make_float(l.AFFt, s); make_float(l.ACFt, s); make_float(l.PFt, s); make_float(l.Mt, s);
            if (l.RFt.nr) make_float(l.RFt, s);
            if (l.iluLt.nr) { make_float(l.iluLt, s); make_float(l.iluUt, s); }
        }
    }
    if (l.famg) amg_make_trans(*l.famg, S);
    l.have_trans = true;
}

// the level's FP32 copies, converted on stream run (c.s when null)
static void mgr_level_make_float(Ctx& c, MgrLevel& l, F32Batch& fb) {
    if (l.have_float) return;
    hipStream_t s = c.s;
    if (l.fused) {
        make_float_on(l.RJ, s, fb); make_float_on(l.PJ, s, fb);
        if (l.have_trans) { make_float_on(l.RJt, s, fb); make_float_on(l.PJt, s, fb); }
    } else {
        make_float_on(l.AFF, s, fb); make_float_on(l.ACF, s, fb);
        make_float_on(l.PF, s, fb); make_float_on(l.M, s, fb);
        if (l.RF.nr) make_float_on(l.RF, s, fb);
        if (l.iluL.nr) { make_float_on(l.iluL, s, fb); make_float_on(l.iluU, s, fb); }
        if (l.have_trans && l.iluLt.nr) { make_float_on(l.iluLt, s, fb); make_float_on(l.iluUt, s, fb); }
        if (l.have_trans) {
            make_float_on(l.AFFt, s, fb); make_float_on(l.ACFt, s, fb);
            make_float_on(l.PFt, s, fb); make_float_on(l.Mt, s, fb);
            if (l.RFt.nr) make_float_on(l.RFt, s, fb);
        }
        l.vFf.alloc((size_t)l.nF + 1, s); l.vCf.alloc((size_t)l.nC + 1, s);
        l.zFf.alloc((size_t)l.nF + 1, s); l.rFf.alloc((size_t)l.nF + 1, s); l.tFf.alloc((size_t)l.nF + 1, s);
    }
    l.rcf.alloc((size_t)l.nC + 1, s);
    l.ecf.alloc((size_t)l.nC + 1, s);
    if (l.fused && &l == &c.L.front()) l.vinf.alloc((size_t)l.n + 1, s);
    if (l.famg) amg_make_float(*l.famg, s, fb);
    l.have_float = true;
}

template <typename T> struct LV;
template <> struct LV<double> {
    static double* rc(MgrLevel& l) { return l.rcd.p; }
    static double* ec(MgrLevel& l) { return l.ecd.p; }
    static double* vF(MgrLevel& l) { return l.vFd.p; }
    static double* vC(MgrLevel& l) { return l.vCd.p; }
    static double* zF(MgrLevel& l) { return l.zFd.p; }
    static double* rF(MgrLevel& l) { return l.rFd.p; }
    static double* tF(MgrLevel& l) { return l.tFd.p; }
};
template <> struct LV<float> {
    static float* rc(MgrLevel& l) { return l.rcf.p; }
    static float* ec(MgrLevel& l) { return l.ecf.p; }
    static float* vF(MgrLevel& l) { return l.vFf.p; }
    static float* vC(MgrLevel& l) { return l.vCf.p; }
    static float* zF(MgrLevel& l) { return l.zFf.p; }
    static float* rF(MgrLevel& l) { return l.rFf.p; }
    static float* tF(MgrLevel& l) { return l.tFf.p; }
};

// tF = M_FF^{-1} rF (trans: M_FF^{-T}) for Jacobi / block-Jacobi / AMG F-relaxation
template <typename T>
static void frelax_apply(MgrLevel& l, const T* rF, T* tF, bool tr, hipStream_t s) {
    if (l.o.frelax == MGR_FRELAX_ILU0) {
        // (LU)^{-1} r: L y = r (unit lower), U z = y; (LU)^{-T} r: U^T y = r, L^T z = y
        if (!tr) {
            trsv<T>(l.schL, l.iluL, rF, tF, true, s);
            trsv<T>(l.schU, l.iluU, tF, tF, false, s);
        } else {
            trsv<T>(l.schUt, l.iluUt, rF, tF, false, s);
            trsv<T>(l.schLt, l.iluLt, tF, tF, true, s);
        }
        return;
    }
    if (l.o.frelax == MGR_FRELAX_AMG) {
        amg_vcycle<T>(*l.famg, 0, rF, tF, tr, s);
        return;
    }
    spmv<T, T, T, T, T>(view<T>(tr ? l.Mt : l.M), rF, (const T*)nullptr, INT_MAX, (const T*)nullptr, tF, T(1),
                        T(0), s);
}

template <typename T>
static void mgr_apply_rec(Ctx& c, int lev, const void* vin, void* zout, bool tr, const void* bd = nullptr);

// D^-1 of the first AMG level when the last MGR restriction can form D^-1 b
// for its pre-smoothing (a plain level with a sweep), else null.
template <typename T>
static const T* amg_first_dinv(Ctx& c, bool tr) {
    Amg& H = c.camg;
    if (H.lv.size() < 2 || H.lv[0].composed || (tr ? H.nu_post : H.nu_pre) < 1) return nullptr;
    if (H.smoother != MGR_SMOOTH_L1_JACOBI) return nullptr;   // the first sweep is not D^-1 b
    return Prec<T>::dinv(H.lv[0]);
}

// The one-sweep level: r_c = R_J v, the coarse solve, z = P_J [e_c ; v];
// XT is the type the transfers read v in, ZT the type of z.
template <typename T, typename XT, typename ZT>
static void fused_level_apply(Ctx& c, int lev, MgrLevel& l, const XT* v, ZT* z, bool tr) {
    hipStream_t s = c.s;
    T* rc = LV<T>::rc(l);
    T* ec = LV<T>::ec(l);
    SpOp<T> R = view<T>(tr ? l.RJt : l.RJ);
    SpOp<T> P = view<T>(tr ? l.PJt : l.PJ);
    const T* d0 = (lev + 1 == (int)c.L.size()) ? amg_first_dinv<T>(c, tr) : nullptr;
    if (d0) {
        // the coarse AMG's first pre-smoothing gathers D^-1 r_c formed here
        T* sc = Prec<T>::sb(c.camg.lv[0]);
        restrict_scaled<T, XT>(R, v, d0, rc, sc, s);
        mgr_apply_rec<T>(c, lev + 1, rc, ec, tr, sc);
    } else {
        spmv<T, XT, XT, T, T>(R, v, (const XT*)nullptr, INT_MAX, (const T*)nullptr, rc, T(1), T(0), s);
        mgr_apply_rec<T>(c, lev + 1, rc, ec, tr);
    }
    spmv<T, T, XT, ZT, ZT>(P, ec, v, l.nC, (const ZT*)nullptr, z, T(1), T(0), s);
}

// Algorithm 1 at level `lev` with working precision T; VT is the type of v and
// z at this level (FP64 at level 0, T below).
template <typename T, typename VT>
static void mgr_level_apply(Ctx& c, int lev, const VT* v, VT* z, bool tr) {
    hipStream_t s = c.s;
    MgrLevel& l = c.L[lev];
    T* rc = LV<T>::rc(l);
    T* ec = LV<T>::ec(l);
    if (l.fused) {
        if constexpr (std::is_same_v<T, float> && std::is_same_v<VT, double>) {
            if (l.vinf.p) {
                // the FP32 transfers read each value of v rounded to FP32:
                // rounded once here, both read FP32 columns (the same values;
                // one column type lets the interpolation issue one load per
                // entry instead of one per source)
                copy<double, float>(l.n, v, l.vinf.p, s);
                fused_level_apply<T, float, VT>(c, lev, l, l.vinf.p, z, tr);
                return;
            }
        }
        fused_level_apply<T, VT, VT>(c, lev, l, v, z, tr);
        return;
    }
    T* vF = LV<T>::vF(l);
    T* vC = LV<T>::vC(l);
    T* zF = LV<T>::zF(l);
    T* rF = LV<T>::rF(l);
    T* tF = LV<T>::tF(l);
    T om = (T)l.o.omega;
    gather<VT, T>(l.nF, l.fmap.p, v, vF, s);
    gather<VT, T>(l.nC, l.cmap.p, v, vC, s);
    if (!tr) {
        // F-relaxation sweeps from z = 0 (the C part of z stays 0 meanwhile)
        for (int q = 0; q < l.o.sweeps; ++q) {
            const T* res = vF;
            if (q > 0) {
                spmv<T, T, T, T, T>(view<T>(l.AFF), zF, (const T*)nullptr, INT_MAX, vF, rF, T(-1), T(1), s);
                res = rF;
            }
            frelax_apply<T>(l, res, tF, false, s);
            axpby<T>(l.nF, om, tF, q == 0 ? T(0) : T(1), zF, s);
        }
        // restriction: r_c = v_C - A_CF z_F (+ R_F (v_F - A_FF z_F))
        spmv<T, T, T, T, T>(view<T>(l.ACF), zF, (const T*)nullptr, INT_MAX, vC, rc, T(-1), T(1), s);
        if (l.o.restrict_type == MGR_RESTRICT_JACOBI) {
            spmv<T, T, T, T, T>(view<T>(l.AFF), zF, (const T*)nullptr, INT_MAX, vF, rF, T(-1), T(1), s);
            spmv<T, T, T, T, T>(view<T>(l.RF), rF, (const T*)nullptr, INT_MAX, rc, rc, T(1), T(1), s);
        }
        mgr_apply_rec<T>(c, lev + 1, rc, ec, false);
        // interpolation and correction: z_F += P_F e_c ; z_C = e_c
        spmv<T, T, T, T, T>(view<T>(l.PF), ec, (const T*)nullptr, INT_MAX, zF, zF, T(1), T(1), s);
    } else {
        // u_c = v_C + P_F^T v_F ; e = C^T u_c ; y_F = R_F^T e ;
        // z_F = y_F + omega M^T (v_F - A_FF^T y_F - A_CF^T e) ; z_C = e
        spmv<T, T, T, T, T>(view<T>(l.PFt), vF, (const T*)nullptr, INT_MAX, vC, rc, T(1), T(1), s);
        mgr_apply_rec<T>(c, lev + 1, rc, ec, true);
        spmv<T, T, T, T, T>(view<T>(l.ACFt), ec, (const T*)nullptr, INT_MAX, vF, rF, T(-1), T(1), s);
        bool jr = (l.o.restrict_type == MGR_RESTRICT_JACOBI);
        if (jr) {
            spmv<T, T, T, T, T>(view<T>(l.RFt), ec, (const T*)nullptr, INT_MAX, (const T*)nullptr, zF, T(1), T(0), s);
            spmv<T, T, T, T, T>(view<T>(l.AFFt), zF, (const T*)nullptr, INT_MAX, rF, rF, T(-1), T(1), s);
        }
        frelax_apply<T>(l, rF, tF, true, s);
        axpby<T>(l.nF, om, tF, jr ? T(1) : T(0), zF, s);
    }
    scatter<T, VT>(l.nF, l.fmap.p, zF, z, s);
    scatter<T, VT>(l.nC, l.cmap.p, ec, z, s);
}

template <typename T>
static void mgr_apply_rec(Ctx& c, int lev, const void* vin, void* zout, bool tr, const void* bd) {
    if (lev == (int)c.L.size()) {
        amg_vcycle<T>(c.camg, 0, (const T*)vin, (T*)zout, tr, c.s, (const T*)bd);
        return;
    }
    if (lev == 0)
        mgr_level_apply<T, double>(c, 0, (const double*)vin, (double*)zout, tr);
    else
        mgr_level_apply<T, T>(c, lev, (const T*)vin, (T*)zout, tr);
}

// z = M^{-1} v (or M^{-T} v), FP64 in and out whatever the apply precision.
static void mgr_apply_top(Ctx& c, const double* v, double* z, bool tr) {
    if (!c.ready) throw Error(MGR_ERR_ARG, "apply before setup");
    if (tr) {
        for (auto& l : c.L) mgr_level_make_trans(c, l);
        amg_make_trans(c.camg, c.slots);
    }
    bool f32 = (c.o.apply_precision == 32);
    if (f32) {
        F32Batch fb;
        for (auto& l : c.L) mgr_level_make_float(c, l, fb);
        amg_make_float(c.camg, c.s, fb);
        fb.flush(c.s);
    }
    if (c.L.empty()) {
        // no reduction level: the preconditioner is the AMG cycle on A itself
        if (f32) {
            if (!c.apply_tmp.p) c.apply_tmp.alloc((size_t)c.n * 2 + 2, c.s);
            float* vf = reinterpret_cast<float*>(c.apply_tmp.p);
            float* zf = vf + c.n + 1;
            copy<double, float>(c.n, v, vf, c.s);
            amg_vcycle<float>(c.camg, 0, vf, zf, tr, c.s);
            copy<float, double>(c.n, zf, z, c.s);
        } else {
            amg_vcycle<double>(c.camg, 0, v, z, tr, c.s);
        }
        c.warm[tr ? 1 : 0] = true;
        return;
    }
    if (f32) mgr_apply_rec<float>(c, 0, v, z, tr);
    else mgr_apply_rec<double>(c, 0, v, z, tr);
    c.warm[tr ? 1 : 0] = true;
}

// ====================================================================== no-allocation apply
// Work vectors of mgr_apply_noalloc live in one static device array per GPU,
// held until the process ends.  In host code the array's name only stands in
// for the symbol: its device address (one per device) comes from
// hipGetSymbolAddress, looked up once per device when a handle is created on
// it, and only that address is ever passed to kernels.
static __device__ __align__(256) unsigned char scratch[MGR_NOALLOC_SCRATCH_BYTES];

static unsigned char* scratch_for_device(int dev) {
    static std::mutex mu;
    static std::map<int, unsigned char*> addr;
    std::lock_guard<std::mutex> g(mu);
    auto it = addr.find(dev);
    if (it != addr.end()) return it->second;
    void* p = nullptr;
    hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p)
        throw Error(MGR_ERR_HIP, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    addr[dev] = static_cast<unsigned char*>(p);
    return static_cast<unsigned char*>(p);
}

// Every work vector of the apply (level vectors of the MGR levels, of the
// F-relaxation and coarse AMG hierarchies, and the FP32 staging of a pure AMG
// preconditioner): the only device memory an apply writes besides z.
template <typename F>
static void for_each_work(Amg& H, F&& f) {
    for (auto& L : H.lv) {
        f(L.rd); f(L.td); f(L.bd); f(L.xd); f(L.sd);
        f(L.rf); f(L.tf); f(L.bf); f(L.xf); f(L.sf);
    }
}
template <typename F>
static void for_each_work(Ctx& c, F&& f) {
    for (auto& l : c.L) {
        f(l.rcd); f(l.ecd); f(l.vFd); f(l.vCd); f(l.zFd); f(l.rFd); f(l.tFd);
        f(l.rcf); f(l.ecf); f(l.vFf); f(l.vCf); f(l.zFf); f(l.rFf); f(l.tFf); f(l.vinf);
        if (l.famg) for_each_work(*l.famg, f);
    }
    for_each_work(c.camg, f);
    f(c.apply_tmp);
}

// z = M^{-1} v with every work vector placed in the device's scratch array:
// the hierarchy's own work vectors are pointed into it for the enqueue and
// pointed back afterwards (kernels take their addresses at launch).  Needs a
// hierarchy on which a forward apply has already run, so that every operator
// copy the apply reads exists; allocates nothing.
static void mgr_apply_noalloc_impl(Ctx& c, const double* v, double* z) {
    if (!c.ready) throw Error(MGR_ERR_ARG, "apply before setup");
    if (!c.warm[0])
        throw Error(MGR_ERR_ARG, "mgr_apply_noalloc needs one mgr_apply (or mgr_solve) on this hierarchy first");
    if (!c.scratch) throw Error(MGR_ERR_ARG, "internal: no scratch address for this device");
    // the work vectors of the apply precision in use (the FP32 apply of a pure
    // AMG preconditioner also stages v and z in apply_tmp)
    const bool f32 = (c.o.apply_precision == 32);
    auto used = [&](auto& a) {
        using T = std::remove_pointer_t<decltype(a.p)>;
        if (!a.p) return false;
        if ((const void*)&a == (const void*)&c.apply_tmp) return f32;
        return std::is_same_v<T, float> == f32;
    };
    size_t need = 0;
    auto round = [](size_t b) { return (b + 255) & ~size_t(255); };
    for_each_work(c, [&](auto& a) { if (used(a)) need += round(a.bytes()); });
    if (need > MGR_NOALLOC_SCRATCH_BYTES)
        throw Error(MGR_ERR_UNSUPPORTED, "mgr_apply_noalloc: the hierarchy's work vectors need " +
                                             std::to_string(need) + " bytes, above the scratch size of " +
                                             std::to_string((size_t)MGR_NOALLOC_SCRATCH_BYTES) + " bytes");
    struct Restore {
        Ctx& c;
        ~Restore() {
            for (auto& q : c.saved_d) q.first->p = q.second;
            for (auto& q : c.saved_f) q.first->p = q.second;
            c.saved_d.clear();
            c.saved_f.clear();
            tl_noalloc = false;
        }
    } restore{c};
    size_t off = 0;
    for_each_work(c, [&](auto& a) {
        if (!used(a)) return;
        using T = std::remove_pointer_t<decltype(a.p)>;
        T* q = reinterpret_cast<T*>(c.scratch + off);
        if constexpr (std::is_same_v<T, double>) c.saved_d.emplace_back(&a, a.p);
        else c.saved_f.emplace_back(&a, a.p);
        a.p = q;
        off += round(a.bytes());
    });
    tl_noalloc = true;
    mgr_apply_top(c, v, z, false);
}

static void ensure_At(Ctx& c) {
    if (c.have_At) return;
    hipStream_t s = c.s;
    if (c.b == 1) {
        c.A0t = csr_transpose(c.A0, c.slots);
    } else {
        c.ATrp.alloc((size_t)c.nbr + 1, s);
        c.ATci.alloc((size_t)(c.nnzb > 0 ? c.nnzb : 1), s);
        c.ATv.alloc((size_t)(c.nnzb > 0 ? c.nnzb : 1) * c.b * c.b, s);
        bsr_transpose_blocks(c.b, c.nbr, c.Arp.p, c.Aci.p, c.Av.p, c.ATrp.p, c.ATci.p, c.ATv.p, s);
    }
    MGR_HIP(hipStreamSynchronize(s));
    c.have_At = true;
}

// y = alpha * op(A) x + beta * w in FP64 (block SpMV on the input layout)
static void matvec(Ctx& c, bool tr, const double* x, const double* w, double* y, double alpha, double beta) {
    if (tr) ensure_At(c);
    if (c.b == 1) {
        spmv<double, double, double, double, double>(view<double>(tr ? c.A0t : c.A0), x, (const double*)nullptr,
                                                     INT_MAX, w, y, alpha, beta, c.s, 1);
    } else {
        bsr_spmv(c.b, c.nbr, tr ? c.ATrp.p : c.Arp.p, tr ? c.ATci.p : c.Aci.p, tr ? c.ATv.p : c.Av.p, c.nnzb, x, w,
                 y, alpha, beta, c.s);
    }
}

// ====================================================================== FGMRES
static void ensure_krylov(Ctx& c) {
    int m = c.o.restart;
    if (c.kr_m == m && c.kr_n == c.n && c.V.p) return;
    hipStream_t s = c.s;
    c.V.alloc((size_t)(m + 1) * c.n, s);
    c.Z.alloc((size_t)m * c.n, s);
    c.hbuf.alloc(512, s);
    c.part.alloc((size_t)2 * (m + 2) * KRYLOV_PARTS, s);
    c.yd.alloc(64, s);
    if (c.hpin) (void)hipHostFree(c.hpin);
    c.hpin = nullptr;
    c.hpin_dev = nullptr;
    MGR_HIP(hipHostMalloc(reinterpret_cast<void**>(&c.hpin), sizeof(double) * Ctx::HROW * (m + 1),
                          hipHostMallocDefault));
    MGR_HIP(hipHostGetDevicePointer(reinterpret_cast<void**>(&c.hpin_dev), c.hpin, 0));
    c.kr_m = m;
    c.kr_n = c.n;
}

// Wait until a kernel has set the host-mapped ready flag *f to 1 (and then
// read what it stored before it).  The stream is polled now and then, so
// that a flag that can no longer be set ends in an error, not a hang.
static void wait_flag(const double* f, hipStream_t s) {
    const volatile double* vf = f;
    for (long spins = 1; *vf != 1.0; ++spins) {
        if (spins % 4096 == 0) {
            hipError_t e = hipStreamQuery(s);
            if (e == hipSuccess) {
                if (*vf == 1.0) break;
                throw Error(MGR_ERR_HIP, "FGMRES: the stream finished without publishing the Arnoldi step");
            }
            if (e != hipErrorNotReady) MGR_HIP(e);
        }
    }
    std::atomic_thread_fence(std::memory_order_acquire);
}

// Flexible GMRES(m) with right preconditioning (Saad 1993): x0 = 0, Givens
// rotations on the host, stop when |g_{k}| <= rtol ||b||, then the true
// residual ||b - A x|| is checked and the cycle restarted if needed.
//
// Arnoldi: classical Gram-Schmidt applied twice, with the second pass of each
// basis vector delayed into the next step (two passes over the basis per
// step instead of three).  Step j starts from u_j, the newest basis vector
// after one pass and a normalisation, stored as V_j: z_j = M^-1 u_j, w = A z_j;
// the first pass forms V_i . u_j and V_i . w (i <= j); the second turns u_j into
// the final v_j = (u_j - sum_{i<j} a_i v_i) / alpha_j and orthogonalises w once
// against v_0 .. v_j with coefficients c_i, leaving w' = nu_j u_{j+1}.  Since
// u_{j+1} = sum_{i<=j} a'_i v_i + alpha_{j+1} v_{j+1}, column j of the
// Hessenberg matrix is c_i + nu_j a'_i (i <= j) and nu_j alpha_{j+1}: it is
// complete once the next step's first pass (or a separate one at the end of a
// cycle or near convergence) has given a' and alpha_{j+1}.  z_j comes from u_j
// rather than v_j, which the flexible method allows (A Z = V H holds with the
// final basis).
//
// The coefficients of step j reach a pinned host row from the kernel that
// ends the step, so step j+1 is queued before the host has seen step j; the
// host processes step j-1 meanwhile.  When the residual estimate predicts
// convergence with the newest column, the host completes that column with a
// separate first pass on the newest vector instead of queuing another step.
static int fgmres(Ctx& c, bool tr, const double* b, double* x, mgr_solve_info* info) {
    hipStream_t s = c.s;
    ensure_krylov(c);
    const long n = c.n;
    const int m = c.o.restart;
    double* V = c.V.p;
    double* Z = c.Z.p;
    // device scalars: [0, 2 nv) first-pass dots, [HC, HC + nv) coefficients c,
    // [HA] alpha, [HN] ||w'||^2, [HF, HF + nv + 1) dots of a separate pass,
    // [HS] a norm
    double* hb = c.hbuf.p;
    constexpr int HC = 128, HA = 192, HN = 193, HF = 256, HS = 511, NPUB = 194;
    double* hscr = c.hpin + (size_t)Ctx::HROW * m;   // host row for the scalar reads
    std::vector<double> H((size_t)(m + 1) * m), cs(m), sn(m), g(m + 1), y(m), cpend(m + 1);
    set<double>(n, x, 0.0, s);
    auto read_scalar = [&](const double* dptr) {
        MGR_HIP(hipMemcpyAsync(hscr, dptr, sizeof(double), hipMemcpyDeviceToHost, s));
        MGR_HIP(hipStreamSynchronize(s));
        return hscr[0];
    };
    mdot(n, b, n, 1, b, c.part.p, hb + HS, s);
    double bnorm = std::sqrt(read_scalar(hb + HS));
    mgr_solve_info inf{};
    if (bnorm == 0.0) {
        inf.status = MGR_OK;
        if (info) *info = inf;
        return MGR_OK;
    }
    const double tol = c.o.rtol * bnorm;
    int iters = 0;
    bool converged = false;
    double est = 1.0, truer = 1.0;
    bool first = true;
    for (int cycle = 0;; ++cycle) {
        // V_0 = b - A x
        if (first) copy<double, double>(n, b, V, s);
        else matvec(c, tr, x, b, V, -1.0, 1.0);
        first = false;
        mdot(n, V, n, 1, V, c.part.p, hb + HS, s);
        double beta = std::sqrt(read_scalar(hb + HS));
        if (beta <= tol) {
            converged = true;
            est = truer = beta / bnorm;
            break;
        }
        if (cycle > 0) inf.restarts++;
        scale(n, 1.0 / beta, V, s);
        std::fill(g.begin(), g.end(), 0.0);
        std::fill(H.begin(), H.end(), 0.0);
        g[0] = beta;  // times alpha_0 (about 1) once step 0 is read
        const int jmax = std::min(m, c.o.maxiter - iters);
        int k = 0;          // Hessenberg columns completed
        int rows = 0;       // steps whose coefficients the host has read
        bool stop = false;  // converged, broke down, or out of iterations
        double rate = 1.0;  // last ratio |g_{k+1}| / |g_k|
        double nupend = 0.0;
        // Givens update of column col = k from its entries (H column already filled)
        auto rotate = [&](int col) {
            for (int i = 0; i < col; ++i) {
                double a0 = H[(size_t)i * m + col], a1 = H[(size_t)(i + 1) * m + col];
                H[(size_t)i * m + col] = cs[i] * a0 + sn[i] * a1;
                H[(size_t)(i + 1) * m + col] = -sn[i] * a0 + cs[i] * a1;
            }
            const double hn = H[(size_t)(col + 1) * m + col];
            double a0 = H[(size_t)col * m + col], a1 = hn;
            double den = std::sqrt(a0 * a0 + a1 * a1);
            if (den == 0.0) { cs[col] = 1.0; sn[col] = 0.0; }
            else { cs[col] = a0 / den; sn[col] = a1 / den; }
            H[(size_t)col * m + col] = cs[col] * a0 + sn[col] * a1;
            H[(size_t)(col + 1) * m + col] = 0.0;
            double gprev = std::fabs(g[col]);
            g[col + 1] = -sn[col] * g[col];
            g[col] = cs[col] * g[col];
            ++iters;
            k = col + 1;
            est = std::fabs(g[col + 1]) / bnorm;
            if (gprev > 0.0) rate = std::min(1.0, std::max(0.05, std::fabs(g[col + 1]) / gprev));
            if (hn == 0.0 || std::fabs(g[col + 1]) <= tol || iters >= c.o.maxiter) stop = true;
        };
        // column col from its pending coefficients and the next vector's
        // first-pass dots a[0..col] and normalisation alpha
        auto complete = [&](int col, const double* a, double alpha) {
            for (int i = 0; i <= col; ++i) H[(size_t)i * m + col] = cpend[i] + nupend * a[i];
            H[(size_t)(col + 1) * m + col] = nupend * alpha;
            rotate(col);
        };
        auto alpha_of = [](const double* sdots, int j) {
            double ss = 0.0;
            for (int i = 0; i < j; ++i) ss += sdots[i] * sdots[i];
            double a2 = sdots[j] - ss;
            return a2 > 0.0 ? std::sqrt(a2) : 0.0;
        };
        // read step r's row: complete column r-1 (unless done already), keep column r pending
        auto process_row = [&](int r) {
            const double* hh = c.hpin + (size_t)Ctx::HROW * r;
            wait_flag(hh + NPUB, s);
            const double alpha = hh[HA];
            if (r == 0) g[0] = beta * alpha;
            else if (k == r - 1) complete(r - 1, hh, alpha);
            if (!(alpha > 0.0) && !stop) stop = true;  // breakdown of the basis
            for (int i = 0; i <= r; ++i) cpend[i] = hh[HC + i];
            nupend = std::sqrt(hh[HN]);
        };
        // a separate first pass on u_{col+1} = V_{col+1} completes column col
        auto finish_column = [&](int col) {
            mdot(n, V, n, col + 2, V + (long)(col + 1) * n, c.part.p, hb + HF, s);
            MGR_HIP(hipMemcpyAsync(hscr, hb + HF, sizeof(double) * (col + 2), hipMemcpyDeviceToHost, s));
            MGR_HIP(hipStreamSynchronize(s));
            complete(col, hscr, alpha_of(hscr, col + 1));
        };
        for (int j = 0; j < jmax && !stop; ++j) {
            if (j >= 1 && k < j) {
                // would column j-1 converge?  (predicted from the last rate)
                double pred = std::fabs(g[k]) * std::pow(rate, (double)(j - k));
                if (pred <= 4.0 * tol) {
                    while (rows < j && !stop) process_row(rows++);
                    if (stop) break;
                    // tentative: column j-1 as if u_j were final
                    std::vector<double> col(j + 1);
                    for (int i = 0; i < j; ++i) col[i] = cpend[i];
                    col[j] = nupend;
                    for (int i = 0; i < j - 1; ++i) {
                        double a0 = col[i], a1 = col[i + 1];
                        col[i] = cs[i] * a0 + sn[i] * a1;
                        col[i + 1] = -sn[i] * a0 + cs[i] * a1;
                    }
                    double den = std::sqrt(col[j - 1] * col[j - 1] + col[j] * col[j]);
                    double tg = den > 0.0 ? std::fabs(g[j - 1] * col[j] / den) : 0.0;
                    if (tg <= 2.0 * tol) {
                        finish_column(j - 1);
                        if (stop) break;
                    }
                }
            }
            double* uj = V + (long)j * n;
            double* zj = Z + (long)j * n;
            double* w = V + (long)(j + 1) * n;
            // clear the row's ready flag (no kernel of this solve writes row j
            // before the step queued below)
            *(volatile double*)(c.hpin + (size_t)Ctx::HROW * j + NPUB) = 0.0;
            mgr_apply_top(c, uj, zj, tr);
            matvec(c, tr, zj, nullptr, w, 1.0, 0.0);
            arnoldi_dots(n, V, n, j + 1, w, c.part.p, hb, s);
            // the norm's reduction also stores the step's coefficients to its pinned row
            arnoldi_update(n, V, n, j + 1, hb, w, c.part.p, hb + HN, hb + HC, hb, c.hpin_dev + (size_t)Ctx::HROW * j,
                           NPUB, s);
            scale_by_norm(n, hb + HN, w, s);
            while (rows < j && !stop) process_row(rows++);
        }
        if (!stop) {
            while (rows < jmax && !stop) process_row(rows++);
            if (!stop && k < jmax) finish_column(jmax - 1);
        }
        for (int i = k - 1; i >= 0; --i) {
            double t = g[i];
            for (int q = i + 1; q < k; ++q) t -= H[(size_t)i * m + q] * y[q];
            y[i] = t / H[(size_t)i * m + i];
        }
        MGR_HIP(hipMemcpyAsync(c.yd.p, y.data(), sizeof(double) * k, hipMemcpyHostToDevice, s));
        maxpy(n, Z, n, k, c.yd.p, -1.0, x, c.part.p, nullptr, s);
        // true residual
        double* r = V;
        matvec(c, tr, x, b, r, -1.0, 1.0);
        mdot(n, r, n, 1, r, c.part.p, hb + HS, s);
        truer = std::sqrt(read_scalar(hb + HS)) / bnorm;
        if (truer <= c.o.rtol) { converged = true; break; }
        if (iters >= c.o.maxiter) break;
        first = false;
    }
    inf.iterations = iters;
    inf.rel_res_est = est;
    inf.rel_res_true = truer;
    inf.status = converged ? MGR_OK : MGR_NOT_CONVERGED;
    if (info) *info = inf;
    return inf.status;
}

// Whether a sliced ELL copy pays (see ensure_ell) is decided here for the
// operators of the apply and of the FGMRES matvec, with one sync for all of
// them instead of one per operator on its first use inside a solve; the copies
// themselves are made on first use (no sync).
static void prepare_ell(Ctx& c) {
    std::vector<const DCsr*> ops;
    auto add = [&](const DCsr& A) {
        if (A.ell_state == 0 && ell_ok(A)) ops.push_back(&A);
    };
    auto add_amg = [&](const Amg& H) {
        for (const auto& L : H.lv) {
            add(L.A);
            add(L.P);
            add(L.R);
        }
    };
    if (c.b == 1) add(c.A0);
    for (const auto& l : c.L) {
        add(l.RJ);
        add(l.PJ);
        if (l.famg) add_amg(*l.famg);
    }
    add_amg(c.camg);
    Slots& S = c.slots;
    constexpr size_t BATCH = 24;   // two slots each
    for (size_t i0 = 0; i0 < ops.size(); i0 += BATCH) {
        const size_t i1 = std::min(ops.size(), i0 + BATCH);
        std::vector<long long*> slot(i1 - i0);
        std::vector<DArr<int>> tmp(i1 - i0);
        for (size_t i = i0; i < i1; ++i) {
            DCsr& M = const_cast<DCsr&>(*ops[i]);
            const int nsl = (M.nr + ELL_SLICE - 1) / ELL_SLICE;
            M.esw.alloc((size_t)nsl, c.s);
            ell_widths(M.nr, M.rp.p, M.esw.p, c.s);
            tmp[i - i0].alloc((size_t)nsl + 1, c.s);
            slot[i - i0] = S.take(2);
            scan_async(M.esw.p, tmp[i - i0].p, nsl, slot[i - i0], c.s);
        }
        S.sync("sliced ELL widths");
        for (size_t i = i0; i < i1; ++i) {
            DCsr& M = const_cast<DCsr&>(*ops[i]);
            const long used = (long)S.val(slot[i - i0]) * ELL_SLICE;
            if (!ell_pays(used, M.nnz)) {
                M.esw.reset();
                M.ell_state = -1;
            } else {
                M.ell_state = 1;
            }
        }
    }
}

// ====================================================================== setup
static void build_hierarchy(Ctx& c);

// Scalar level-0 operator from the block-CSR input (exact zeros inside blocks
// left out, the diagonal kept).
static void expand_input(Ctx& c) {
    hipStream_t s = c.s;
    DArr<int> cnt((size_t)c.n + 1, s);
    bsr_count(c.b, c.nbr, c.nnzb, c.Arp.p, c.Aci.p, in_values(c), cnt.p, s);
    Pend pe = csr_begin(c.A0, c.n, c.n, cnt.p, c.slots);
    c.slots.sync("input matrix");
    csr_finish(pe, c.slots);
    bsr_fill(c.b, c.nbr, c.nnzb, c.Arp.p, c.Aci.p, in_values(c), c.A0, s);
}

// The scalar level-0 operator is needed for a plain CSR input (its matvec and
// first level) and for an AMG without MGR levels; the first MGR level of a
// block input is extracted from the blocks directly, and then only the label
// histogram (which sizes the levels) has to reach the host.
// The library's copy of the input values (c.Av): a block input with MGR
// levels gets it from its first block extraction (which reads every block);
// otherwise a copy on the auxiliary stream.  Until then setup steps read the
// caller's array.
static void copy_input_values(Ctx& c, const double* values, int nlevels) {
    c.Avin = values;
    if (c.b > 1 && nlevels > 0) {
        c.copy_in_extract = true;
        return;
    }
    aux_fork(c);
    MGR_HIP(hipMemcpyAsync(c.Av.p, values, sizeof(double) * c.nnzb * c.b * c.b, hipMemcpyDeviceToDevice, c.aux));
}

static void prepare_input(Ctx& c, int nlevels) {
    if (c.b == 1 || nlevels == 0) {
        expand_input(c);
        return;
    }
    c.A0 = DCsr();
    c.slots.sync("input labels");
}

static void setup(Ctx& c, const mgr_matrix* A, const int32_t* field, int32_t nlevels, const mgr_level_opts* lvl,
                  const int32_t* block) {
    hipStream_t s = c.s;
    if (!A || !field) throw Error(MGR_ERR_ARG, "null matrix or field array");
    if (A->block_size < 1 || A->block_size > 4) throw Error(MGR_ERR_ARG, "block_size must be 1..4");
    if (A->n_block_rows <= 0 || !A->row_ptr || !A->col_idx || !A->values) throw Error(MGR_ERR_ARG, "empty matrix");
    if (nlevels < 0 || nlevels > 8 || (nlevels > 0 && !lvl)) throw Error(MGR_ERR_ARG, "nlevels must be 0..8");
    if (c.o.restart < 1 || c.o.restart > 63) throw Error(MGR_ERR_ARG, "restart must be 1..63");
    for (int l = 0; l < nlevels; ++l) {
        if (lvl[l].sweeps < 1) throw Error(MGR_ERR_ARG, "sweeps must be >= 1");
        if (lvl[l].frelax < 0 || lvl[l].frelax > 3) throw Error(MGR_ERR_ARG, "unknown F-relaxation");
        if (lvl[l].restrict_type < 0 || lvl[l].restrict_type > 1) throw Error(MGR_ERR_ARG, "unknown restriction");
        if (lvl[l].f_field_mask == 0) throw Error(MGR_ERR_BAD_LABELS, "empty F-field mask");
        if (lvl[l].amg_agg_levels < 0) throw Error(MGR_ERR_ARG, "amg_agg_levels must be >= 0");
        if (lvl[l].amg_unknown_based < MGR_AMG_SCALAR || lvl[l].amg_unknown_based > MGR_AMG_SEPARATE)
            throw Error(MGR_ERR_ARG, "unknown AMG kind of an F-relaxation level");
    }
    c.ready = false;
    c.L.clear();
    c.camg = Amg();
    c.have_At = false;
    c.b = A->block_size;
    c.nbr = A->n_block_rows;
    c.n = c.b * c.nbr;
    c.Arp.alloc((size_t)c.nbr + 1, s);
    MGR_HIP(hipMemcpyAsync(c.Arp.p, A->row_ptr, sizeof(int) * ((size_t)c.nbr + 1), hipMemcpyDeviceToDevice, s));
    c.nnzb = read_int(c.Arp.p + c.nbr, s);
    if (c.nnzb <= 0) throw Error(MGR_ERR_ARG, "matrix has no entries");
    long bb = (long)c.b * c.b;
    c.Aci.alloc((size_t)c.nnzb, s);
    c.Av.alloc((size_t)c.nnzb * bb, s);
    MGR_HIP(hipMemcpyAsync(c.Aci.p, A->col_idx, sizeof(int) * c.nnzb, hipMemcpyDeviceToDevice, s));
    // the values (the bulk of the input) are copied by the first block
    // extraction, or else on the auxiliary stream, while the setup reads the
    // caller's array
    AuxScope aux_scope{c};
    copy_input_values(c, A->values, nlevels);
    if (c.nnzb * bb > INT_MAX) throw Error(MGR_ERR_UNSUPPORTED, "more than 2^31 scalar entries");
    c.field0.alloc((size_t)c.n, s);
    MGR_HIP(hipMemcpyAsync(c.field0.p, field, sizeof(int) * c.n, hipMemcpyDeviceToDevice, s));
    if (block) {
        c.block0.alloc((size_t)c.n, s);
        MGR_HIP(hipMemcpyAsync(c.block0.p, block, sizeof(int) * c.n, hipMemcpyDeviceToDevice, s));
    } else {
        c.block0.reset();
    }
    // the label histogram reaches the host with the input matrix's sync
    if (!c.fhist_h) MGR_HIP(hipHostMalloc(reinterpret_cast<void**>(&c.fhist_h), sizeof(int) * 32, hipHostMallocDefault));
    c.fhist.alloc(32, s);
    field_hist(c.n, c.field0.p, c.fhist.p, c.slots.flag(), s);
    MGR_HIP(hipMemcpyAsync(c.fhist_h, c.fhist.p, sizeof(int) * 32, hipMemcpyDeviceToHost, s));
    prepare_input(c, nlevels);
    c.lvl.assign(lvl, lvl + nlevels);
    build_hierarchy(c);
}

// coarse-AMG level size from which the held-back auxiliary-stream work runs
// (one piece per level; on larger levels the pieces slow the level's own
// bandwidth-bound kernels more than they gain)
constexpr int AUX_DEFER_ROWS = 20000;

// The MGR levels and the coarse AMG on the current input (c.A0, c.field0, c.lvl);
// AMG hierarchies found in c.reuse_* are reused instead of coarsened again.
static void build_hierarchy(Ctx& c) {
    hipStream_t s = c.s;
    c.warm[0] = c.warm[1] = false;
    const int nlevels = (int)c.lvl.size();
    const mgr_level_opts* lvl = c.lvl.data();
    DArr<int> fld((size_t)c.n, s), blk((size_t)c.n, s);
    MGR_HIP(hipMemcpyAsync(fld.p, c.field0.p, sizeof(int) * c.n, hipMemcpyDeviceToDevice, s));
    if (c.block0.p) MGR_HIP(hipMemcpyAsync(blk.p, c.block0.p, sizeof(int) * c.n, hipMemcpyDeviceToDevice, s));
    else iota_div(c.n, c.b, blk.p, s);
    // a block input's first level is extracted from the blocks themselves
    const DCsr* cur = c.A0.nr ? &c.A0 : nullptr;
    DCsr next;
    c.L.resize(nlevels);
    uint32_t used = 0;  // fields that were F on an earlier level
    for (int l = 0; l < nlevels; ++l) {
        // F-points of this level: the remaining points whose field is in the mask
        long nF = 0, nrem = 0;
        for (int f = 0; f < 32; ++f) {
            if ((used >> f) & 1u) continue;
            nrem += c.fhist_h[f];
            if ((lvl[l].f_field_mask >> f) & 1u) nF += c.fhist_h[f];
        }
        used |= lvl[l].f_field_mask;
        if (nrem != (cur ? cur->nr : c.n)) throw Error(MGR_ERR_ARG, "internal: label histogram and level size differ");
        DCsr Ac = mgr_setup_level(c, c.L[l], cur, fld.p, blk.p, lvl[l], l, (int)nF);
        MgrLevel& L = c.L[l];
        DArr<int> f2((size_t)L.nC, s), b2((size_t)L.nC, s);
        gather_int(L.nC, L.cmap.p, fld.p, f2.p, s);
        gather_int(L.nC, L.cmap.p, blk.p, b2.p, s);
        fld = std::move(f2);
        blk = std::move(b2);
        if (l + 1 < nlevels) {
            L.Aout = std::move(Ac);
            cur = &L.Aout;
        } else {
            next = std::move(Ac);
            cur = &next;
        }
    }
    c.slots.level_hook = [&c](int n) {
        if (n <= AUX_DEFER_ROWS) run_deferred(c, 1);
    };
    if (c.reuse_camg) {
        c.camg = std::move(*c.reuse_camg);
        c.reuse_camg.reset();
        amg_refresh(c.camg, nlevels > 0 ? std::move(next) : csr_copy(c.A0, s), c.slots);
    } else {
        amg_setup(c.camg, nlevels > 0 ? std::move(next) : csr_copy(c.A0, s),
                  c.o.amg.unknown_based ? fld.p : nullptr, c.o.amg, c.o.amg.seed, c.slots);
    }
    c.slots.level_hook = nullptr;
    run_deferred(c);
    c.reuse_famg.clear();
    c.Avin = nullptr;
    if (c.o.apply_precision == 32) {
        // the FP32 copies on the auxiliary stream, beside the sliced-ELL sizing
        aux_fork(c);
        F32Batch fb;
        for (auto& l : c.L) mgr_level_make_float(c, l, fb);
        amg_make_float(c.camg, s, fb);
        fb.flush(c.aux);
    }
    prepare_ell(c);
    aux_join(c);
    MGR_HIP(hipStreamSynchronize(s));
    c.ready = true;
}

// Setup reuse (Sec. 3.3 and Sec. 4.4: AMG data reuse across Newton solves): new
// values on the pattern of the last setup.  The MGR levels are formed again;
// the coarse AMG keeps its C/F splits and interpolation and forms its Galerkin
// products anew; the F-relaxation AMG hierarchies do the same, or are kept
// whole with MGR_REUSE_KEEP_FRELAX_AMG (their A_FF unchanged).
static void update_values(Ctx& c, const double* values, int flags) {
    hipStream_t s = c.s;
    if (!c.ready) throw Error(MGR_ERR_ARG, "update before setup");
    if (!values) throw Error(MGR_ERR_ARG, "null values");
    if (flags & ~MGR_REUSE_KEEP_FRELAX_AMG) throw Error(MGR_ERR_ARG, "unknown reuse flags");
    c.ready = false;
    AuxScope aux_scope{c};
    copy_input_values(c, values, (int)c.lvl.size());
    prepare_input(c, (int)c.lvl.size());
    c.A0t = DCsr();
    c.ATrp.reset(); c.ATci.reset(); c.ATv.reset();
    c.have_At = false;
    c.reuse_famg.clear();
    c.reuse_famg.resize(c.L.size());
    for (size_t l = 0; l < c.L.size(); ++l) c.reuse_famg[l] = std::move(c.L[l].famg);
    c.reuse_camg.reset(new Amg(std::move(c.camg)));
    c.reuse_keep_famg = (flags & MGR_REUSE_KEEP_FRELAX_AMG) != 0;
    c.L.clear();
    c.camg = Amg();
    try {
        build_hierarchy(c);
    } catch (...) {
        c.reuse_famg.clear();
        c.reuse_camg.reset();
        throw;
    }
}

// ====================================================================== export
static void export_csr(const DCsr& A, int64_t* sizes, void* b0, void* b1, void* b2, hipStream_t s) {
    sizes[0] = A.nr;
    sizes[1] = A.nc;
    sizes[2] = A.nnz;
    if (b0 && A.rp.p) MGR_HIP(hipMemcpyAsync(b0, A.rp.p, sizeof(int) * ((size_t)A.nr + 1), hipMemcpyDeviceToHost, s));
    if (b1 && A.nnz > 0) MGR_HIP(hipMemcpyAsync(b1, A.ci.p, sizeof(int) * A.nnz, hipMemcpyDeviceToHost, s));
    if (b2 && A.nnz > 0) MGR_HIP(hipMemcpyAsync(b2, A.v.p, sizeof(double) * A.nnz, hipMemcpyDeviceToHost, s));
    MGR_HIP(hipStreamSynchronize(s));
}

static int do_export(Ctx& c, int kind, int level, int what, int sub, int64_t* sizes, void* b0, void* b1,
                     void* b2) {
    hipStream_t s = c.s;
    if (!c.ready) throw Error(MGR_ERR_ARG, "export before setup");
    if (kind == 0) {
        if (level < 0 || level >= (int)c.L.size()) throw Error(MGR_ERR_ARG, "no such MGR level");
        MgrLevel& l = c.L[level];
        if (what == 0) {
            sizes[0] = l.n; sizes[1] = 0; sizes[2] = 0;
            if (b0) {
                std::vector<int> t(l.n);
                MGR_HIP(hipMemcpyAsync(t.data(), l.isF.p, sizeof(int) * l.n, hipMemcpyDeviceToHost, s));
                MGR_HIP(hipStreamSynchronize(s));
                int* o = (int*)b0;
                for (int i = 0; i < l.n; ++i) o[i] = t[i] ? 0 : 1;
            }
            return MGR_OK;
        }
        const DCsr* A = nullptr;
        if (what == 1) A = (level + 1 < (int)c.L.size()) ? &l.Aout : &c.camg.lv[0].A;
        if (what == 2) A = &l.PF;
        if (what == 3) A = &l.RF;
        if (what == 4) {
            ensure_full_aff(c, level);
            A = &l.AFF;
        }
        if (what == 5) A = &l.M;
        if ((what == 6 || what == 7) && !l.fused) throw Error(MGR_ERR_ARG, "level has no fused apply operators");
        if (what == 6) A = &l.RJ;
        if (what == 7) A = &l.PJ;
        if (what == 8) A = &l.AFC;
        if (what == 9) A = &l.ACF;
        if (what == 10) A = &l.ACC;
        if (!A) throw Error(MGR_ERR_ARG, "unknown export item");
        export_csr(*A, sizes, b0, b1, b2, s);
        return MGR_OK;
    }
    Amg* H = (kind == 1) ? &c.camg : ((sub >= 0 && sub < (int)c.L.size()) ? c.L[sub].famg.get() : nullptr);
    if (!H || level < 0 || level >= (int)H->lv.size()) throw Error(MGR_ERR_ARG, "no such AMG level");
    AmgLevel& L = H->lv[level];
    if (what == 0) {
        if (level + 1 >= (int)H->lv.size()) throw Error(MGR_ERR_ARG, "coarsest AMG level has no C/F split");
        sizes[0] = L.n; sizes[1] = 0; sizes[2] = 0;
        if (b0) {
            MGR_HIP(hipMemcpyAsync(b0, L.cf.p, sizeof(int) * L.n, hipMemcpyDeviceToHost, s));
            MGR_HIP(hipStreamSynchronize(s));
        }
        return MGR_OK;
    }
    if (what == 1) { export_csr(L.A, sizes, b0, b1, b2, s); return MGR_OK; }
    if (what == 2 && level + 1 < (int)H->lv.size()) { export_csr(L.P, sizes, b0, b1, b2, s); return MGR_OK; }
    if ((what == 4 || what == 5) && level + 1 < (int)H->lv.size()) {
        // composed form of the level: G, or [W | Q]; the level above the
        // coarsest whose cycle is one dense operator reports G and [W | Q] too
        if (!L.composed) throw Error(MGR_ERR_ARG, "level is not applied in composed form");
        export_csr(what == 4 ? L.G : L.WQ, sizes, b0, b1, b2, s);
        return MGR_OK;
    }
    if (what == 6) {
        // the dense cycle operator T = W + Q C^-1 G of the level above the coarsest
        if (level != H->tail) throw Error(MGR_ERR_ARG, "level has no dense cycle operator");
        sizes[0] = L.n; sizes[1] = L.n; sizes[2] = (int64_t)L.n * L.n;
        if (b2) MGR_HIP(hipMemcpyAsync(b2, H->td.p, sizeof(double) * L.n * L.n, hipMemcpyDeviceToHost, s));
        MGR_HIP(hipStreamSynchronize(s));
        return MGR_OK;
    }
    if ((what == 7 || what == 8) && level + 1 < (int)H->lv.size()) {
        // slot tables of the hybrid Gauss-Seidel sweeps on A (7: forward, the
        // in-chunk entries left of the diagonal; 8: backward, right of it):
        // rows = chunk positions x table chunks, cols = slots per row
        if (H->smoother != MGR_SMOOTH_HYBRID_GS || !L.dT.p) throw Error(MGR_ERR_ARG, "level has no Gauss-Seidel tables");
        const HgsTri& t = what == 7 ? L.lo : L.up;
        const long per = (long)H->chunk * L.nchp;
        sizes[0] = per; sizes[1] = t.w; sizes[2] = per * t.w;
        const size_t m = (size_t)per * t.w;
        if (b1 && m) {
            std::vector<unsigned char> cc(m);
            MGR_HIP(hipMemcpyAsync(cc.data(), t.c.p, m, hipMemcpyDeviceToHost, s));
            MGR_HIP(hipStreamSynchronize(s));
            int* o = (int*)b1;
            for (size_t q = 0; q < m; ++q) o[q] = cc[q];
        }
        if (b2 && m) MGR_HIP(hipMemcpyAsync(b2, t.v.p, sizeof(double) * m, hipMemcpyDeviceToHost, s));
        MGR_HIP(hipStreamSynchronize(s));
        return MGR_OK;
    }
    if (what == 3 && level + 1 == (int)H->lv.size()) {
        // the coarsest level's dense inverse, n x n row-major in b2
        sizes[0] = H->nc; sizes[1] = H->nc; sizes[2] = (int64_t)H->nc * H->nc;
        if (b2 && H->nc > 0)
            MGR_HIP(hipMemcpyAsync(b2, H->cinv.p, sizeof(double) * H->nc * H->nc, hipMemcpyDeviceToHost, s));
        MGR_HIP(hipStreamSynchronize(s));
        return MGR_OK;
    }
    throw Error(MGR_ERR_ARG, "unknown export item");
}

}  // namespace mgr

// ====================================================================== C-ABI
struct mgr_ctx {
    mgr::Ctx c;
};

using mgr::Error;

template <typename F>
static int guarded(mgr_handle h, F&& f) {
    if (!h) return MGR_ERR_ARG;
    // device arrays made during the call come from the context's block cache
    struct CacheScope {
        mgr::BlockCache* prev;
        explicit CacheScope(mgr::BlockCache* c) : prev(mgr::tl_cache) { mgr::tl_cache = c; }
        ~CacheScope() { mgr::tl_cache = prev; }
    } scope(&h->c.cache);
    try {
        h->c.err.clear();
        return f();
    } catch (const Error& e) {
        h->c.err = e.what();
        return e.code;
    } catch (const std::exception& e) {
        h->c.err = e.what();
        return MGR_ERR_HIP;
    }
}

extern "C" {

void mgr_default_opts(mgr_opts* o) {
    if (!o) return;
    std::memset(o, 0, sizeof(*o));
    o->apply_precision = 64;
    o->restart = 50;
    o->maxiter = 1000;
    o->rtol = 1e-8;
    o->ortho = MGR_ORTHO_CGS2;
    o->amg.theta = 0.25;
    o->amg.max_levels = 25;
    o->amg.max_coarse = 128;
    o->amg.nu_pre = 1;
    o->amg.nu_post = 1;
    o->amg.unknown_based = 0;
    o->amg.interp = MGR_INTERP_DIRECT;
    o->amg.smoother = MGR_SMOOTH_L1_JACOBI;
    o->amg.gs_chunk = 32;
    o->amg.agg_levels = 0;
    o->amg.seed = 12345;
}

static int check_opts(const mgr_opts* o) {
    if (o->apply_precision != 32 && o->apply_precision != 64) return MGR_ERR_ARG;
    if (o->restart < 1 || o->restart > 63 || o->maxiter < 1 || !(o->rtol >= 0.0)) return MGR_ERR_ARG;
    if (o->amg.max_levels < 1 || o->amg.max_coarse < 1 || o->amg.nu_pre < 0 || o->amg.nu_post < 0) return MGR_ERR_ARG;
    if (o->amg.interp != MGR_INTERP_DIRECT && o->amg.interp != MGR_INTERP_EXT_I) return MGR_ERR_ARG;
    if (o->amg.smoother != MGR_SMOOTH_L1_JACOBI && o->amg.smoother != MGR_SMOOTH_HYBRID_GS) return MGR_ERR_ARG;
    if (o->amg.agg_levels < 0) return MGR_ERR_ARG;
    if (o->amg.smoother == MGR_SMOOTH_HYBRID_GS && (o->amg.gs_chunk < 1 || o->amg.gs_chunk > mgr::HGS_CHUNK_MAX))
        return MGR_ERR_ARG;
    return MGR_OK;
}

int mgr_create(mgr_handle* h, const mgr_opts* o, void* hip_stream, mgr_alloc_fn alloc, mgr_free_fn free_,
               void* alloc_ctx) {
    if (!h) return MGR_ERR_ARG;
    *h = nullptr;
    if ((alloc == nullptr) != (free_ == nullptr)) return MGR_ERR_ARG;
    mgr_opts d;
    mgr_default_opts(&d);
    if (o) {
        if (check_opts(o) != MGR_OK) return MGR_ERR_ARG;
        d = *o;
    }
    mgr_ctx* c = new (std::nothrow) mgr_ctx();
    if (!c) return MGR_ERR_OOM;
    c->c.s = (hipStream_t)hip_stream;
    c->c.cache.s = c->c.s;
    c->c.cache.af = alloc;
    c->c.cache.ff = free_;
    c->c.cache.actx = alloc_ctx;
    c->c.o = d;
    // the handle's own arrays made here come from its block cache too
    mgr::BlockCache* prev_cache = mgr::tl_cache;
    mgr::tl_cache = &c->c.cache;
    try {
        // keep freed blocks in the stream-ordered pool across synchronisations:
        // a setup re-allocates the same sizes every time it runs
        int dev = 0;
        MGR_HIP(hipGetDevice(&dev));
        hipMemPool_t pool;
        MGR_HIP(hipDeviceGetDefaultMemPool(&pool, dev));
        uint64_t thr = UINT64_MAX;
        MGR_HIP(hipMemPoolSetAttribute(pool, hipMemPoolAttrReleaseThreshold, &thr));
        c->c.slots.init(c->c.s);
        // this device's scratch array of the no-allocation apply, and room for
        // the addresses it swaps (so that call allocates no host memory either)
        c->c.scratch = mgr::scratch_for_device(dev);
        c->c.saved_d.reserve(4096);
        c->c.saved_f.reserve(4096);
        hipError_t e = hipStreamSynchronize(c->c.s);
        if (e != hipSuccess) throw Error(MGR_ERR_HIP, hipGetErrorString(e));
    } catch (const Error& e) {
        mgr::tl_cache = prev_cache;
        delete c;
        return e.code;
    } catch (...) {
        mgr::tl_cache = prev_cache;
        delete c;
        return MGR_ERR_HIP;
    }
    mgr::tl_cache = prev_cache;
    *h = c;
    return MGR_OK;
}

int mgr_set_opts(mgr_handle h, const mgr_opts* o) {
    return guarded(h, [&]() {
        if (!o || check_opts(o) != MGR_OK) throw Error(MGR_ERR_ARG, "invalid options");
        // another apply precision reads other operator copies, made by the next apply
        if (o->apply_precision != h->c.o.apply_precision) h->c.warm[0] = h->c.warm[1] = false;
        h->c.o = *o;
        return MGR_OK;
    });
}

int mgr_setup(mgr_handle h, const mgr_matrix* A, const int32_t* field_of_dof, int32_t nlevels,
              const mgr_level_opts* lvl, const int32_t* block_of_dof) {
    return guarded(h, [&]() {
        mgr::setup(h->c, A, field_of_dof, nlevels, lvl, block_of_dof);
        return MGR_OK;
    });
}

int mgr_update_values(mgr_handle h, const double* values, int32_t flags) {
    return guarded(h, [&]() {
        mgr::update_values(h->c, values, flags);
        return MGR_OK;
    });
}

int mgr_apply(mgr_handle h, const double* r, double* z) {
    return guarded(h, [&]() {
        if (!r || !z) throw Error(MGR_ERR_ARG, "null vector");
        mgr::mgr_apply_top(h->c, r, z, false);
        return MGR_OK;
    });
}

int mgr_apply_noalloc(mgr_handle h, const double* r, double* z) {
    return guarded(h, [&]() {
        if (!r || !z) throw Error(MGR_ERR_ARG, "null vector");
        mgr::mgr_apply_noalloc_impl(h->c, r, z);
        return MGR_OK;
    });
}

int mgr_apply_transpose(mgr_handle h, const double* r, double* z) {
    return guarded(h, [&]() {
        if (!r || !z) throw Error(MGR_ERR_ARG, "null vector");
        mgr::mgr_apply_top(h->c, r, z, true);
        return MGR_OK;
    });
}

int mgr_matvec(mgr_handle h, int32_t trans, const double* x, double* y) {
    return guarded(h, [&]() {
        if (!h->c.ready) throw Error(MGR_ERR_ARG, "matvec before setup");
        if (!x || !y) throw Error(MGR_ERR_ARG, "null vector");
        mgr::matvec(h->c, trans != 0, x, nullptr, y, 1.0, 0.0);
        return MGR_OK;
    });
}

static int solve_impl(mgr_handle h, bool tr, int32_t nrhs, const double* B, double* X, mgr_solve_info* info) {
    return guarded(h, [&]() {
        if (!h->c.ready) throw Error(MGR_ERR_ARG, "solve before setup");
        if (nrhs < 1 || !B || !X) throw Error(MGR_ERR_ARG, "bad right-hand sides");
        int st = MGR_OK;
        for (int k = 0; k < nrhs; ++k) {
            mgr_solve_info inf{};
            int r = mgr::fgmres(h->c, tr, B + (long)k * h->c.n, X + (long)k * h->c.n, &inf);
            if (info) info[k] = inf;
            if (r != MGR_OK) st = r;
        }
        return st;
    });
}

int mgr_solve(mgr_handle h, int32_t nrhs, const double* B, double* X, mgr_solve_info* info) {
    return solve_impl(h, false, nrhs, B, X, info);
}

int mgr_solve_transpose(mgr_handle h, int32_t nrhs, const double* B, double* X, mgr_solve_info* info) {
    return solve_impl(h, true, nrhs, B, X, info);
}

int mgr_grad_values(mgr_handle h, int32_t nrhs, const double* Lam, const double* X, double* dvalues) {
    return guarded(h, [&]() {
        mgr::Ctx& c = h->c;
        if (!c.ready) throw Error(MGR_ERR_ARG, "grad before setup");
        if (nrhs < 1 || !Lam || !X || !dvalues) throw Error(MGR_ERR_ARG, "bad arguments");
        mgr::grad_values(c.b, c.nbr, c.Arp.p, c.Aci.p, c.nnzb, nrhs, Lam, X, dvalues, c.s);
        return MGR_OK;
    });
}

int mgr_hierarchy_info(mgr_handle h, int64_t* out, int32_t cap) {
    return guarded(h, [&]() {
        mgr::Ctx& c = h->c;
        if (!c.ready) throw Error(MGR_ERR_ARG, "info before setup");
        if (!out || cap < 2) throw Error(MGR_ERR_ARG, "bad buffer");
        int o = 0;
        out[o++] = (int64_t)c.L.size();
        out[o++] = (int64_t)c.camg.lv.size();
        for (size_t l = 0; l < c.L.size() && o + 4 <= cap; ++l) {
            out[o++] = c.L[l].n;
            out[o++] = c.L[l].nF;
            out[o++] = c.L[l].nC;
            out[o++] = (l + 1 < c.L.size()) ? c.L[l].Aout.nnz : c.camg.lv[0].A.nnz;
        }
        for (size_t k = 0; k < c.camg.lv.size() && o + 2 <= cap; ++k) {
            out[o++] = c.camg.lv[k].n;
            out[o++] = c.camg.lv[k].A.nnz;
        }
        return o;
    });
}

int mgr_export(mgr_handle h, int32_t kind, int32_t level, int32_t what, int32_t sub, int64_t* sizes, void* b0,
               void* b1, void* b2) {
    return guarded(h, [&]() {
        if (!sizes) throw Error(MGR_ERR_ARG, "null sizes");
        return mgr::do_export(h->c, kind, level, what, sub, sizes, b0, b1, b2);
    });
}

const char* mgr_last_error(mgr_handle h) { return h ? h->c.err.c_str() : "null handle"; }

void mgr_destroy(mgr_handle h) {
    if (!h) return;
    hipStream_t s = h->c.s;
    (void)hipStreamSynchronize(s);
    delete h;
    (void)hipStreamSynchronize(s);
}

}  // extern "C"
