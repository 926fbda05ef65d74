// k_apply.hip -- solve-phase kernels for gfx950: CSR / block-CSR SpMV variants
// (FGMRES matvec, MGR restriction / interpolation, AMG residual, transfer and
// L1-Jacobi smoothing), the coarsest dense apply, the FGMRES vector kernels
// (multi-dot, multi-axpy, norms) and the adjoint gradient.
//
// Every solve-phase kernel is bound by HBM bandwidth (about 0.1-0.3 flop per
// byte), so the designs favour coalesced streaming of the matrix arrays,
// sub-wavefront row groups sized to the row length and fused vector updates;
// there is no dense contraction here that the matrix cores could speed up.
#include <climits>

#include "apply.hpp"

namespace mgr {

namespace {

constexpr int TPB = 256;
constexpr int WAVE = 64;

template <typename T>
__device__ inline T group_sum(T v, int G) {
    for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, G);
    return v;
}

// ---------------------------------------------------------------- CSR-stream SpMV
// Rows are partitioned into row blocks of about SPMV_CHUNK nonzeros, a row
// itself counting as 1/SPMV_ROW_COST of a nonzero so that mostly empty rows
// still spread over many blocks (rowblocks(), made once per operator).  A
// workgroup streams its block's nonzeros with fully coalesced loads of the
// values and column indices, forms the products in LDS, then reduces the rows:
// one thread per row when the block holds many short rows, a power-of-two lane
// group per row otherwise.  A block whose nonzeros exceed the LDS stage (a
// long row) is reduced row by row across the whole workgroup.
//
// The product and the row epilogue are supplied by an operation class:
//   SpmvOp     y = alpha * A [x | x2] + beta * w   (w may alias y)
//   JacobiOp   y = x + dinv .* (b - A x)          (one L1-Jacobi sweep, out of place)
//   PreOp      x = dinv .* b,  r = b - A x        (first sweep from zero + residual)
// Every operation splits its row epilogue in two: pre(r) loads the vectors the
// epilogue reads (issued by the kernels before their gathers, so those loads
// overlap the row's products instead of following them), fin(r, s, p) forms
// and stores the row's results; done(r, s) = fin(r, s, pre(r)).
template <typename MT, typename XT, typename X2T, typename YT, typename WT>
struct SpmvOp {
    const XT* x; const X2T* x2; int split; const WT* w; YT* y; MT alpha, beta;
    struct Pre { MT w; };
    __device__ MT xval(int c) const { return (c < split) ? (MT)x[c] : (MT)x2[c - split]; }
    __device__ Pre pre(int r) const { return Pre{w ? (MT)w[r] : MT(0)}; }
    __device__ void fin(int r, MT s, const Pre& p) const {
        MT o = alpha * s;
        if (w) o += beta * p.w;
        y[r] = (YT)o;
    }
    __device__ void done(int r, MT s) const { fin(r, s, pre(r)); }
};

template <typename T>
struct JacobiOp {
    const T* dinv; const T* b; const T* x; T* y;
    struct Pre { T d, b, x; };
    __device__ T xval(int c) const { return x[c]; }
    __device__ Pre pre(int r) const { return Pre{dinv[r], b[r], x[r]}; }
    __device__ void fin(int r, T s, const Pre& p) const { y[r] = p.x + p.d * (p.b - s); }
    __device__ void done(int r, T s) const { fin(r, s, pre(r)); }
};

template <typename T>
struct PreOp {
    const T* dinv; const T* b; T* x; T* r_;
    struct Pre { T d, b; };
    __device__ T xval(int c) const { return dinv[c] * b[c]; }
    __device__ Pre pre(int r) const { return Pre{dinv[r], b[r]}; }
    __device__ void fin(int r, T s, const Pre& p) const {
        x[r] = p.d * p.b;
        r_[r] = p.b - s;
    }
    __device__ void done(int r, T s) const { fin(r, s, pre(r)); }
};

// RestrictOp  y = A x  and  yd = dsc .* y  (the next level's D^-1 b); x may be
// FP64 while the operator is FP32 (the first MGR restriction of the FP32 apply)
template <typename T, typename XT>
struct RestrictOp {
    const XT* x; const T* dsc; T* y; T* yd;
    struct Pre { T d; };
    __device__ T xval(int c) const { return (T)x[c]; }
    __device__ Pre pre(int r) const { return Pre{dsc[r]}; }
    __device__ void fin(int r, T s, const Pre& p) const {
        y[r] = s;
        yd[r] = p.d * s;
    }
    __device__ void done(int r, T s) const { fin(r, s, pre(r)); }
};

// PreOpD  x = bd,  r = b - A bd  with bd = dinv .* b already formed
template <typename T>
struct PreOpD {
    const T* bd; const T* b; T* x; T* r_;
    struct Pre { T bd, b; };
    __device__ T xval(int c) const { return bd[c]; }
    __device__ Pre pre(int r) const { return Pre{bd[r], b[r]}; }
    __device__ void fin(int r, T s, const Pre& p) const {
        x[r] = p.bd;
        r_[r] = p.b - s;
    }
    __device__ void done(int r, T s) const { fin(r, s, pre(r)); }
};

template <typename MT, int TAG, class Op>
__global__ __launch_bounds__(TPB) void k_spmv_stream(const int* __restrict__ blk, const int* __restrict__ bpos,
                                                     const int* __restrict__ rp, const int* __restrict__ ci,
                                                     const MT* __restrict__ v, Op op) {
    __shared__ MT sh[SPMV_LDS];
    __shared__ MT red[TPB / WAVE];
    const int tid = threadIdx.x;
    // the block's rows and entries, four independent loads
    const int r0 = blk[blockIdx.x], r1 = blk[blockIdx.x + 1];
    const int p0 = bpos[blockIdx.x], p1 = bpos[blockIdx.x + 1];
    if (r0 >= r1) return;
    const int nnz = p1 - p0;
    if (nnz <= SPMV_LDS) {
        // the epilogue inputs of the (first) row this thread finishes, loaded
        // with the entries
        const int nrows = r1 - r0;
        int G = 64;
        while (G > 1 && G * nrows > TPB) G >>= 1;
        const int rl = tid / G, lane = tid & (G - 1);
        // and, with FP64 values, the bounds of that row, so that the reduction
        // after the barrier starts without a memory round trip (measured: the
        // FP64 applies 3-4% faster, the FP32 ones 1-6% slower, so FP32 blocks
        // read the bounds after the barrier)
        constexpr bool early = sizeof(MT) == 8;
        typename Op::Pre pre{};
        int rs = 0, re = 0;
        if (nrows > TPB / 4) {
            if (r0 + tid < r1) {
                pre = op.pre(r0 + tid);
                if (early) {
                    rs = rp[r0 + tid];
                    re = rp[r0 + tid + 1];
                }
            }
        } else if (rl < nrows) {
            if (lane == 0) pre = op.pre(r0 + rl);
            if (early) {
                rs = rp[r0 + rl];
                re = rp[r0 + rl + 1];
            }
        }
        // issue every index and value load of this thread before the gathers
        constexpr int PER = SPMV_LDS / TPB;
        int cc[PER];
        MT vv[PER];
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            int q = tid + t * TPB;
            if (q < nnz) { cc[t] = ci[p0 + q]; vv[t] = v[p0 + q]; }
        }
#pragma unroll
        for (int t = 0; t < PER; ++t) {
            int q = tid + t * TPB;
            if (q < nnz) sh[q] = vv[t] * op.xval(cc[t]);
        }
        __syncthreads();
        if (nrows > TPB / 4) {
            for (int r = r0 + tid; r < r1; r += TPB) {
                MT s = MT(0);
                const bool first = r == r0 + tid;
                const int qe = (first && early ? re : rp[r + 1]) - p0;
                for (int q = (first && early ? rs : rp[r]) - p0; q < qe; ++q) s += sh[q];
                if (first) op.fin(r, s, pre);
                else op.done(r, s);
            }
        } else {
            int r = r0 + rl;
            MT s = MT(0);
            if (rl < nrows) {
                const int qe = (early ? re : rp[r + 1]) - p0;
                for (int q = (early ? rs : rp[r]) - p0 + lane; q < qe; q += G) s += sh[q];
            }
            for (int off = G >> 1; off > 0; off >>= 1) s += __shfl_xor(s, off, WAVE);
            if (rl < nrows && lane == 0) op.fin(r, s, pre);
        }
        return;
    }
    for (int r = r0; r < r1; ++r) {
        MT s = MT(0);
        for (int p = rp[r] + tid; p < rp[r + 1]; p += TPB) s += v[p] * op.xval(ci[p]);
        for (int off = WAVE / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, WAVE);
        if ((tid & (WAVE - 1)) == 0) red[tid / WAVE] = s;
        __syncthreads();
        if (tid == 0) {
            MT t = MT(0);
            for (int q = 0; q < TPB / WAVE; ++q) t += red[q];
            op.done(r, t);
        }
        __syncthreads();
    }
}

__global__ void k_rowblocks(int nr, int nb, const int* __restrict__ rp, int* __restrict__ blk,
                            int* __restrict__ bpos) {
    int b = blockIdx.x * blockDim.x + threadIdx.x;
    if (b > nb) return;
    if (b == nb) {
        blk[b] = nr;
        bpos[b] = rp[nr];
        return;
    }
    long target = (long)b * SPMV_CHUNK;
    int lo = 0, hi = nr;  // first row r in [0, nr] with cost(r) >= target
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if ((long)rp[mid] + mid / SPMV_ROW_COST < target) lo = mid + 1;
        else hi = mid;
    }
    blk[b] = lo;
    bpos[b] = rp[lo];
}

// Block-CSR SpMV, b x b row-major blocks, G lanes per block row:
// y = alpha * A x + beta * w.
template <int B, int G>
__global__ __launch_bounds__(TPB) void k_bsr_spmv(int nbr, const int* __restrict__ rp, const int* __restrict__ ci,
                                                  const double* __restrict__ v, const double* __restrict__ x,
                                                  const double* w, double* y, double alpha, double beta) {
    long gid = (long)blockIdx.x * TPB + threadIdx.x;
    int I = (int)(gid / G), lane = (int)(gid % G);
    if (I >= nbr) return;
    double s[B];
#pragma unroll
    for (int r = 0; r < B; ++r) s[r] = 0.0;
    for (int p = rp[I] + lane; p < rp[I + 1]; p += G) {
        int J = ci[p];
        const double* blk = v + (long)p * B * B;
        double xv[B];
#pragma unroll
        for (int c = 0; c < B; ++c) xv[c] = x[(long)J * B + c];
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int c = 0; c < B; ++c) s[r] += blk[r * B + c] * xv[c];
    }
#pragma unroll
    for (int r = 0; r < B; ++r) s[r] = group_sum<double>(s[r], G);
#pragma unroll
    for (int r = 0; r < B; ++r)
        if (r % G == lane) {
            long i = (long)I * B + r;
            double o = alpha * s[r];
            if (w) o += beta * w[i];
            y[i] = o;
        }
}

// Coarsest level: y = Minv x with a dense n x n inverse, one wavefront per row.
template <typename T, typename XT>
__global__ __launch_bounds__(TPB) void k_dense_gemv(int n, const T* __restrict__ m, const XT* __restrict__ x,
                                                    T* __restrict__ y) {
    int row = blockIdx.x * (TPB / WAVE) + threadIdx.x / WAVE;
    int lane = threadIdx.x & (WAVE - 1);
    if (row >= n) return;
    T s = T(0);
    for (int j = lane; j < n; j += WAVE) s += m[(long)row * n + j] * (T)x[j];
    s = group_sum<T>(s, WAVE);
    if (lane == 0) y[row] = s;
}

template <typename S, typename D>
__global__ void k_gather(int n, const int* __restrict__ map, const S* __restrict__ src, D* __restrict__ dst) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = (D)src[map[i]];
}

template <typename S, typename D>
__global__ void k_scatter(int n, const int* __restrict__ map, const S* __restrict__ src, D* __restrict__ dst) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[map[i]] = (D)src[i];
}

template <typename T>
__global__ void k_axpby(long n, T a, const T* __restrict__ x, T b, T* __restrict__ y) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = (b == T(0)) ? a * x[i] : a * x[i] + b * y[i];
}

template <typename T>
__global__ void k_mul(long n, const T* __restrict__ d, const T* __restrict__ x, T* __restrict__ y, T w) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] = w * (d[i] * x[i]);
}

template <typename T>
__global__ void k_addmul(long n, const T* __restrict__ d, const T* __restrict__ x, T* __restrict__ y, T w) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) y[i] += w * (d[i] * x[i]);
}

template <typename S, typename D>
__global__ void k_copy(long n, const S* __restrict__ s, D* __restrict__ d) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = (D)s[i];
}

template <typename T>
__global__ void k_set(long n, T* __restrict__ d, T v) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = v;
}

__global__ void k_scale(long n, double a, double* __restrict__ x) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] *= a;
}

// x /= sqrt(*norm2) with the norm read on the device (x is left at zero when the
// norm is zero, which only happens at an Arnoldi breakdown).
__global__ void k_scale_by_norm(long n, const double* __restrict__ norm2, double* __restrict__ x) {
    double q = *norm2;
    double a = q > 0.0 ? 1.0 / sqrt(q) : 0.0;
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = x[i] * a;
}

// ---------------------------------------------------------------- Krylov reductions
template <int NB>
__device__ inline void block_reduce_write(double (&acc)[NB], double* __restrict__ out, int stride) {
    __shared__ double sh[NB][TPB / WAVE];
    int wid = threadIdx.x / WAVE, lane = threadIdx.x & (WAVE - 1);
#pragma unroll
    for (int t = 0; t < NB; ++t) {
        double v = group_sum<double>(acc[t], WAVE);
        if (lane == 0) sh[t][wid] = v;
    }
    __syncthreads();
    if ((int)threadIdx.x < NB) {
        double s = 0.0;
#pragma unroll
        for (int q = 0; q < TPB / WAVE; ++q) s += sh[threadIdx.x][q];
        out[(long)threadIdx.x * stride] = s;
    }
}

// Workgroup sums of NB per-thread accumulators: out[t * stride] = sum over the
// workgroup of acc[t], for t < nv.  Eight accumulators at a time go through
// LDS; then 32 lanes per accumulator add eight values each and finish with a
// shuffle tree (a fixed order, so every call rounds alike).
template <int NB>
__device__ inline void block_sums(const double (&acc)[NB], int nv, double* __restrict__ out, long stride) {
    constexpr int G = 8, L = TPB / G;
    __shared__ double sh[G][TPB];
    const int tid = threadIdx.x, v = tid / L, k = tid % L;
#pragma unroll
    for (int g0 = 0; g0 < NB; g0 += G) {
        if (g0 >= nv) break;
        if (g0 > 0) __syncthreads();
#pragma unroll
        for (int t = 0; t < G; ++t)
            if (g0 + t < NB) sh[t][tid] = acc[g0 + t];
        __syncthreads();
        double s = 0.0;
#pragma unroll
        for (int m = 0; m < G; ++m) s += sh[v][k + L * m];
        for (int off = L / 2; off > 0; off >>= 1) s += __shfl_xor(s, off, L);
        if (k == 0 && g0 + v < nv) out[(long)(g0 + v) * stride] = s;
    }
}

// part[(i0+t) * gridDim.x + block] = partial of <V_{i0+t}, w>
template <int NB>
__global__ __launch_bounds__(TPB) void k_mdot(long n, const double* __restrict__ V, long ldv, int nvec,
                                              const double* __restrict__ w, double* __restrict__ part) {
    int i0 = blockIdx.y * NB;
    double acc[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) acc[t] = 0.0;
    long stride = (long)gridDim.x * TPB;
    for (long r = (long)blockIdx.x * TPB + threadIdx.x; r < n; r += stride) {
        double wr = w[r];
#pragma unroll
        for (int t = 0; t < NB; ++t)
            if (i0 + t < nvec) acc[t] += V[(long)(i0 + t) * ldv + r] * wr;
    }
    block_sums<NB>(acc, min(NB, nvec - i0), part + (long)i0 * gridDim.x + blockIdx.x, gridDim.x);
}

// out[i] = sum over the nparts partials of vector i, in a fixed tree order.
// With ncopy > 0 (a single workgroup), csrc[0..ncopy) -- which may include
// out[0] -- is then also stored to cdst, a host-mapped buffer, released to the
// host, and cdst[ncopy] = 1 is stored after it as the host's ready flag.
__global__ __launch_bounds__(TPB) void k_reduce_parts(int nparts, const double* __restrict__ part,
                                                      double* __restrict__ out, const double* csrc,
                                                      double* __restrict__ cdst, int ncopy) {
    __shared__ double sh[TPB / WAVE];
    const double* p = part + (long)blockIdx.x * nparts;
    double s = 0.0;
    for (int q = threadIdx.x; q < nparts; q += TPB) s += p[q];
    s = group_sum<double>(s, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) sh[threadIdx.x / WAVE] = s;
    __syncthreads();
    if (threadIdx.x == 0) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < TPB / WAVE; ++q) t += sh[q];
        out[blockIdx.x] = t;
    }
    if (ncopy > 0) {
        __syncthreads();
        for (int q = threadIdx.x; q < ncopy; q += TPB) cdst[q] = csrc[q];
        __threadfence_system();
        __syncthreads();
        if (threadIdx.x == 0) {
            *(volatile double*)(cdst + ncopy) = 1.0;
            __threadfence_system();
        }
    }
}

// w -= sum_i h[i] V_i  (h on the device); optionally partial sums of w_new^2.
__global__ __launch_bounds__(TPB) void k_maxpy(long n, const double* __restrict__ V, long ldv, int nvec,
                                               const double* __restrict__ h, double hscale, double* __restrict__ w,
                                               double* __restrict__ normpart) {
    __shared__ double hs[64];
    if ((int)threadIdx.x < nvec) hs[threadIdx.x] = hscale * h[threadIdx.x];
    __syncthreads();
    double acc = 0.0;
    long stride = (long)gridDim.x * TPB;
    for (long r = (long)blockIdx.x * TPB + threadIdx.x; r < n; r += stride) {
        double s = 0.0;
        for (int i = 0; i < nvec; ++i) s += hs[i] * V[(long)i * ldv + r];
        double wn = w[r] - s;
        w[r] = wn;
        acc += wn * wn;
    }
    if (normpart) {
        double a[1] = {acc};
        block_reduce_write<1>(a, normpart + blockIdx.x, 0);
    }
}

// Arnoldi step with delayed reorthogonalisation, first pass: the dots of
// V_0 .. V_{nvec-1} with u = V_{nvec-1} (the newest basis vector, so far
// orthogonalised once) and with w = A z, as partials part[i * np + block] (u)
// and part[(nvec + i) * np + block] (w).
template <int NB>
__global__ __launch_bounds__(TPB) void k_mdot2(long n, const double* __restrict__ V, long ldv, int nvec,
                                               const double* __restrict__ w, double* __restrict__ part) {
    const int i0 = blockIdx.y * NB;
    const double* u = V + (long)(nvec - 1) * ldv;
    double au[NB], aw[NB];
#pragma unroll
    for (int t = 0; t < NB; ++t) au[t] = aw[t] = 0.0;
    long stride = (long)gridDim.x * TPB;
    for (long r = (long)blockIdx.x * TPB + threadIdx.x; r < n; r += stride) {
        const double ur = u[r], wr = w[r];
#pragma unroll
        for (int t = 0; t < NB; ++t)
            if (i0 + t < nvec) {
                const double x = V[(long)(i0 + t) * ldv + r];
                au[t] += x * ur;
                aw[t] += x * wr;
            }
    }
    const int nv = min(NB, nvec - i0);
    block_sums<NB>(au, nv, part + (long)i0 * gridDim.x + blockIdx.x, gridDim.x);
    __syncthreads();
    block_sums<NB>(aw, nv, part + (long)(nvec + i0) * gridDim.x + blockIdx.x, gridDim.x);
}

// Second pass.  From the first pass's s_i = V_i . u and h_i = V_i . w (i <= j =
// nvec - 1): u's coefficients a_i = s_i (i < j) and alpha = sqrt(s_j - sum a_i^2)
// give the final basis vector v_j = (u - sum_{i<j} a_i V_i) / alpha, and w's
// coefficients in the final basis are c_i = h_i (i < j), c_j = (h_j - sum_{i<j}
// a_i h_i) / alpha.  Then V_j = v_j, w -= sum_{i<j} c_i V_i + c_j v_j, with
// partial sums of ||w||^2; block 0 stores c_0..c_j at coef[0..j] and alpha at
// coef[64].  alpha = 0 (u in the span of V_0..V_{j-1}) leaves v_j = 0.
__global__ __launch_bounds__(TPB) void k_arnoldi_update(long n, double* __restrict__ V, long ldv, int nvec,
                                                        const double* __restrict__ sh, double* __restrict__ w,
                                                        double* __restrict__ normpart, double* __restrict__ coef) {
    __shared__ double as[64], cs[64];
    __shared__ double scal[2];
    const int j = nvec - 1;
    const double* sd = sh;
    const double* hd = sh + nvec;
    if ((int)threadIdx.x < j) { as[threadIdx.x] = sd[threadIdx.x]; cs[threadIdx.x] = hd[threadIdx.x]; }
    if (threadIdx.x == 0) {
        double ss = 0.0, sx = 0.0;
        for (int i = 0; i < j; ++i) {
            ss += sd[i] * sd[i];
            sx += sd[i] * hd[i];
        }
        const double a2 = sd[j] - ss;
        const double alpha = a2 > 0.0 ? sqrt(a2) : 0.0;
        const double ainv = alpha > 0.0 ? 1.0 / alpha : 0.0;
        const double cj = (hd[j] - sx) * ainv;
        scal[0] = ainv;
        scal[1] = cj;
        if (blockIdx.x == 0) { coef[64] = alpha; coef[j] = cj; }
    }
    if (blockIdx.x == 0 && (int)threadIdx.x < j) coef[threadIdx.x] = hd[threadIdx.x];
    __syncthreads();
    const double ainv = scal[0], cj = scal[1];
    double* u = V + (long)j * ldv;
    double acc = 0.0;
    long stride = (long)gridDim.x * TPB;
    for (long r = (long)blockIdx.x * TPB + threadIdx.x; r < n; r += stride) {
        double t = u[r], q = w[r];
        for (int i = 0; i < j; ++i) {
            const double x = V[(long)i * ldv + r];
            t -= as[i] * x;
            q -= cs[i] * x;
        }
        const double v = t * ainv;
        q -= cj * v;
        u[r] = v;
        w[r] = q;
        acc += q * q;
    }
    double a[1] = {acc};
    block_reduce_write<1>(a, normpart + blockIdx.x, 0);
}

// One level of a triangular solve: for the rows of this level,
// x_i = (b_i - sum_{j != i} t_ij x_j) / t_ii (unit: no division, no diagonal stored).
template <typename T>
__global__ void k_trsv_level(int cnt, const int* __restrict__ rows, const int* __restrict__ rp,
                             const int* __restrict__ ci, const T* __restrict__ v, const T* b, T* x, int unit) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    int i = rows[t];
    T s = b[i], d = T(1);
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        int j = ci[p];
        if (j == i) d = v[p];
        else s -= v[p] * x[j];
    }
    x[i] = unit ? s : s / d;
}

// Second pass of one hybrid L1 Gauss-Seidel sweep (the first is r = b - A x on
// the whole operator).  Thread c of the workgroup owns chunk c of its 64
// chunks of `chunk` consecutive rows and relaxes them one after another
// (forward: increasing, backward: decreasing), x_i += delta_i with
//   delta_i = (r_i - sum_{j in the chunk, already relaxed} a_ij delta_j) / d_i,
// which with r_i = b_i - sum_j a_ij x_j is the sweep
//   x_i <- x_i + (b_i - sum_j a_ij y_j) / d_i,  y_j new for the chunk's rows
// already relaxed and old for every other unknown.  The in-chunk entries come
// from slot tables made at setup (slot k of position t of chunk c at
// (t W + k) nchp + c: the 64 threads read adjacent addresses, and a step's
// loads are issued one step ahead, so the sequential part waits on LDS, not
// on memory); padding slots hold 0.  r is staged in LDS with coalesced loads,
// row t of thread c at t * 65 + c (conflict-free for the threads of a step),
// each r_i there is overwritten by delta_i, and x is updated with coalesced
// stores at the end.  WMAX > 0: tables of at most WMAX slots per row held in
// registers; WMAX = 0: any width, loads inside the step.  from_zero: x starts
// at 0 (r = b) and is overwritten.
constexpr int HGS_LDS_STRIDE = 65;
// Batched staging: every thread issues HGS_BATCH loads before its first LDS
// store, so a workgroup waits for memory once per batch rather than once per
// element.
constexpr int HGS_BATCH = 16;

// r[q] (q < span, the workgroup's rows) to LDS at (q % chunk) stride + q / chunk
template <typename T, int NT>
__device__ inline void hgs_stage_r(T* buf, int stride, int chunk, const T* __restrict__ r, int span) {
    for (int q0 = threadIdx.x; q0 < span; q0 += NT * HGS_BATCH) {
        T v[HGS_BATCH];
#pragma unroll
        for (int u = 0; u < HGS_BATCH; ++u) {
            const int q = q0 + u * NT;
            v[u] = q < span ? r[q] : T(0);
        }
#pragma unroll
        for (int u = 0; u < HGS_BATCH; ++u) {
            const int q = q0 + u * NT;
            if (q < span) buf[(q % chunk) * stride + q / chunk] = v[u];
        }
    }
}

// x[q] = delta (from_zero) or x[q] + delta for the workgroup's rows
template <typename T, int NT>
__device__ inline void hgs_write_x(const T* buf, int stride, int chunk, T* __restrict__ x, int span, int from_zero) {
    for (int q0 = threadIdx.x; q0 < span; q0 += NT * HGS_BATCH) {
        T v[HGS_BATCH];
#pragma unroll
        for (int u = 0; u < HGS_BATCH; ++u) {
            const int q = q0 + u * NT;
            v[u] = (q < span && !from_zero) ? x[q] : T(0);
        }
#pragma unroll
        for (int u = 0; u < HGS_BATCH; ++u) {
            const int q = q0 + u * NT;
            if (q < span) {
                const T del = buf[(q % chunk) * stride + q / chunk];
                x[q] = from_zero ? del : v[u] + del;
            }
        }
    }
}
// below this many 64-chunk workgroups a level takes the LDS-staged kernel,
// whose LDS is kept within the default 64 KB limit
constexpr int HGS_SMALL_GRID = 256;
constexpr size_t HGS_LDS_MAX = 65536;

template <typename T, int WMAX>
__global__ __launch_bounds__(64) void k_hgs_tri(int n, int chunk, int w, int nchp,
                                                const unsigned char* __restrict__ lc, const T* __restrict__ lv,
                                                const T* __restrict__ dT, const T* __restrict__ r,
                                                T* __restrict__ x, int backward, int from_zero) {
    extern __shared__ unsigned char hgs_lds[];
    T* buf = reinterpret_cast<T*>(hgs_lds);
    const int me = threadIdx.x;
    const int c = blockIdx.x * 64 + me;
    const long base = (long)blockIdx.x * 64 * chunk;
    const int span = (int)min((long)64 * chunk, (long)n - base);
    hgs_stage_r<T, 64>(buf, HGS_LDS_STRIDE, chunk, r + base, span);
    __syncthreads();
    const long c0 = (long)c * chunk;
    const int len = c0 < n ? (int)min((long)chunk, (long)n - c0) : 0;
    if (WMAX > 0) {
        constexpr int WR = WMAX > 0 ? WMAX : 1;
        int cc[WR] = {}, nc[WR] = {};
        T cv[WR] = {}, nv[WR] = {};
        T cd = T(1), nd = T(1);
        // slots past w read column 0 with value 0, so every step issues all
        // WMAX gathers before its first product (no per-slot branch)
        auto load = [&](int t, int* kc, T* kv, T& kd) {
#pragma unroll
            for (int k = 0; k < WR; ++k) {
                const size_t o = ((size_t)t * w + k) * nchp + c;
                kc[k] = k < w ? lc[o] : 0;
                kv[k] = k < w ? lv[o] : T(0);
            }
            kd = dT[(size_t)t * nchp + c];
        };
        if (len > 0) load(backward ? len - 1 : 0, cc, cv, cd);
        for (int s = 0; s < len; ++s) {
            const int t = backward ? len - 1 - s : s;
            if (s + 1 < len) load(backward ? t - 1 : t + 1, nc, nv, nd);
            T g[WR];
#pragma unroll
            for (int k = 0; k < WR; ++k) g[k] = buf[cc[k] * HGS_LDS_STRIDE + me];
            T acc = buf[t * HGS_LDS_STRIDE + me];
#pragma unroll
            for (int k = 0; k < WR; ++k) acc -= cv[k] * g[k];
            buf[t * HGS_LDS_STRIDE + me] = acc * cd;
#pragma unroll
            for (int k = 0; k < WR; ++k) {
                cc[k] = nc[k];
                cv[k] = nv[k];
            }
            cd = nd;
        }
    } else {
        for (int s = 0; s < len; ++s) {
            const int t = backward ? len - 1 - s : s;
            T acc = buf[t * HGS_LDS_STRIDE + me];
            for (int k = 0; k < w; ++k) {
                const size_t o = ((size_t)t * w + k) * nchp + c;
                acc -= lv[o] * buf[lc[o] * HGS_LDS_STRIDE + me];
            }
            buf[t * HGS_LDS_STRIDE + me] = acc * dT[(size_t)t * nchp + c];
        }
    }
    __syncthreads();
    hgs_write_x<T, 64>(buf, HGS_LDS_STRIDE, chunk, x + base, span, from_zero);
}

// Adjoint gradient on the block pattern: dv[p,r,c] = -sum_k lam_k[I b + r] x_k[J b + c].
__global__ void k_grad(long nnzb, int b, int nbr, const int* __restrict__ rp, const int* __restrict__ ci, long n,
                       int nrhs, const double* __restrict__ lam, const double* __restrict__ x,
                       double* __restrict__ dv) {
    long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p >= nnzb) return;
    int lo = 0, hi = nbr;  // find I with rp[I] <= p < rp[I+1]
    while (hi - lo > 1) {
        int mid = (lo + hi) >> 1;
        if (rp[mid] <= p) lo = mid;
        else hi = mid;
    }
    int I = lo, J = ci[p];
    for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) {
            double s = 0.0;
            for (int k = 0; k < nrhs; ++k) s += lam[k * n + (long)I * b + r] * x[k * n + (long)J * b + c];
            dv[p * b * b + r * b + c] = -s;
        }
}

inline int nblk(long n, int t = TPB) { return (int)((n + t - 1) / t); }

int pick_group(double avg) {
    if (avg <= 1.5) return 1;
    if (avg <= 3.0) return 2;
    if (avg <= 6.0) return 4;
    if (avg <= 14.0) return 8;
    if (avg <= 28.0) return 16;
    if (avg <= 56.0) return 32;
    return 64;
}

}  // namespace

#define MGR_DISPATCH_G(G, ...)                          \
    switch (G) {                                        \
        case 1: { constexpr int GG = 1; __VA_ARGS__; } break;   \
        case 2: { constexpr int GG = 2; __VA_ARGS__; } break;   \
        case 4: { constexpr int GG = 4; __VA_ARGS__; } break;   \
        case 8: { constexpr int GG = 8; __VA_ARGS__; } break;   \
        case 16: { constexpr int GG = 16; __VA_ARGS__; } break; \
        case 32: { constexpr int GG = 32; __VA_ARGS__; } break; \
        default: { constexpr int GG = 64; __VA_ARGS__; } break; \
    }

static_assert(ELL_SLICE == TPB, "an ELL slice is one workgroup's rows");

// One thread per row over the operator's sliced ELL copy: the workgroup's
// slice holds its rows slot-major (slot k of row r at base + k TPB + r % TPB,
// base = slice * w * TPB) up to the slice's width; every slot's column and
// value come in with coalesced loads, all of them before the first gather, and
// the products are summed in row order (padding slots hold zero values and the
// row's own column, or column 0 beyond the last column).
// WMAX bounds the slots a thread holds in registers.
template <typename MT, int TAG, int WMAX, class Op>
__global__ __launch_bounds__(TPB) void k_spmv_ell(int nr, int w, const int* __restrict__ esw,
                                                  const int* __restrict__ eci, const MT* __restrict__ ev, Op op) {
    const int r = blockIdx.x * TPB + threadIdx.x;
    const int sw = min(esw[blockIdx.x], w);
    if (r >= nr) return;
    const long base = (long)blockIdx.x * w * TPB + threadIdx.x;
    const typename Op::Pre pre = op.pre(r);
    int c[WMAX];
    MT a[WMAX];
#pragma unroll
    for (int k = 0; k < WMAX; ++k)
        if (k < sw) {
            c[k] = eci[base + (long)k * TPB];
            a[k] = ev[base + (long)k * TPB];
        }
    MT s = MT(0);
#pragma unroll
    for (int k = 0; k < WMAX; ++k)
        if (k < sw) s += a[k] * op.xval(c[k]);
    op.fin(r, s, pre);
}

// esw[slice] = the longest row of the slice's TPB rows
__global__ __launch_bounds__(TPB) void k_ell_widths(int nr, const int* __restrict__ rp, int* __restrict__ esw) {
    __shared__ int red[TPB / WAVE];
    const int r = blockIdx.x * TPB + threadIdx.x;
    int len = r < nr ? rp[r + 1] - rp[r] : 0;
    for (int off = WAVE / 2; off > 0; off >>= 1) len = max(len, __shfl_xor(len, off, WAVE));
    if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = len;
    __syncthreads();
    if (threadIdx.x == 0) {
        int m = 0;
        for (int q = 0; q < TPB / WAVE; ++q) m = max(m, red[q]);
        esw[blockIdx.x] = m;
    }
}

// One workgroup per slice: the slice's entries (one contiguous range of the
// CSR arrays) come into LDS with coalesced loads, a window of ELL_STAGE_W * TPB
// entries at a time, and each thread writes the slots of its row that the
// window holds (coalesced across the slice's rows); the padding slots last.
constexpr int ELL_STAGE_W = 16;
template <typename MT>
__global__ __launch_bounds__(TPB) void k_to_ell(int nr, int nc, int w, const int* __restrict__ esw,
                                                const int* __restrict__ rp, const int* __restrict__ ci,
                                                const MT* __restrict__ v, int* __restrict__ eci,
                                                MT* __restrict__ ev) {
    constexpr int STAGE = ELL_STAGE_W * TPB;
    __shared__ int srp[TPB + 1];
    __shared__ int sci[STAGE];
    __shared__ MT sv[STAGE];
    const int r0 = blockIdx.x * TPB;
    const int rows = min(TPB, nr - r0);
    const int sw = min(esw[blockIdx.x], w);
    for (int t = threadIdx.x; t <= rows; t += TPB) srp[t] = rp[r0 + t];
    __syncthreads();
    const int p0 = srp[0], cnt = srp[rows] - p0;
    const bool active = (int)threadIdx.x < rows;
    const int r = r0 + threadIdx.x;
    const int b = active ? srp[threadIdx.x] - p0 : 0;
    const int len = active ? min(srp[threadIdx.x + 1] - srp[threadIdx.x], sw) : 0;
    const long base = (long)blockIdx.x * w * TPB + threadIdx.x;
    for (int w0 = 0; w0 < cnt; w0 += STAGE) {
        const int wn = min(STAGE, cnt - w0);
        __syncthreads();
        for (int q = threadIdx.x; q < wn; q += TPB) {
            if (eci) sci[q] = ci[p0 + w0 + q];
            sv[q] = v[p0 + w0 + q];
        }
        __syncthreads();
        const int k0 = max(0, w0 - b), k1 = min(len, w0 + wn - b);
        for (int k = k0; k < k1; ++k) {
            if (eci) eci[base + (long)k * TPB] = sci[b + k - w0];
            ev[base + (long)k * TPB] = sv[b + k - w0];
        }
    }
    if (!active) return;
    const int pad = r < nc ? r : 0;
    for (int k = len; k < sw; ++k) {
        if (eci) eci[base + (long)k * TPB] = pad;
        ev[base + (long)k * TPB] = MT(0);
    }
}

__global__ __launch_bounds__(TPB) void k_sum_widths(const int* __restrict__ esw, int nsl, long long* __restrict__ out) {
    __shared__ long long red[TPB / WAVE];
    long long t = 0;
    for (int q = threadIdx.x; q < nsl; q += TPB) t += esw[q];
    for (int off = WAVE / 2; off > 0; off >>= 1) t += __shfl_xor(t, off, WAVE);
    if ((threadIdx.x & (WAVE - 1)) == 0) red[threadIdx.x / WAVE] = t;
    __syncthreads();
    if (threadIdx.x == 0) {
        long long m = 0;
        for (int q = 0; q < TPB / WAVE; ++q) m += red[q];
        *out = m;
    }
}

long ell_total_width(const int* esw, int nsl, hipStream_t s) {
    if (nsl <= 0) return 0;
    DArr<long long> d(1, s);
    k_sum_widths<<<1, TPB, 0, s>>>(esw, nsl, d.p);
    MGR_LAUNCH_CHECK();
    long long h = 0;
    MGR_HIP(hipMemcpyAsync(&h, d.p, sizeof(long long), hipMemcpyDeviceToHost, s));
    MGR_HIP(hipStreamSynchronize(s));
    return (long)h;
}

void ell_widths(int nr, const int* rp, int* esw, hipStream_t s) {
    if (nr <= 0) return;
    k_ell_widths<<<nblk(nr), TPB, 0, s>>>(nr, rp, esw);
    MGR_LAUNCH_CHECK();
}

void to_ell(int nr, int nc, int w, const int* esw, const int* rp, const int* ci, const double* v, int* eci,
            double* ev, hipStream_t s) {
    if (nr <= 0) return;
    k_to_ell<double><<<nblk(nr), TPB, 0, s>>>(nr, nc, w, esw, rp, ci, v, eci, ev);
    MGR_LAUNCH_CHECK();
}

void to_ell(int nr, int nc, int w, const int* esw, const int* rp, const int* ci, const float* v, int* eci,
            float* ev, hipStream_t s) {
    if (nr <= 0) return;
    k_to_ell<float><<<nblk(nr), TPB, 0, s>>>(nr, nc, w, esw, rp, ci, v, eci, ev);
    MGR_LAUNCH_CHECK();
}

// the sliced ELL kernel where the operator has that copy, else the CSR stream
template <typename MT, int TAG, class Op>
static void launch_rows(const SpOp<MT>& A, const Op& op, hipStream_t s) {
    if (A.ew > 0 && A.eci && A.ev && A.esw)
        k_spmv_ell<MT, TAG, ELL_MAX_W, Op><<<nblk(A.nr), TPB, 0, s>>>(A.nr, A.ew, A.esw, A.eci, A.ev, op);
    else
        k_spmv_stream<MT, TAG><<<A.nblk, TPB, 0, s>>>(A.blk, A.bpos, A.rp, A.ci, A.v, op);
}

int rowblock_count(int nr, long nnz) {
    long cost = nnz + (long)nr / SPMV_ROW_COST;
    return cost > 0 ? (int)((cost + SPMV_CHUNK - 1) / SPMV_CHUNK) : 1;
}

void rowblocks(int nr, long nnz, const int* rp, int* blk, int* bpos, hipStream_t s) {
    int nb = rowblock_count(nr, nnz);
    k_rowblocks<<<nblk(nb + 1), TPB, 0, s>>>(nr, nb, rp, blk, bpos);
    MGR_LAUNCH_CHECK();
}

template <typename MT, typename XT, typename X2T, typename YT, typename WT>
void spmv(const SpOp<MT>& A, const XT* x, const X2T* x2, int split, const WT* w, YT* y, MT alpha, MT beta,
          hipStream_t s, int tag) {
    if (A.nr <= 0) return;
    if (!A.blk) throw Error(-1, "spmv: operator without row blocks");
    SpmvOp<MT, XT, X2T, YT, WT> op{x, x2, split, w, y, alpha, beta};
    if (tag == 1)
        launch_rows<MT, 1>(A, op, s);
    else
        launch_rows<MT, 0>(A, op, s);
    MGR_LAUNCH_CHECK();
}

template <typename T>
void jacobi_sweep(const SpOp<T>& A, const T* dinv, const T* b, const T* x, T* y, hipStream_t s) {
    if (A.nr <= 0) return;
    JacobiOp<T> op{dinv, b, x, y};
    launch_rows<T, 0>(A, op, s);
    MGR_LAUNCH_CHECK();
}

template <typename T>
void presmooth(const SpOp<T>& A, const T* dinv, const T* b, T* x, T* r, hipStream_t s) {
    if (A.nr <= 0) return;
    PreOp<T> op{dinv, b, x, r};
    launch_rows<T, 0>(A, op, s);
    MGR_LAUNCH_CHECK();
}

template <typename T>
void presmooth_scaled(const SpOp<T>& A, const T* bd, const T* b, T* x, T* r, hipStream_t s) {
    if (A.nr <= 0) return;
    if (!A.blk) throw Error(-1, "presmooth: operator without row blocks");
    PreOpD<T> op{bd, b, x, r};
    launch_rows<T, 0>(A, op, s);
    MGR_LAUNCH_CHECK();
}

template <typename T, typename XT>
void restrict_scaled(const SpOp<T>& A, const XT* x, const T* dsc, T* y, T* yd, hipStream_t s) {
    if (A.nr <= 0) return;
    if (!A.blk) throw Error(-1, "restrict: operator without row blocks");
    RestrictOp<T, XT> op{x, dsc, y, yd};
    launch_rows<T, 0>(A, op, s);
    MGR_LAUNCH_CHECK();
}

void bsr_spmv(int bsize, int nbr, const int* rp, const int* ci, const double* v, long nnzb, const double* x,
              const double* w, double* y, double alpha, double beta, hipStream_t s) {
    if (nbr <= 0) return;
    int G = pick_group((double)nnzb / nbr);
    long threads = (long)nbr * G;
    switch (bsize) {
        case 2: MGR_DISPATCH_G(G, (k_bsr_spmv<2, GG><<<nblk(threads), TPB, 0, s>>>(nbr, rp, ci, v, x, w, y, alpha, beta))); break;
        case 3: MGR_DISPATCH_G(G, (k_bsr_spmv<3, GG><<<nblk(threads), TPB, 0, s>>>(nbr, rp, ci, v, x, w, y, alpha, beta))); break;
        case 4: MGR_DISPATCH_G(G, (k_bsr_spmv<4, GG><<<nblk(threads), TPB, 0, s>>>(nbr, rp, ci, v, x, w, y, alpha, beta))); break;
        default: throw Error(-6, "block size not supported by the block SpMV");
    }
    MGR_LAUNCH_CHECK();
}

template <typename T, typename XT>
void dense_gemv(int n, const T* m, const XT* x, T* y, hipStream_t s) {
    if (n <= 0) return;
    k_dense_gemv<T, XT><<<ceil_div(n, TPB / WAVE), TPB, 0, s>>>(n, m, x, y);
    MGR_LAUNCH_CHECK();
}

template <typename S, typename D>
void gather(int n, const int* map, const S* src, D* dst, hipStream_t s) {
    if (n <= 0) return;
    k_gather<S, D><<<nblk(n), TPB, 0, s>>>(n, map, src, dst);
    MGR_LAUNCH_CHECK();
}

template <typename S, typename D>
void scatter(int n, const int* map, const S* src, D* dst, hipStream_t s) {
    if (n <= 0) return;
    k_scatter<S, D><<<nblk(n), TPB, 0, s>>>(n, map, src, dst);
    MGR_LAUNCH_CHECK();
}

template <typename T>
void axpby(long n, T a, const T* x, T b, T* y, hipStream_t s) {
    if (n <= 0) return;
    k_axpby<T><<<nblk(n), TPB, 0, s>>>(n, a, x, b, y);
    MGR_LAUNCH_CHECK();
}

template <typename T>
void mul(long n, const T* d, const T* x, T* y, T w, hipStream_t s) {
    if (n <= 0) return;
    k_mul<T><<<nblk(n), TPB, 0, s>>>(n, d, x, y, w);
    MGR_LAUNCH_CHECK();
}

template <typename T>
void addmul(long n, const T* d, const T* x, T* y, T w, hipStream_t s) {
    if (n <= 0) return;
    k_addmul<T><<<nblk(n), TPB, 0, s>>>(n, d, x, y, w);
    MGR_LAUNCH_CHECK();
}

template <typename S, typename D>
void copy(long n, const S* src, D* dst, hipStream_t s) {
    if (n <= 0) return;
    k_copy<S, D><<<nblk(n), TPB, 0, s>>>(n, src, dst);
    MGR_LAUNCH_CHECK();
}

template <typename T>
void set(long n, T* dst, T v, hipStream_t s) {
    if (n <= 0) return;
    k_set<T><<<nblk(n), TPB, 0, s>>>(n, dst, v);
    MGR_LAUNCH_CHECK();
}

void scale(long n, double a, double* x, hipStream_t s) {
    if (n <= 0) return;
    k_scale<<<nblk(n), TPB, 0, s>>>(n, a, x);
    MGR_LAUNCH_CHECK();
}

void scale_by_norm(long n, const double* norm2, double* x, hipStream_t s) {
    if (n <= 0) return;
    k_scale_by_norm<<<nblk(n), TPB, 0, s>>>(n, norm2, x);
    MGR_LAUNCH_CHECK();
}

int krylov_parts(long n) {
    long b = (n + TPB - 1) / TPB;
    return (int)(b < KRYLOV_PARTS ? (b > 0 ? b : 1) : KRYLOV_PARTS);
}

void mdot(long n, const double* V, long ldv, int nvec, const double* w, double* part, double* out, hipStream_t s) {
    if (nvec <= 0) return;
    int np = krylov_parts(n);
    constexpr int NB = 8;
    dim3 grid(np, ceil_div(nvec, NB));
    k_mdot<NB><<<grid, TPB, 0, s>>>(n, V, ldv, nvec, w, part);
    k_reduce_parts<<<nvec, TPB, 0, s>>>(np, part, out, nullptr, nullptr, 0);
    MGR_LAUNCH_CHECK();
}

void maxpy(long n, const double* V, long ldv, int nvec, const double* h, double hscale, double* w, double* part,
           double* norm2_out, hipStream_t s) {
    if (nvec > 64) throw Error(-1, "maxpy: at most 64 vectors");
    int np = krylov_parts(n);
    if (nvec <= 0 && !norm2_out) return;
    k_maxpy<<<np, TPB, 0, s>>>(n, V, ldv, nvec, h, hscale, w, norm2_out ? part : nullptr);
    if (norm2_out) k_reduce_parts<<<1, TPB, 0, s>>>(np, part, norm2_out, nullptr, nullptr, 0);
    MGR_LAUNCH_CHECK();
}

void arnoldi_dots(long n, const double* V, long ldv, int nvec, const double* w, double* part, double* out,
                  hipStream_t s) {
    if (nvec <= 0 || nvec > 64) throw Error(-1, "arnoldi_dots: 1 to 64 vectors");
    int np = krylov_parts(n);
    constexpr int NB = 8;
    dim3 grid(np, ceil_div(nvec, NB));
    k_mdot2<NB><<<grid, TPB, 0, s>>>(n, V, ldv, nvec, w, part);
    k_reduce_parts<<<2 * nvec, TPB, 0, s>>>(np, part, out, nullptr, nullptr, 0);
    MGR_LAUNCH_CHECK();
}

void arnoldi_update(long n, double* V, long ldv, int nvec, const double* sh, double* w, double* part,
                    double* norm2_out, double* coef, const double* csrc, double* cdst, int ncopy, hipStream_t s) {
    if (nvec <= 0 || nvec > 64) throw Error(-1, "arnoldi_update: 1 to 64 vectors");
    int np = krylov_parts(n);
    k_arnoldi_update<<<np, TPB, 0, s>>>(n, V, ldv, nvec, sh, w, part, coef);
    k_reduce_parts<<<1, TPB, 0, s>>>(np, part, norm2_out, csrc, cdst, ncopy);
    MGR_LAUNCH_CHECK();
}

// The same pass for levels too small to hide memory latency behind other
// waves (fewer workgroups than compute units).  Each workgroup first stages
// the slot tables and diagonals of its chunks in LDS with batched coalesced
// loads, so the sequential steps wait only on LDS; then a single wave, one
// lane per chunk, runs the steps, and there the instruction count per step is
// what bounds the time (each wave instruction costs the same however few lanes
// are active).  The fast variant (chunks of at most HGS_FAST_CHUNK rows, at
// most WMAX slots per row) therefore fixes the table width and the number of
// chunks TG at compile time, so that slot reads take immediate offsets, reads
// a step's slots one step ahead into alternating register sets, issues every
// gather of a step before its first product and multiplies by the stored 1/d.
// LDS: r / delta of position t of chunk c at t (TG + 1) + c, slot k of
// position t at (t WMAX + k) TG + c (slots past the table's width hold column
// 0 and value 0), 1/d at t TG + c.  The general variant takes any chunk and
// width with loops over runtime bounds.
constexpr int HGS_LDS_NT = 256;
constexpr int HGS_FAST_CHUNK = 32;

template <typename T, int WMAX>
constexpr size_t hgs_fast_lds(int tg) {
    return (size_t)HGS_FAST_CHUNK * (tg + 1) * sizeof(T) + (size_t)HGS_FAST_CHUNK * WMAX * tg * (sizeof(T) + 1) +
           (size_t)HGS_FAST_CHUNK * tg * sizeof(T);
}

// chunks per workgroup of the fast variant: the most that fit HGS_LDS_MAX
template <typename T, int WMAX>
constexpr int hgs_fast_tg() {
    int tg = 64;
    while (tg > 1 && hgs_fast_lds<T, WMAX>(tg) > HGS_LDS_MAX) tg /= 2;
    return tg;
}

template <typename T, int WMAX>
__global__ __launch_bounds__(HGS_LDS_NT) void k_hgs_tri_fast(int n, int chunk, int w, int nchp,
                                                             const unsigned char* __restrict__ lc,
                                                             const T* __restrict__ lv, const T* __restrict__ dT,
                                                             const T* __restrict__ r, T* __restrict__ x,
                                                             int backward, int from_zero) {
    constexpr int NT = HGS_LDS_NT, TG = hgs_fast_tg<T, WMAX>(), ST = TG + 1, C = HGS_FAST_CHUNK;
    static_assert(hgs_fast_lds<T, WMAX>(TG) <= HGS_LDS_MAX, "fast Gauss-Seidel tables exceed the LDS budget");
    __shared__ T buf[C * ST];
    __shared__ T tv[C * WMAX * TG];
    __shared__ T td[C * TG];
    __shared__ unsigned char tc[C * WMAX * TG];
    const int me = threadIdx.x;
    const int cb = blockIdx.x * TG;
    const long base = (long)cb * chunk;
    const int span = (int)min((long)TG * chunk, (long)n - base);
    hgs_stage_r<T, NT>(buf, ST, chunk, r + base, span);
    const int ts = chunk * WMAX * TG;
    for (int q0 = me; q0 < ts; q0 += NT * HGS_BATCH) {
        T v[HGS_BATCH];
        unsigned char cc[HGS_BATCH];
#pragma unroll
        for (int u = 0; u < HGS_BATCH; ++u) {
            const int q = q0 + u * NT;
            const int t = q / (WMAX * TG), k = (q / TG) % WMAX, c = q % TG;
            const bool in = q < ts && k < w;
            const size_t o = ((size_t)t * w + k) * nchp + cb + c;
            v[u] = in ? lv[o] : T(0);
            cc[u] = in ? lc[o] : 0;
        }
#pragma unroll
        for (int u = 0; u < HGS_BATCH; ++u) {
            const int q = q0 + u * NT;
            if (q < ts) {
                tv[q] = v[u];
                tc[q] = cc[u];
            }
        }
    }
    for (int q0 = me; q0 < chunk * TG; q0 += NT * HGS_BATCH) {
        T v[HGS_BATCH];
#pragma unroll
        for (int u = 0; u < HGS_BATCH; ++u) {
            const int q = q0 + u * NT;
            v[u] = q < chunk * TG ? dT[(size_t)(q / TG) * nchp + cb + q % TG] : T(1);
        }
#pragma unroll
        for (int u = 0; u < HGS_BATCH; ++u) {
            const int q = q0 + u * NT;
            if (q < chunk * TG) td[q] = v[u];
        }
    }
    __syncthreads();
    if (me < TG) {
        const long c0 = (long)(cb + me) * chunk;
        const int len = c0 < n ? (int)min((long)chunk, (long)n - c0) : 0;
        int ca[WMAX], cbk[WMAX];
        T va[WMAX], vb[WMAX];
        T da = T(1), db = T(1);
        auto load = [&](int t, int* kc, T* kv, T& kd) {
            const int q0 = t * WMAX * TG + me;
#pragma unroll
            for (int k = 0; k < WMAX; ++k) {
                kc[k] = tc[q0 + k * TG];
                kv[k] = tv[q0 + k * TG];
            }
            kd = td[t * TG + me];
        };
        auto step = [&](int t, const int* kc, const T* kv, T kd) {
            T g[WMAX];
#pragma unroll
            for (int k = 0; k < WMAX; ++k) g[k] = buf[kc[k] * ST + me];
            T acc = buf[t * ST + me];
#pragma unroll
            for (int k = 0; k < WMAX; ++k) acc -= kv[k] * g[k];
            buf[t * ST + me] = acc * kd;
        };
        const int dir = backward ? -1 : 1, t0 = backward ? len - 1 : 0;
        if (len > 0) load(t0, ca, va, da);
        for (int s = 0; s < len; s += 2) {
            const int t = t0 + dir * s;
            if (s + 1 < len) load(t + dir, cbk, vb, db);
            step(t, ca, va, da);
            if (s + 1 >= len) break;
            if (s + 2 < len) load(t + 2 * dir, ca, va, da);
            step(t + dir, cbk, vb, db);
        }
    }
    __syncthreads();
    hgs_write_x<T, NT>(buf, ST, chunk, x + base, span, from_zero);
}

// General variant: tg chunks per workgroup (runtime), any chunk and width;
// LDS as above with the table's own width w.
template <typename T>
__global__ __launch_bounds__(HGS_LDS_NT) void k_hgs_tri_lds(int n, int chunk, int w, int nchp, int tg,
                                                            const unsigned char* __restrict__ lc,
                                                            const T* __restrict__ lv, const T* __restrict__ dT,
                                                            const T* __restrict__ r, T* __restrict__ x,
                                                            int backward, int from_zero) {
    extern __shared__ unsigned char hgs_lds[];
    constexpr int NT = HGS_LDS_NT;
    const int me = threadIdx.x, st = tg + 1;
    T* buf = reinterpret_cast<T*>(hgs_lds);
    T* tv = buf + (size_t)chunk * st;
    T* td = tv + (size_t)chunk * w * tg;
    unsigned char* tc = reinterpret_cast<unsigned char*>(td + (size_t)chunk * tg);
    const int cb = blockIdx.x * tg;
    const long base = (long)cb * chunk;
    const int span = (int)min((long)tg * chunk, (long)n - base);
    hgs_stage_r<T, NT>(buf, st, chunk, r + base, span);
    // slot q of the workgroup's table = global slot (q / tg) nchp + cb + q % tg
    const int ts = chunk * w * tg;
    for (int q0 = me; q0 < ts; q0 += NT * HGS_BATCH) {
        T v[HGS_BATCH];
        unsigned char cc[HGS_BATCH];
#pragma unroll
        for (int u = 0; u < HGS_BATCH; ++u) {
            const int q = q0 + u * NT;
            const size_t o = (size_t)(q / tg) * nchp + cb + q % tg;
            v[u] = q < ts ? lv[o] : T(0);
            cc[u] = q < ts ? lc[o] : 0;
        }
#pragma unroll
        for (int u = 0; u < HGS_BATCH; ++u) {
            const int q = q0 + u * NT;
            if (q < ts) {
                tv[q] = v[u];
                tc[q] = cc[u];
            }
        }
    }
    for (int q0 = me; q0 < chunk * tg; q0 += NT * HGS_BATCH) {
        T v[HGS_BATCH];
#pragma unroll
        for (int u = 0; u < HGS_BATCH; ++u) {
            const int q = q0 + u * NT;
            v[u] = q < chunk * tg ? dT[(size_t)(q / tg) * nchp + cb + q % tg] : T(1);
        }
#pragma unroll
        for (int u = 0; u < HGS_BATCH; ++u) {
            const int q = q0 + u * NT;
            if (q < chunk * tg) td[q] = v[u];
        }
    }
    __syncthreads();
    if (me < tg) {
        const long c0 = (long)(cb + me) * chunk;
        const int len = c0 < n ? (int)min((long)chunk, (long)n - c0) : 0;
        for (int s = 0; s < len; ++s) {
            const int t = backward ? len - 1 - s : s;
            T acc = buf[t * st + me];
            for (int k = 0; k < w; ++k) {
                const int q = (t * w + k) * tg + me;
                acc -= tv[q] * buf[tc[q] * st + me];
            }
            buf[t * st + me] = acc * td[t * tg + me];
        }
    }
    __syncthreads();
    hgs_write_x<T, NT>(buf, st, chunk, x + base, span, from_zero);
}

// LDS bytes of k_hgs_tri_lds for tg threads
template <typename T>
size_t hgs_lds_bytes(int chunk, int w, int tg) {
    return (size_t)chunk * (tg + 1) * sizeof(T) + (size_t)chunk * w * tg * (sizeof(T) + 1) +
           (size_t)chunk * tg * sizeof(T);
}

template <typename T, int WMAX>
void hgs_fast_launch(int n, int chunk, int w, int nchp, const unsigned char* lc, const T* lv, const T* dT, const T* r,
                     T* x, int bw, int fz, hipStream_t s) {
    constexpr int TG = hgs_fast_tg<T, WMAX>();
    const long nch = ((long)n + chunk - 1) / chunk;
    k_hgs_tri_fast<T, WMAX><<<(unsigned)((nch + TG - 1) / TG), HGS_LDS_NT, 0, s>>>(n, chunk, w, nchp, lc, lv, dT, r, x,
                                                                                  bw, fz);
}

template <typename T>
void hgs_tri(int n, int chunk, int w, int nchp, const unsigned char* lc, const T* lv, const T* dT, const T* r, T* x,
             bool backward, bool from_zero, hipStream_t s) {
    if (n <= 0) return;
    if (chunk < 1 || chunk > HGS_CHUNK_MAX || w < 0 || (long)nchp * chunk < n || nchp % 64)
        throw Error(-1, "hgs_tri: chunk, width or table size out of range");
    const int grid = nchp / 64;
    const size_t lds = (size_t)chunk * HGS_LDS_STRIDE * sizeof(T);
    const int bw = backward ? 1 : 0, fz = from_zero ? 1 : 0;
    if (grid < HGS_SMALL_GRID && chunk <= HGS_FAST_CHUNK && w <= 32) {
        if (w <= 4) hgs_fast_launch<T, 4>(n, chunk, w, nchp, lc, lv, dT, r, x, bw, fz, s);
        else if (w <= 8) hgs_fast_launch<T, 8>(n, chunk, w, nchp, lc, lv, dT, r, x, bw, fz, s);
        else if (w <= 16) hgs_fast_launch<T, 16>(n, chunk, w, nchp, lc, lv, dT, r, x, bw, fz, s);
        else hgs_fast_launch<T, 32>(n, chunk, w, nchp, lc, lv, dT, r, x, bw, fz, s);
        MGR_LAUNCH_CHECK();
        return;
    }
    if (grid < HGS_SMALL_GRID) {
        // small level with wide rows or long chunks: the general LDS variant
        // with the widest workgroup that fits
        const long nch = ((long)n + chunk - 1) / chunk;
        int tg = 64;
        while (tg > 1 && hgs_lds_bytes<T>(chunk, w, tg) > HGS_LDS_MAX) tg >>= 1;
        if (hgs_lds_bytes<T>(chunk, w, tg) <= HGS_LDS_MAX) {
            k_hgs_tri_lds<T><<<(unsigned)((nch + tg - 1) / tg), HGS_LDS_NT, hgs_lds_bytes<T>(chunk, w, tg), s>>>(
                n, chunk, w, nchp, tg, lc, lv, dT, r, x, bw, fz);
            MGR_LAUNCH_CHECK();
            return;
        }
    }
    if (w <= 4)
        k_hgs_tri<T, 4><<<grid, 64, lds, s>>>(n, chunk, w, nchp, lc, lv, dT, r, x, bw, fz);
    else if (w <= 8)
        k_hgs_tri<T, 8><<<grid, 64, lds, s>>>(n, chunk, w, nchp, lc, lv, dT, r, x, bw, fz);
    else if (w <= 16)
        k_hgs_tri<T, 16><<<grid, 64, lds, s>>>(n, chunk, w, nchp, lc, lv, dT, r, x, bw, fz);
    else
        k_hgs_tri<T, 0><<<grid, 64, lds, s>>>(n, chunk, w, nchp, lc, lv, dT, r, x, bw, fz);
    MGR_LAUNCH_CHECK();
}
template void hgs_tri<double>(int, int, int, int, const unsigned char*, const double*, const double*,
                              const double*, double*, bool, bool, hipStream_t);
template void hgs_tri<float>(int, int, int, int, const unsigned char*, const float*, const float*, const float*,
                             float*, bool, bool, hipStream_t);

template <typename T>
void trsv_level(int cnt, const int* rows, const SpOp<T>& A, const T* b, T* x, bool unit, hipStream_t s) {
    if (cnt <= 0) return;
    k_trsv_level<T><<<nblk(cnt), TPB, 0, s>>>(cnt, rows, A.rp, A.ci, A.v, b, x, unit ? 1 : 0);
    MGR_LAUNCH_CHECK();
}
template void trsv_level<double>(int, const int*, const SpOp<double>&, const double*, double*, bool, hipStream_t);
template void trsv_level<float>(int, const int*, const SpOp<float>&, const float*, float*, bool, hipStream_t);

void grad_values(int b, int nbr, const int* rp, const int* ci, long nnzb, int nrhs, const double* lam,
                 const double* x, double* dv, hipStream_t s) {
    if (nnzb <= 0) return;
    k_grad<<<nblk(nnzb), TPB, 0, s>>>(nnzb, b, nbr, rp, ci, (long)nbr * b, nrhs, lam, x, dv);
    MGR_LAUNCH_CHECK();
}

// ---------------------------------------------------------------- explicit instantiations
#define INST_SPMV(MT, XT, X2T, YT, WT) \
    template void spmv<MT, XT, X2T, YT, WT>(const SpOp<MT>&, const XT*, const X2T*, int, const WT*, YT*, MT, MT, hipStream_t, int);
INST_SPMV(double, double, double, double, double)
INST_SPMV(float, float, float, float, float)
INST_SPMV(float, double, double, float, float)
INST_SPMV(float, double, double, float, double)
INST_SPMV(float, float, double, double, double)
INST_SPMV(float, float, double, double, float)
INST_SPMV(float, float, float, double, double)
INST_SPMV(double, double, double, float, float)

template void jacobi_sweep<double>(const SpOp<double>&, const double*, const double*, const double*, double*, hipStream_t);
template void jacobi_sweep<float>(const SpOp<float>&, const float*, const float*, const float*, float*, hipStream_t);
template void presmooth<double>(const SpOp<double>&, const double*, const double*, double*, double*, hipStream_t);
template void presmooth<float>(const SpOp<float>&, const float*, const float*, float*, float*, hipStream_t);
template void presmooth_scaled<double>(const SpOp<double>&, const double*, const double*, double*, double*,
                                       hipStream_t);
template void presmooth_scaled<float>(const SpOp<float>&, const float*, const float*, float*, float*, hipStream_t);
template void restrict_scaled<double, double>(const SpOp<double>&, const double*, const double*, double*, double*,
                                              hipStream_t);
template void restrict_scaled<float, float>(const SpOp<float>&, const float*, const float*, float*, float*,
                                            hipStream_t);
template void restrict_scaled<float, double>(const SpOp<float>&, const double*, const float*, float*, float*,
                                             hipStream_t);
template void dense_gemv<double, double>(int, const double*, const double*, double*, hipStream_t);
template void dense_gemv<float, float>(int, const float*, const float*, float*, hipStream_t);
template void dense_gemv<float, double>(int, const float*, const double*, float*, hipStream_t);
template void gather<double, double>(int, const int*, const double*, double*, hipStream_t);
template void gather<double, float>(int, const int*, const double*, float*, hipStream_t);
template void gather<float, float>(int, const int*, const float*, float*, hipStream_t);
template void scatter<double, double>(int, const int*, const double*, double*, hipStream_t);
template void scatter<float, double>(int, const int*, const float*, double*, hipStream_t);
template void scatter<float, float>(int, const int*, const float*, float*, hipStream_t);
template void axpby<double>(long, double, const double*, double, double*, hipStream_t);
template void axpby<float>(long, float, const float*, float, float*, hipStream_t);
template void mul<double>(long, const double*, const double*, double*, double, hipStream_t);
template void mul<float>(long, const float*, const float*, float*, float, hipStream_t);
template void addmul<double>(long, const double*, const double*, double*, double, hipStream_t);
template void addmul<float>(long, const float*, const float*, float*, float, hipStream_t);
template void copy<double, double>(long, const double*, double*, hipStream_t);
template void copy<double, float>(long, const double*, float*, hipStream_t);
template void copy<float, double>(long, const float*, double*, hipStream_t);
template void copy<float, float>(long, const float*, float*, hipStream_t);
template void set<double>(long, double*, double, hipStream_t);
template void set<float>(long, float*, float, hipStream_t);

}  // namespace mgr
