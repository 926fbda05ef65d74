// k_setup.hip -- setup kernels for gfx950: block extraction by C/F split,
// F-relaxation operators, SpGEMM / sparse add / transpose (Petrov-Galerkin
// coarse operators of MGR and Galerkin products of AMG), PMIS coarsening,
// direct interpolation and the coarsest dense inverse.
//
// Built with -ffp-contract=off: the coarse values feed the strength-of-
// connection test of the next AMG level, so every sum is formed exactly in the
// order written (a separate multiply and add, no fused multiply-add).
#include <climits>

#include <algorithm>

#include "kernels.hpp"

namespace mgr {

namespace {

constexpr int TPB = 256;
constexpr int WAVE = 64;
constexpr int SCAN_T = 256;
constexpr int SCAN_I = 8;
static_assert(SCAN_I % 4 == 0, "scan runs are moved in 16-byte vectors");
constexpr int SCAN_B = SCAN_T * SCAN_I;

inline int nblk(long n, int t = TPB) { return (int)((n + t - 1) / t); }

__device__ inline int wave_min_int(int v) {
    for (int off = WAVE / 2; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, WAVE));
    return v;
}

__device__ inline void set_flag(int* flag, int code) { atomicMax(flag, code); }

// ------------------------------------------------------------------ scan
// Exclusive prefix sum in two passes: block sums (and block maxima), then block
// scans, each block first adding up the sums of the blocks before it (there
// are at most a few thousand).  The scan also reports the total and the
// largest input value (the longest row when the inputs are row counts) into a
// device slot.
__global__ void k_scan_reduce(const int* __restrict__ in, int n, long long* __restrict__ bsum,
                              long long* __restrict__ bmax) {
    __shared__ long long sh[SCAN_T];
    __shared__ int sm[SCAN_T];
    long long s = 0;
    int m = 0;
    int base = blockIdx.x * SCAN_B;
    for (int t = 0; t < SCAN_I; ++t) {
        int i = base + t * SCAN_T + threadIdx.x;
        if (i < n) { int v = in[i]; s += v; m = max(m, v); }
    }
    sh[threadIdx.x] = s;
    sm[threadIdx.x] = m;
    __syncthreads();
    for (int off = SCAN_T / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) {
            sh[threadIdx.x] += sh[threadIdx.x + off];
            sm[threadIdx.x] = max(sm[threadIdx.x], sm[threadIdx.x + off]);
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) { bsum[blockIdx.x] = sh[0]; bmax[blockIdx.x] = sm[0]; }
}

__global__ void k_scan_apply(const int* __restrict__ in, int n, const long long* __restrict__ bsum,
                             const long long* __restrict__ bmax, int nb, int* __restrict__ out,
                             long long* __restrict__ slot) {
    __shared__ int sh[SCAN_T];
    __shared__ long long wa[SCAN_T / WAVE], wm[SCAN_T / WAVE];
    __shared__ long long boff;
    const int tid = threadIdx.x, lane = tid & (WAVE - 1), wid = tid / WAVE;
    const bool last = (int)blockIdx.x == nb - 1;
    // this block's offset (and, in the last block, the total and the maximum)
    long long a = 0, m = 0;
    for (int b = tid; b < (int)blockIdx.x; b += SCAN_T) a += bsum[b];
    if (last)
        for (int b = tid; b < nb; b += SCAN_T) m = max(m, bmax[b]);
    for (int off = WAVE / 2; off > 0; off >>= 1) {
        a += __shfl_xor(a, off, WAVE);
        m = max(m, __shfl_xor(m, off, WAVE));
    }
    if (lane == 0) { wa[wid] = a; wm[wid] = m; }
    __syncthreads();
    if (tid == 0) {
        long long ta = 0, tm = 0;
        for (int q = 0; q < SCAN_T / WAVE; ++q) { ta += wa[q]; tm = max(tm, wm[q]); }
        boff = ta;
        if (last) {
            long long total = ta + bsum[nb - 1];
            out[n] = (total > INT_MAX) ? INT_MAX : (int)total;
            if (slot) { slot[0] = total; slot[1] = tm; }
        }
    }
    // each thread's SCAN_I consecutive inputs, in 16-byte loads where the
    // arrays are aligned and the run is whole
    int base = blockIdx.x * SCAN_B + tid * SCAN_I;
    const bool vec = base + SCAN_I - 1 < n &&
                     ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    int v[SCAN_I];
    int s = 0;
    if (vec) {
#pragma unroll
        for (int q = 0; q < SCAN_I / 4; ++q) {
            const int4 x = *reinterpret_cast<const int4*>(in + base + 4 * q);
            v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
        }
    } else {
#pragma unroll
        for (int t = 0; t < SCAN_I; ++t) {
            int i = base + t;
            v[t] = (i < n) ? in[i] : 0;
        }
    }
#pragma unroll
    for (int t = 0; t < SCAN_I; ++t) s += v[t];
    sh[tid] = s;
    __syncthreads();
    for (int off = 1; off < SCAN_T; off <<= 1) {
        int t = (tid >= off) ? sh[tid - off] : 0;
        __syncthreads();
        sh[tid] += t;
        __syncthreads();
    }
    long long off = boff + (tid ? sh[tid - 1] : 0);
    if (vec) {
#pragma unroll
        for (int q = 0; q < SCAN_I / 4; ++q) {
            int o[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                o[j] = (int)off;
                off += v[4 * q + j];
            }
            *reinterpret_cast<int4*>(out + base + 4 * q) = make_int4(o[0], o[1], o[2], o[3]);
        }
    } else {
        for (int t = 0; t < SCAN_I; ++t) {
            int i = base + t;
            if (i < n) out[i] = (int)off;
            off += v[t];
        }
    }
}

// Whole scan in one workgroup of SCAN_SMALL_T threads for n <= SCAN_SMALL:
// thread t owns a run of up to SCAN_SMALL_CH consecutive inputs (rounded up
// to a multiple of four and, with both arrays 16-byte aligned, read and
// written four at a time); wavefront scans, then a scan of the wave totals.
// A workgroup no larger than the setup's other kernels' gets a CU while an
// auxiliary-stream kernel fills the GPU (a 1024-thread one waited up to
// 0.23 ms for sixteen free wave slots on one CU).
constexpr int SCAN_SMALL_T = 256;
constexpr int SCAN_SMALL_CH = 64;
constexpr int SCAN_SMALL = SCAN_SMALL_T * SCAN_SMALL_CH;
constexpr int SCAN_SMALL_W = SCAN_SMALL_T / WAVE;

__global__ __launch_bounds__(SCAN_SMALL_T) void k_scan_small(const int* __restrict__ in, int n,
                                                             int* __restrict__ out, long long* __restrict__ slot) {
    __shared__ long long wsum[SCAN_SMALL_W];
    __shared__ int wmax[SCAN_SMALL_W];
    const int t = threadIdx.x, lane = t & (WAVE - 1), wid = t / WAVE;
    int chunk = (n + SCAN_SMALL_T - 1) / SCAN_SMALL_T;
    if (chunk > 1) chunk = (chunk + 3) & ~3;
    const bool vec = (chunk & 3) == 0 && ((reinterpret_cast<uintptr_t>(in) | reinterpret_cast<uintptr_t>(out)) & 15) == 0;
    const int b0 = t * chunk;
    int v[SCAN_SMALL_CH];
    long long sum = 0;
    int m = 0;
    if (vec) {
#pragma unroll
        for (int q = 0; q < SCAN_SMALL_CH / 4; ++q) {
            const int i = b0 + 4 * q;
            if (4 * q < chunk && i + 3 < n) {
                const int4 x = *reinterpret_cast<const int4*>(in + i);
                v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j) v[4 * q + j] = (4 * q < chunk && i + j < n) ? in[i + j] : 0;
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < SCAN_SMALL_CH; ++u) {
            const int i = b0 + u;
            v[u] = (u < chunk && i < n) ? in[i] : 0;
        }
    }
#pragma unroll
    for (int u = 0; u < SCAN_SMALL_CH; ++u) {
        sum += v[u];
        m = max(m, v[u]);
    }
    long long inc = sum;
    for (int off = 1; off < WAVE; off <<= 1) {
        long long o = __shfl_up(inc, off, WAVE);
        if (lane >= off) inc += o;
    }
    for (int off = WAVE / 2; off > 0; off >>= 1) m = max(m, __shfl_xor(m, off, WAVE));
    if (lane == WAVE - 1) wsum[wid] = inc;
    if (lane == 0) wmax[wid] = m;
    __syncthreads();
    // the waves before this one, and (thread 0) the total and the maximum
    long long before = 0, total = 0;
    int mx = 0;
#pragma unroll
    for (int q = 0; q < SCAN_SMALL_W; ++q) {
        if (q < wid) before += wsum[q];
        total += wsum[q];
        mx = max(mx, wmax[q]);
    }
    long long run = before + inc - sum;
    if (vec) {
#pragma unroll
        for (int q = 0; q < SCAN_SMALL_CH / 4; ++q) {
            const int i = b0 + 4 * q;
            int o[4];
#pragma unroll
            for (int j = 0; j < 4; ++j) {
                o[j] = (int)run;
                run += v[4 * q + j];
            }
            if (4 * q < chunk && i + 3 < n) {
                *reinterpret_cast<int4*>(out + i) = make_int4(o[0], o[1], o[2], o[3]);
            } else {
#pragma unroll
                for (int j = 0; j < 4; ++j)
                    if (4 * q < chunk && i + j < n) out[i + j] = o[j];
            }
        }
    } else {
#pragma unroll
        for (int u = 0; u < SCAN_SMALL_CH; ++u) {
            int i = b0 + u;
            if (u < chunk && i < n) out[i] = (int)run;
            run += v[u];
        }
    }
    if (t == 0) {
        out[n] = (total > INT_MAX) ? INT_MAX : (int)total;
        if (slot) { slot[0] = total; slot[1] = mx; }
    }
}

__global__ void k_fill_ll(long long* p, long long v, int n) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

// ------------------------------------------------------------------ misc
__global__ void k_fill_u8(unsigned char* p, unsigned char v, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_fill_int(int* p, int v, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) p[i] = v;
}

__global__ void k_to_float(const double* __restrict__ s, float* __restrict__ d, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) d[i] = (float)s[i];
}

// Several arrays converted by one launch: segment q owns the blocks from
// boff[q] on, each block TPB * F32_PER consecutive elements of it.
constexpr int F32_PER = 4;
__global__ __launch_bounds__(TPB) void k_to_float_batch(F32Segs sg) {
    const int b = blockIdx.x;
    int q = 0;
    while (q + 1 < sg.k && sg.boff[q + 1] <= b) ++q;
    const double* __restrict__ src = sg.src[q];
    float* __restrict__ dst = sg.dst[q];
    const long n = sg.n[q];
    const long base = (long)(b - sg.boff[q]) * TPB * F32_PER + threadIdx.x;
#pragma unroll
    for (int j = 0; j < F32_PER; ++j) {
        const long i = base + (long)j * TPB;
        if (i < n) dst[i] = (float)src[i];
    }
}

__global__ void k_negate(double* v, long n) {
    long i = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) v[i] = -v[i];
}

__global__ void k_iota_div(int n, int b, int* __restrict__ out) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) out[i] = i / b;
}

__global__ void k_gather_int(int n, const int* __restrict__ map, const int* __restrict__ src, int* __restrict__ dst) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) dst[i] = src[map[i]];
}

// ------------------------------------------------------------------ block layout
// Scalar row i = I*b + r holds, for each block of block row I in order, the b
// entries of block row r: the same order the block values are stored in.
__global__ void k_bsr_tcount(long nnzb, const int* __restrict__ ci, int* __restrict__ cnt) {
    long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnzb) atomicAdd(&cnt[ci[p]], 1);
}

__global__ void k_bsr_tscatter(int nbr, const int* __restrict__ rp, const int* __restrict__ ci,
                               int* __restrict__ cursor, int* __restrict__ tci, int* __restrict__ src) {
    int I = blockIdx.x * blockDim.x + threadIdx.x;
    if (I >= nbr) return;
    for (int p = rp[I]; p < rp[I + 1]; ++p) {
        int q = atomicAdd(&cursor[ci[p]], 1);
        tci[q] = I;
        src[q] = p;
    }
}

__global__ void k_bsr_tsort(int nbr, const int* __restrict__ trp, int* __restrict__ tci, int* __restrict__ src) {
    int J = blockIdx.x * blockDim.x + threadIdx.x;
    if (J >= nbr) return;
    int q0 = trp[J], q1 = trp[J + 1];
    for (int q = q0 + 1; q < q1; ++q) {
        int key = tci[q], s = src[q], t = q - 1;
        while (t >= q0 && tci[t] > key) { tci[t + 1] = tci[t]; src[t + 1] = src[t]; --t; }
        tci[t + 1] = key;
        src[t + 1] = s;
    }
}

__global__ void k_bsr_tvalues(long nnzb, int b, const int* __restrict__ src, const double* __restrict__ v,
                              double* __restrict__ tv) {
    long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nnzb) return;
    const double* a = v + (long)src[q] * b * b;
    double* t = tv + q * b * b;
    for (int r = 0; r < b; ++r)
        for (int c = 0; c < b; ++c) t[r * b + c] = a[c * b + r];
}

// ------------------------------------------------------------------ C/F split and block extraction
// Histogram of the field labels (32 bins, hist zeroed beforehand); a label
// outside [0, 32) sets *flag to 5.
__global__ __launch_bounds__(TPB) void k_field_hist(int n, const int* __restrict__ field, int* __restrict__ hist,
                                                    int* __restrict__ flag) {
    __shared__ int h[32];
    if (threadIdx.x < 32) h[threadIdx.x] = 0;
    __syncthreads();
    // per wavefront, one atomic per distinct label (there are few)
    for (int base = blockIdx.x * TPB; base < n; base += gridDim.x * TPB) {
        const int i = base + threadIdx.x;
        int f = (i < n) ? field[i] : -1;
        if (i < n && (f < 0 || f >= 32)) {
            set_flag(flag, 5);
            f = -1;
        }
        bool left = f >= 0;
        while (__any(left)) {
            const unsigned long long act = __ballot(left);
            const int lead = __ffsll(act) - 1;
            const int fl = __shfl(f, lead, WAVE);
            const unsigned long long same = __ballot(left && f == fl);
            if ((int)(threadIdx.x & (WAVE - 1)) == lead) atomicAdd(&h[fl], (int)__popcll(same));
            if (left && f == fl) left = false;
        }
    }
    __syncthreads();
    if (threadIdx.x < 32 && h[threadIdx.x]) atomicAdd(&hist[threadIdx.x], h[threadIdx.x]);
}

__global__ void k_cf_flags(int n, const int* __restrict__ field, uint32_t mask, int* __restrict__ isF,
                           int* __restrict__ flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int f = field[i];
    if (f < 0 || f >= 32) { set_flag(flag, 5); isF[i] = 0; return; }
    isF[i] = (int)((mask >> f) & 1u);
}

__global__ void k_cf_maps(int n, const int* __restrict__ isF, const int* __restrict__ fpos, int* __restrict__ lmap,
                          int* __restrict__ fmap, int* __restrict__ cmap) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    if (isF[i]) { int k = fpos[i]; lmap[i] = k; fmap[k] = i; }
    else { int c = i - fpos[i]; lmap[i] = c; cmap[c] = i; }
}



// ------------------------------------------------------------------ F-relaxation operator
__global__ void k_frelax_flags(int nF, const int* __restrict__ bid, int* __restrict__ flagk) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nF) return;
    flagk[k] = (bid == nullptr || k == 0 || bid[k] != bid[k - 1]) ? 1 : 0;
}

__global__ void k_frelax_starts(int nF, const int* __restrict__ flagk, const int* __restrict__ excl,
                                int* __restrict__ bstart, int* __restrict__ bnum) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nF) return;
    int b = excl[k] + flagk[k] - 1;
    bnum[k] = b;
    if (flagk[k]) bstart[b] = k;
    if (k == nF - 1) bstart[excl[nF]] = nF;
}

// Row lengths of M: the size of the row's block, at most 4.  A larger block
// (caller-supplied groups) is flagged unsupported and its rows get a single
// (zero) entry, so that M stays small and valid until the flag is read.
__global__ void k_frelax_len(int nF, const int* __restrict__ bnum, const int* __restrict__ bstart,
                             int* __restrict__ len, int* __restrict__ flag) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= nF) return;
    int b = bnum[k];
    const int bs = bstart[b + 1] - bstart[b];
    if (bs > 4) {
        len[k] = 1;
        if (k == bstart[b]) set_flag(flag, 6);
    } else {
        len[k] = bs;
    }
}

// Inverse of one BS x BS diagonal block by Gauss-Jordan with partial pivoting
// (ties keep the row with the lower index): scale the pivot row by 1/pivot,
// then subtract f times it from every other row.  Every index is static so the
// block stays in registers.  Returns false on a zero or non-finite pivot.
template <int BS>
__device__ inline bool block_inverse(double (&a)[BS][BS], double (&e)[BS][BS]) {
#pragma unroll
    for (int r = 0; r < BS; ++r)
#pragma unroll
        for (int c = 0; c < BS; ++c) e[r][c] = (r == c) ? 1.0 : 0.0;
#pragma unroll
    for (int c = 0; c < BS; ++c) {
        int pv = c;
        double best = fabs(a[c][c]);
#pragma unroll
        for (int r = c + 1; r < BS; ++r)
            if (fabs(a[r][c]) > best) { best = fabs(a[r][c]); pv = r; }
        if (!(best > 0.0) || !isfinite(best)) return false;
#pragma unroll
        for (int r = c + 1; r < BS; ++r)
            if (r == pv)
#pragma unroll
                for (int k = 0; k < BS; ++k) {
                    double x = a[c][k]; a[c][k] = a[r][k]; a[r][k] = x;
                    x = e[c][k]; e[c][k] = e[r][k]; e[r][k] = x;
                }
        double ip = 1.0 / a[c][c];
#pragma unroll
        for (int k = 0; k < BS; ++k) { a[c][k] = a[c][k] * ip; e[c][k] = e[c][k] * ip; }
#pragma unroll
        for (int r = 0; r < BS; ++r) {
            if (r == c) continue;
            double f = a[r][c];
#pragma unroll
            for (int k = 0; k < BS; ++k) {
                a[r][k] = a[r][k] - f * a[c][k];
                e[r][k] = e[r][k] - f * e[c][k];
            }
        }
    }
    return true;
}

// One block with a group of four lanes: lane r reads the diagonal-block part of
// row s0 + r (eight entries per load batch), the rows are exchanged, every
// lane inverts the block and lane r writes row r of M.
template <int BS>
__device__ inline void frelax_block(int s0, int gl, int gbase, const int* __restrict__ arp,
                                    const int* __restrict__ aci, const double* __restrict__ av,
                                    const int* __restrict__ mrp, int* __restrict__ mci, double* __restrict__ mv,
                                    int* __restrict__ flag) {
    double row[BS];
#pragma unroll
    for (int c = 0; c < BS; ++c) row[c] = 0.0;
    if (gl < BS) {
        const int p1 = arp[s0 + gl + 1];
        for (int p = arp[s0 + gl]; p < p1; p += 8) {
            int cs[8];
            double vs[8];
#pragma unroll
            for (int u = 0; u < 8; ++u) {
                cs[u] = (p + u < p1) ? aci[p + u] - s0 : -1;
                vs[u] = (p + u < p1) ? av[p + u] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < 8; ++u)
#pragma unroll
                for (int c = 0; c < BS; ++c)
                    if (cs[u] == c) row[c] = vs[u];
        }
    }
    double a[BS][BS], e[BS][BS];
#pragma unroll
    for (int r = 0; r < BS; ++r)
#pragma unroll
        for (int c = 0; c < BS; ++c) a[r][c] = __shfl(row[c], gbase + r, WAVE);
    const bool ok = block_inverse<BS>(a, e);
    if (!ok && gl == 0) set_flag(flag, 3);
    if (gl < BS) {
        const int o = mrp[s0 + gl];
#pragma unroll
        for (int c = 0; c < BS; ++c) {
            double x = 0.0;
#pragma unroll
            for (int r = 0; r < BS; ++r)
                if (r == gl) x = e[r][c];
            mci[o + c] = s0 + c;
            mv[o + c] = ok ? x : 0.0;
        }
    }
}

// M = block-diagonal inverse of A_FF over the blocks [bstart[t], bstart[t+1]),
// four lanes per block.  On a failure (block larger than 4, zero or non-finite
// pivot) the flag is raised and the rows are still written, with valid column
// indices and zero values, so that no later kernel reads an unwritten index.
__global__ __launch_bounds__(TPB) void k_frelax_fill(int nb, const int* __restrict__ bstart,
                                                     const int* __restrict__ arp, const int* __restrict__ aci,
                                                     const double* __restrict__ av, const int* __restrict__ mrp,
                                                     int* __restrict__ mci, double* __restrict__ mv,
                                                     int* __restrict__ flag) {
    const int t = (int)(((long)blockIdx.x * TPB + threadIdx.x) / 4);
    const int gl = threadIdx.x & 3, gbase = (threadIdx.x & (WAVE - 1)) - gl;
    if (t >= nb) return;
    const int s0 = bstart[t], bs = bstart[t + 1] - s0;
    switch (bs) {
        case 1: frelax_block<1>(s0, gl, gbase, arp, aci, av, mrp, mci, mv, flag); break;
        case 2: frelax_block<2>(s0, gl, gbase, arp, aci, av, mrp, mci, mv, flag); break;
        case 3: frelax_block<3>(s0, gl, gbase, arp, aci, av, mrp, mci, mv, flag); break;
        case 4: frelax_block<4>(s0, gl, gbase, arp, aci, av, mrp, mci, mv, flag); break;
        default:
            // a block larger than 4 (flagged by k_frelax_len): one zero entry
            // per row on its diagonal, a valid column for the products that
            // may read M before the flag is seen
            if (gl == 0) {
                set_flag(flag, 6);
                for (int r = 0; r < bs; ++r) {
                    int o = mrp[s0 + r];
                    mci[o] = s0 + r;
                    mv[o] = 0.0;
                }
            }
    }
}

// ------------------------------------------------------------------ sparse products
// C = A B, one wavefront per output row.  Each lane owns up to NH entries p of
// row i of A (p = a0 + lane + 64 t) and walks row aci[p] of B: a k-way merge
// whose current minimum column is found by a wave-wide min.  Every output
// value starts at 0.0 and adds a_ip * b_pj over the contributing p in
// ascending order (t-major, then lane), i.e. Gustavson's order.
template <int NH, bool FILL>
__global__ __launch_bounds__(TPB) void k_spgemm(int nr, const int* __restrict__ arp, const int* __restrict__ aci,
                                                const double* __restrict__ av, const int* __restrict__ brp,
                                                const int* __restrict__ bci, const double* __restrict__ bv,
                                                const int* __restrict__ crp, int* __restrict__ cci,
                                                double* __restrict__ cv, int* __restrict__ cnt,
                                                int* __restrict__ flag) {
    int row = blockIdx.x * (TPB / WAVE) + threadIdx.x / WAVE;
    int lane = threadIdx.x & (WAVE - 1);
    if (row >= nr) return;
    int a0 = arp[row], a1 = arp[row + 1];
    if (a1 - a0 > NH * WAVE) {
        // too long for this variant: reported through *flag so the caller reruns
        // the product with more heads per lane
        if (lane == 0) {
            if (!FILL) cnt[row] = 0;
            if (flag) atomicMax(flag, 1);
        }
        return;
    }
    int h[NH], e[NH], c[NH];
    double a[NH];
#pragma unroll
    for (int t = 0; t < NH; ++t) {
        int p = a0 + lane + WAVE * t;
        c[t] = INT_MAX;
        h[t] = 0;
        e[t] = 0;
        a[t] = 0.0;
        if (p < a1) {
            int k = aci[p];
            h[t] = brp[k];
            e[t] = brp[k + 1];
            a[t] = FILL ? av[p] : 0.0;
            if (h[t] < e[t]) c[t] = bci[h[t]];
        }
    }
    int count = 0;
    int o = FILL ? crp[row] : 0;
    for (;;) {
        int mn = c[0];
#pragma unroll
        for (int t = 1; t < NH; ++t) mn = min(mn, c[t]);
        mn = wave_min_int(mn);
        if (mn == INT_MAX) break;
        if (FILL) {
            double acc = 0.0;
#pragma unroll
            for (int t = 0; t < NH; ++t) {
                bool m = (c[t] == mn);
                double prod = m ? a[t] * bv[h[t]] : 0.0;
                unsigned long long mask = __ballot(m);
                while (mask) {
                    int l = __ffsll((unsigned long long)mask) - 1;
                    acc = acc + __shfl(prod, l, WAVE);
                    mask &= mask - 1;
                }
            }
            if (lane == 0) {
                cci[o + count] = mn;
                cv[o + count] = acc;
            }
        }
#pragma unroll
        for (int t = 0; t < NH; ++t)
            if (c[t] == mn) {
                ++h[t];
                c[t] = (h[t] < e[t]) ? bci[h[t]] : INT_MAX;
            }
        ++count;
    }
    if (!FILL && lane == 0) cnt[row] = count;
}

// The same product with a lane group of G (<= 32) lanes per row, several rows
// per wavefront, for left factors whose rows have at most G entries.  Control
// flow is kept uniform across the wavefront (groups that are done idle), and
// each output value still adds its products in the order of the entries of the
// row of A (lane order inside the group).
template <int G, bool FILL>
__global__ __launch_bounds__(TPB) void k_spgemm_g(int nr, const int* __restrict__ arp, const int* __restrict__ aci,
                                                  const double* __restrict__ av, const int* __restrict__ brp,
                                                  const int* __restrict__ bci, const double* __restrict__ bv,
                                                  const int* __restrict__ crp, int* __restrict__ cci,
                                                  double* __restrict__ cv, int* __restrict__ cnt,
                                                  int* __restrict__ flag) {
    const int lane = threadIdx.x & (WAVE - 1);
    const int gl = lane & (G - 1);
    const int gbase = lane - gl;
    const unsigned long long gmask_all = (G >= 64) ? ~0ULL : ((1ULL << G) - 1ULL);
    const int row = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    bool valid = row < nr;
    int a0 = 0, a1 = 0;
    if (valid) {
        a0 = arp[row];
        a1 = arp[row + 1];
        if (a1 - a0 > G) {
            if (gl == 0) {
                if (!FILL) cnt[row] = 0;
                if (flag) atomicMax(flag, 1);
            }
            valid = false;
        }
    }
    int h = 0, e = 0, c = INT_MAX;
    double a = 0.0;
    const int p = a0 + gl;
    if (valid && p < a1) {
        int k = aci[p];
        h = brp[k];
        e = brp[k + 1];
        if (FILL) a = av[p];
        if (h < e) c = bci[h];
    }
    int count = 0;
    const int o = (FILL && valid) ? crp[row] : 0;
    for (;;) {
        int mn = c;
        for (int off = G / 2; off > 0; off >>= 1) mn = min(mn, __shfl_xor(mn, off, WAVE));
        if (!__any(mn != INT_MAX)) break;
        const bool m = (mn != INT_MAX) && (c == mn);
        if (FILL) {
            double prod = m ? a * bv[h] : 0.0;
            unsigned long long gm = (__ballot(m) >> gbase) & gmask_all;
            int nb = __popcll(gm);
            for (int off = WAVE / 2; off > 0; off >>= 1) nb = max(nb, __shfl_xor(nb, off, WAVE));
            double acc = 0.0;
            for (int it = 0; it < nb; ++it) {
                int src = gbase + (gm ? (__ffsll((unsigned long long)gm) - 1) : 0);
                double v = __shfl(prod, src, WAVE);
                if (gm) {
                    acc = acc + v;
                    gm &= gm - 1;
                }
            }
            if (gl == 0 && mn != INT_MAX) {
                cci[o + count] = mn;
                cv[o + count] = acc;
            }
        }
        if (m) {
            ++h;
            c = (h < e) ? bci[h] : INT_MAX;
        }
        if (mn != INT_MAX) ++count;
    }
    if (!FILL && valid && gl == 0) cnt[row] = count;
}

// The same product for a right factor with few columns (<= SPGEMM_DENSE): one
// wavefront per output row accumulates into a dense LDS row.  The entries of
// the row of A are taken one after another and, for each, the lanes add the
// products of the distinct columns of the matching row of B, so every output
// value still starts at 0.0 and adds its products in the order of A's entries
// (Gustavson's order).  Row data for four entries of A is loaded ahead, so the
// wave waits on global memory once per four entries; the pattern is the set of
// touched columns (structural, like the merge variants), compacted in column
// order at the end.
constexpr int SPGEMM_DENSE = SPGEMM_DENSE_COLS;
// rows x columns above which clearing and compacting the dense rows costs more
// than the merge
constexpr long SPGEMM_DENSE_WORK = 64L * 1024 * 1024;
// a workgroup per output row: beyond this many rows the short merge variants win
constexpr int SPGEMM_DENSE_ROWS = 65536;

template <bool FILL>
__global__ __launch_bounds__(WAVE) void k_spgemm_dw(int nr, const int* __restrict__ arp, const int* __restrict__ aci,
                                                    const double* __restrict__ av, const int* __restrict__ brp,
                                                    const int* __restrict__ bci, const double* __restrict__ bv,
                                                    int ncols, const int* __restrict__ crp, int* __restrict__ cci,
                                                    double* __restrict__ cv, int* __restrict__ cnt) {
    // dynamic LDS sized to the columns: ncols doubles (fill only), then ncols flags
    extern __shared__ double dyn_lds[];
    double* acc = dyn_lds;
    unsigned char* hit = reinterpret_cast<unsigned char*>(dyn_lds + (FILL ? ncols : 0));
    const int row = blockIdx.x;
    const int lane = threadIdx.x;
    if (row >= nr) return;
    for (int c = lane; c < ncols; c += WAVE) {
        hit[c] = 0;
        if (FILL) acc[c] = 0.0;
    }
    const int a0 = arp[row], a1 = arp[row + 1];
    for (int base = a0; base < a1; base += WAVE) {
        // lane t holds entry base + t of the row of A and the extent of its row of B
        int kb0 = 0, kb1 = 0;
        double ka = 0.0;
        if (base + lane < a1) {
            int k = aci[base + lane];
            kb0 = brp[k];
            kb1 = brp[k + 1];
            if (FILL) ka = av[base + lane];
        }
        const int cnt_here = min(WAVE, a1 - base);
        for (int t0 = 0; t0 < cnt_here; t0 += 4) {
            int jj[4], b0[4], b1[4];
            double vv[4], aa[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                int t = min(t0 + u, cnt_here - 1);
                b0[u] = __shfl(kb0, t, WAVE);
                b1[u] = __shfl(kb1, t, WAVE);
                aa[u] = __shfl(ka, t, WAVE);
                int q = b0[u] + lane;
                jj[u] = -1;
                vv[u] = 0.0;
                if (t0 + u < cnt_here && q < b1[u]) {
                    jj[u] = bci[q];
                    if (FILL) vv[u] = bv[q];
                }
            }
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                if (t0 + u < cnt_here) {
                    if (jj[u] >= 0) {
                        hit[jj[u]] = 1;
                        if (FILL) acc[jj[u]] = acc[jj[u]] + aa[u] * vv[u];
                    }
                    // rows of B longer than a wavefront
                    for (int q = b0[u] + WAVE + lane; q < b1[u]; q += WAVE) {
                        int j = bci[q];
                        hit[j] = 1;
                        if (FILL) acc[j] = acc[j] + aa[u] * bv[q];
                    }
                }
            }
        }
    }
    // compaction in column order: lane l scans columns [l*chunk, (l+1)*chunk)
    const int chunk = (ncols + WAVE - 1) / WAVE;
    const int c0 = min(lane * chunk, ncols), c1 = min(c0 + chunk, ncols);
    int mine = 0;
    for (int c = c0; c < c1; ++c) mine += hit[c];
    int incl = mine;
    for (int off = 1; off < WAVE; off <<= 1) {
        int o = __shfl_up(incl, off, WAVE);
        if (lane >= off) incl += o;
    }
    if (!FILL) {
        if (lane == WAVE - 1) cnt[row] = incl;
        return;
    }
    int o = crp[row] + incl - mine;
    for (int c = c0; c < c1; ++c)
        if (hit[c]) {
            cci[o] = c;
            cv[o] = acc[c];
            ++o;
        }
}

__global__ void k_transpose_count(long nnz, const int* __restrict__ ci, int* __restrict__ cnt) {
    long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) atomicAdd(&cnt[ci[p]], 1);
}

// Row i of the transpose, scattered in arbitrary order into tci / tv, is
// written to ci / v in ascending column order: one wavefront per row, the
// position of each entry is the number of smaller keys in the row (keys of a
// row are distinct).
__global__ __launch_bounds__(TPB) void k_transpose_rank(int nr, const int* __restrict__ rp,
                                                        const int* __restrict__ tci, const double* __restrict__ tv,
                                                        int* __restrict__ ci, double* __restrict__ v) {
    const int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / WAVE);
    const int lane = threadIdx.x & (WAVE - 1);
    if (i >= nr) return;
    const int q0 = rp[i], q1 = rp[i + 1];
    for (int u0 = q0; u0 < q1; u0 += WAVE) {
        const int q = u0 + lane;
        const int key = (q < q1) ? tci[q] : INT_MAX;
        int rank = 0;
        for (int base = q0; base < q1; base += WAVE) {
            int kk = (base + lane < q1) ? tci[base + lane] : INT_MAX;
            const int lim = min(WAVE, q1 - base);
            for (int t = 0; t < lim; ++t) rank += (__shfl(kk, t, WAVE) < key) ? 1 : 0;
        }
        if (q < q1) {
            ci[q0 + rank] = key;
            if (v) v[q0 + rank] = tv[q];
        }
    }
}



__global__ void k_scount(int n, const int* __restrict__ rp, const unsigned char* __restrict__ strong,
                         int* __restrict__ cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) c += strong[p];
    cnt[i] = c;
}


// splitmix64 (Steele, Lea, Flood 2014): output k of the stream seeded with
// `seed` is mix(seed + k * 0x9E3779B97F4A7C15).
__device__ inline uint64_t splitmix64(uint64_t seed, uint64_t k) {
    uint64_t z = seed + k * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

__global__ void k_pmis_init(int n, const int* __restrict__ lam, uint64_t seed, int level, double* __restrict__ w,
                            int* __restrict__ cf) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    uint64_t k = ((uint64_t)(unsigned)level << 32) + (uint64_t)(unsigned)i + 1ULL;
    double u = (double)(splitmix64(seed, k) >> 11) * (1.0 / 9007199254740992.0);
    w[i] = (double)lam[i] + u;
    cf[i] = (lam[i] == 0) ? -1 : 0;
}

__global__ void k_is_c(int n, const int* __restrict__ cf, int* __restrict__ isC) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) isC[i] = (cf[i] == 1) ? 1 : 0;
}




// one workgroup per row: the row (nc entries) is cleared, then its entries are stored
__global__ void k_densify(int nc, const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ v,
                          double* __restrict__ dense) {
    const int i = blockIdx.x;
    double* row = dense + (long)i * nc;
    for (int j = threadIdx.x; j < nc; j += blockDim.x) row[j] = 0.0;
    __syncthreads();
    for (int p = rp[i] + threadIdx.x; p < rp[i + 1]; p += blockDim.x) row[ci[p]] = v[p];
}

// C (m x n) = A (m x k) B (k x n), dense row-major, one thread per entry
// (small factors only: the coarse tail of an AMG cycle).
__global__ void k_dense_gemm(int m, int k, int n, const double* __restrict__ a, const double* __restrict__ b,
                             double* __restrict__ c) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)m * n) return;
    const int i = (int)(idx / n), j = (int)(idx % n);
    double acc = 0.0;
    for (int q = 0; q < k; ++q) acc += a[(long)i * k + q] * b[(long)q * n + j];
    c[idx] = acc;
}

// T (nr x n, dense) += Q X with Q sparse (nr rows) and X dense (rows of n):
// one workgroup per row of T.
__global__ void k_sparse_dense_add(int n, const int* __restrict__ qrp, const int* __restrict__ qci,
                                   const double* __restrict__ qv, const double* __restrict__ x,
                                   double* __restrict__ t) {
    const int i = blockIdx.x;
    const int p0 = qrp[i], p1 = qrp[i + 1];
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        double acc = t[(long)i * n + j];
        for (int p = p0; p < p1; ++p) acc += qv[p] * x[(long)qci[p] * n + j];
        t[(long)i * n + j] = acc;
    }
}

__global__ void k_dense_transpose(int n, const double* __restrict__ a, double* __restrict__ t) {
    const long idx = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (idx >= (long)n * n) return;
    const int i = (int)(idx / n), j = (int)(idx % n);
    t[(long)j * n + i] = a[idx];
}

// Gauss-Jordan inverse with partial pivoting of the coarsest AMG matrix, one
// workgroup (n <= 2048): a and inv are n x n row-major in global memory.
__global__ __launch_bounds__(1024) void k_dense_inverse(int n, double* __restrict__ a, double* __restrict__ inv,
                                                        double* __restrict__ fcol, int* __restrict__ flag) {
    __shared__ double sv[1024];
    __shared__ int si[1024];
    int tid = threadIdx.x, nt = blockDim.x;
    for (long q = tid; q < (long)n * n; q += nt) inv[q] = ((q / n) == (q % n)) ? 1.0 : 0.0;
    __syncthreads();
    for (int c = 0; c < n; ++c) {
        double best = -1.0;
        int bi = n;
        for (int r = c + tid; r < n; r += nt) {
            double t = fabs(a[(long)r * n + c]);
            if (t > best || (t == best && r < bi)) { best = t; bi = r; }
        }
        sv[tid] = best;
        si[tid] = bi;
        __syncthreads();
        for (int off = nt / 2; off > 0; off >>= 1) {
            if (tid < off) {
                double o = sv[tid + off];
                int oi = si[tid + off];
                if (o > sv[tid] || (o == sv[tid] && oi < si[tid])) { sv[tid] = o; si[tid] = oi; }
            }
            __syncthreads();
        }
        int pv = si[0];
        double pbest = sv[0];
        __syncthreads();
        if (!(pbest > 0.0) || !isfinite(pbest)) {
            if (tid == 0) set_flag(flag, 3);
            return;
        }
        if (pv != c)
            for (int k = tid; k < n; k += nt) {
                double x = a[(long)c * n + k]; a[(long)c * n + k] = a[(long)pv * n + k]; a[(long)pv * n + k] = x;
                x = inv[(long)c * n + k]; inv[(long)c * n + k] = inv[(long)pv * n + k]; inv[(long)pv * n + k] = x;
            }
        __syncthreads();
        double ip = 1.0 / a[(long)c * n + c];
        __syncthreads();
        for (int k = tid; k < n; k += nt) {
            a[(long)c * n + k] = a[(long)c * n + k] * ip;
            inv[(long)c * n + k] = inv[(long)c * n + k] * ip;
        }
        for (int r = tid; r < n; r += nt) fcol[r] = a[(long)r * n + c];
        __syncthreads();
        for (long q = tid; q < (long)n * n; q += nt) {
            int r = (int)(q / n), k = (int)(q % n);
            if (r == c) continue;
            double f = fcol[r];
            a[q] = a[q] - f * a[(long)c * n + k];
            inv[q] = inv[q] - f * inv[(long)c * n + k];
        }
        __syncthreads();
    }
}

// ------------------------------------------------------------------ ILU(0) of A_FF
// Level of a row in a triangular dependency graph: rows with no dependency are
// level 0, otherwise 1 + the largest level they depend on.  Computed by
// monotone relaxation sweeps (levels only grow toward the fixed point, so stale
// reads of a neighbour's level during a sweep are harmless).  fwd: row i
// depends on the columns k < i of its row; !fwd: on the columns k > i.
__global__ void k_level_sweep(int n, const int* __restrict__ rp, const int* __restrict__ ci, int fwd,
                              int* lev, int* __restrict__ changed) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int m = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        int k = ci[p];
        if ((fwd && k < i) || (!fwd && k > i)) m = max(m, ((volatile int*)lev)[k] + 1);
    }
    if (m > lev[i]) {
        lev[i] = m;
        *changed = 1;
    }
}

__global__ void k_level_max(int n, const int* __restrict__ lev, int* __restrict__ out) {
    __shared__ int sh[TPB];
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    sh[threadIdx.x] = (i < n) ? lev[i] : 0;
    __syncthreads();
    for (int off = TPB / 2; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) sh[threadIdx.x] = max(sh[threadIdx.x], sh[threadIdx.x + off]);
        __syncthreads();
    }
    if (threadIdx.x == 0) atomicMax(out, sh[0]);
}

__global__ void k_level_count(int n, const int* __restrict__ lev, int* __restrict__ cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) atomicAdd(&cnt[lev[i]], 1);
}

__global__ void k_level_scatter(int n, const int* __restrict__ lev, int* __restrict__ cursor, int* __restrict__ order) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) order[atomicAdd(&cursor[lev[i]], 1)] = i;
}

__global__ void k_diag_pos(int n, const int* __restrict__ rp, const int* __restrict__ ci, int* __restrict__ dpos,
                           int* __restrict__ flag) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int d = -1;
    for (int p = rp[i]; p < rp[i + 1]; ++p)
        if (ci[p] == i) d = p;
    dpos[i] = d;
    if (d < 0) set_flag(flag, 3);
}

// ILU(0) of one level of rows (Saad, Iterative Methods, ILU(0) in IKJ order):
// for each k < i in row i, in column order: l = a_ik / u_kk; a_ik = l; then
// a_ij -= l * u_kj for the entries j > k of row k present in row i.  Every
// row of an earlier level is final, so the arithmetic equals the sequential one.
__global__ void k_ilu_level(int cnt, const int* __restrict__ rows, const int* __restrict__ rp,
                            const int* __restrict__ ci, const int* __restrict__ dpos, double* lu,
                            int* __restrict__ flag) {
    int t = blockIdx.x * blockDim.x + threadIdx.x;
    if (t >= cnt) return;
    int i = rows[t];
    int p0 = rp[i], p1 = rp[i + 1];
    for (int p = p0; p < p1; ++p) {
        int k = ci[p];
        if (k >= i) break;
        double ukk = lu[dpos[k]];
        if (ukk == 0.0) { set_flag(flag, 3); continue; }
        double l = lu[p] / ukk;
        lu[p] = l;
        int q = dpos[k] + 1, qe = rp[k + 1], r = p + 1;
        while (q < qe && r < p1) {
            int cq = ci[q], cr = ci[r];
            if (cq == cr) { lu[r] = lu[r] - l * lu[q]; ++q; ++r; }
            else if (cq < cr) ++q;
            else ++r;
        }
    }
    double d = lu[dpos[i]];
    if (d == 0.0 || !isfinite(d)) set_flag(flag, 3);
}

// split the factors: L = strict lower part (unit diagonal implied), U = diagonal and upper part
__global__ void k_split_count(int n, const int* __restrict__ rp, const int* __restrict__ ci, int* __restrict__ nl,
                              int* __restrict__ nu) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int a = 0, b = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        if (ci[p] < i) ++a;
        else ++b;
    }
    nl[i] = a;
    nu[i] = b;
}

__global__ void k_split_fill(int n, const int* __restrict__ rp, const int* __restrict__ ci, const double* __restrict__ v,
                             const int* __restrict__ lrp, int* __restrict__ lci, double* __restrict__ lv,
                             const int* __restrict__ urp, int* __restrict__ uci, double* __restrict__ uv) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int a = lrp[i], b = urp[i];
    for (int p = rp[i]; p < rp[i + 1]; ++p) {
        if (ci[p] < i) { lci[a] = ci[p]; lv[a] = v[p]; ++a; }
        else { uci[b] = ci[p]; uv[b] = v[p]; ++b; }
    }
}

// ------------------------------------------------------------------ lane-group-per-row variants
// The kernels below give each row a group of G lanes (G a power of two <= 64,
// chosen from the longest row) so that the row's entries are read with
// coalesced loads.  Compaction keeps the entries' order (ballot + prefix
// popcount); every reduction that feeds a bit-exact result is exact (counts,
// maxima) or kept strictly sequential (interpolation sums).
template <int G>
struct Grp {
    int lane, gl, gbase;
    unsigned long long gmask;
    __device__ Grp() {
        lane = threadIdx.x & (WAVE - 1);
        gl = lane & (G - 1);
        gbase = lane - gl;
        gmask = (G >= 64) ? ~0ULL : ((1ULL << G) - 1ULL);
    }
    __device__ unsigned long long bits(bool pred) const { return (__ballot(pred) >> gbase) & gmask; }
    __device__ int below(unsigned long long b) const { return __popcll(b & ((1ULL << gl) - 1ULL)); }
    __device__ int sum(int v) const {
        for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
        return v;
    }
    __device__ double sumd(double v) const {
        for (int off = G / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
        return v;
    }
};

__device__ inline int wave_max_int(int v) {
    for (int off = WAVE / 2; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, WAVE));
    return v;
}

// a thread per point (which stops at the first deciding neighbour) for short
// strong rows or many points; lane groups for small levels with long rows
constexpr int PMIS_GROUP_MIN = 12;
constexpr int PMIS_GROUP_MAX_N = 65536;

// PMIS round, G lanes per point, without the transpose of S.  Selection: an
// undecided point j is beaten when an undecided point of S_j or of S^T_j (a
// point i with j in S_i) has the larger (w, index), judged on the state cf at
// the start of the round.  Each undecided point walks its own row S_j once:
// a neighbour that beats it marks j (pull), a neighbour it beats is marked
// (push: j is in that neighbour's S^T row).  The marks are plain stores of 1.
template <int G>
__global__ __launch_bounds__(TPB) void k_pmis_select_g(int n, const int* __restrict__ srp, const int* __restrict__ sci,
                                                       const double* __restrict__ w, const int* __restrict__ cf,
                                                       unsigned char* __restrict__ beaten) {
    Grp<G> g;
    const int j = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    if (j >= n || cf[j] != 0) return;
    const double wj = w[j];
    bool lost = false;
    for (int q = srp[j] + g.gl; q < srp[j + 1]; q += G) {
        const int i = sci[q];
        if (cf[i] != 0) continue;
        const double wi = w[i];
        if (wi > wj || (wi == wj && i > j)) lost = true;
        else beaten[i] = 1;
    }
    if (lost) beaten[j] = 1;
}

// Update: undecided points that were not beaten become C; an undecided point
// that strongly depends on a new C-point becomes F.  Reads the round's state
// (cf, beaten), writes the next one (cf_next, and beaten_next cleared), and
// counts what is still undecided (one atomic per wave).
template <int G>
__global__ __launch_bounds__(TPB) void k_pmis_update_g(int n, const int* __restrict__ srp, const int* __restrict__ sci,
                                                       const int* __restrict__ cf,
                                                       const unsigned char* __restrict__ beaten,
                                                       int* __restrict__ cf_next, unsigned char* __restrict__ beaten_next,
                                                       int* __restrict__ undecided) {
    Grp<G> g;
    const int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    const bool valid = i < n;
    const int ci_ = valid ? cf[i] : 1;
    const bool isnew = valid && ci_ == 0 && !beaten[i];
    const bool und = valid && ci_ == 0 && !isnew;
    bool hit = false;
    if (und)
        for (int q = srp[i] + g.gl; q < srp[i + 1] && !hit; q += G) {
            const int j = sci[q];
            if (cf[j] == 0 && !beaten[j]) hit = true;
        }
    hit = g.bits(hit) != 0;
    if (valid && g.gl == 0) {
        cf_next[i] = isnew ? 1 : (und ? (hit ? -1 : 0) : ci_);
        beaten_next[i] = 0;
    }
    const unsigned long long left = __ballot(valid && g.gl == 0 && und && !hit);
    if (undecided && g.lane == 0 && left) atomicAdd(undecided, (int)__popcll(left));
}

// C = A + B with a lane group of G lanes per row.  An entry of A with column c
// lands at (its index in A's row) + (entries of B's row below c) - (columns
// below c present in both), found by binary search in the other row and a
// group prefix count of the shared columns; entries of B present in A are
// added to A's value (a + b), the others placed the same way.
__device__ inline int lower_bound_int(const int* __restrict__ a, int len, int key) {
    int lo = 0, hi = len;
    while (lo < hi) {
        int mid = (lo + hi) >> 1;
        if (a[mid] < key) lo = mid + 1;
        else hi = mid;
    }
    return lo;
}

template <int G, bool FILL>
__global__ __launch_bounds__(TPB) void k_add_g(int nr, const int* __restrict__ arp, const int* __restrict__ aci,
                                               const double* __restrict__ av, const int* __restrict__ brp,
                                               const int* __restrict__ bci, const double* __restrict__ bv,
                                               const int* __restrict__ crp, int* __restrict__ cci,
                                               double* __restrict__ cv, int* __restrict__ cnt) {
    Grp<G> g;
    const int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    const bool valid = i < nr;
    int a0 = 0, la = 0, b0 = 0, lb = 0, o = 0;
    if (valid) {
        a0 = arp[i];
        la = arp[i + 1] - a0;
        b0 = brp[i];
        lb = brp[i + 1] - b0;
        if (FILL) o = crp[i];
    }
    const int wla = wave_max_int(la), wlb = wave_max_int(lb);
    int mA = 0;
    for (int base = 0; base < wla; base += G) {
        const int ia = base + g.gl;
        const bool act = ia < la;
        int ca = 0, rb = 0;
        bool eq = false;
        if (act) {
            ca = aci[a0 + ia];
            rb = lower_bound_int(bci + b0, lb, ca);
            eq = rb < lb && bci[b0 + rb] == ca;
        }
        const unsigned long long bits = g.bits(eq);
        if (FILL && act) {
            int pos = o + ia + rb - (mA + g.below(bits));
            cci[pos] = ca;
            cv[pos] = eq ? av[a0 + ia] + bv[b0 + rb] : av[a0 + ia];
        }
        mA += __popcll(bits);
    }
    if (!FILL) {
        if (valid && g.gl == 0) cnt[i] = la + lb - mA;
        return;
    }
    int mB = 0;
    for (int base = 0; base < wlb; base += G) {
        const int jb = base + g.gl;
        const bool act = jb < lb;
        int cb = 0, ra = 0;
        bool eq = false;
        if (act) {
            cb = bci[b0 + jb];
            ra = lower_bound_int(aci + a0, la, cb);
            eq = ra < la && aci[a0 + ra] == cb;
        }
        const unsigned long long bits = g.bits(eq);
        if (act && !eq) {
            int pos = o + jb + ra - (mB + g.below(bits));
            cci[pos] = cb;
            cv[pos] = bv[b0 + jb];
        }
        mB += __popcll(bits);
    }
}

// Numeric product with an LDS hash table per output row (a lane group of G
// lanes per row, CAP >= 2 x the row's output length known from the symbolic
// pass).  The entries of the row of A are taken one after another; for each,
// the lanes insert the distinct columns of the matching row of B (linear
// probing with an LDS compare-and-swap) and add a_ip * b_pj to the slot, so
// every output value starts at 0.0 and adds its products in the order of A's
// entries (Gustavson's order, as the merge).  The filled slots are then
// gathered and written in column order by rank.
constexpr int log2_pow2(int v) { return v <= 1 ? 0 : 1 + log2_pow2(v / 2); }

template <int G, int CAP, bool FILL, bool ADD>
__global__ __launch_bounds__(TPB) void k_spgemm_hash(int nr, const int* __restrict__ arp,
                                                     const int* __restrict__ aci, const double* __restrict__ av,
                                                     const int* __restrict__ brp, const int* __restrict__ bci,
                                                     const double* __restrict__ bv, const int* __restrict__ drp,
                                                     const int* __restrict__ dci, const double* __restrict__ dv,
                                                     const int* __restrict__ crp, int* __restrict__ cci,
                                                     double* __restrict__ cv, int* __restrict__ cnt,
                                                     int* __restrict__ flag, int lo, int hi, double sgn,
                                                     const int* __restrict__ brep) {
    constexpr int NG = TPB / G;
    constexpr int PER = CAP / G;
    __shared__ int keys[NG][CAP];
    __shared__ double vals[NG][FILL ? CAP : 1];
    Grp<G> g;
    const int grp = threadIdx.x / G;
    const int row = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    bool valid = row < nr;
    if (FILL && valid) {
        // this launch takes the rows of C with lo < length <= hi
        const int cl = crp[row + 1] - crp[row];
        valid = cl > lo && cl <= hi;
    }
    int* K = keys[grp];
    double* Vs = vals[grp];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        K[g.gl + G * u] = -1;
        if (FILL) Vs[g.gl + G * u] = 0.0;
    }
    int a0 = 0, a1 = 0;
    if (valid) {
        a0 = arp[row];
        a1 = arp[row + 1];
    }
    const int wl = wave_max_int(a1 - a0);
    if (ADD && valid && a1 == a0) {
        // no products (e.g. a C row away from every well): the row of C is the
        // row of D, already in column order; the group leaves together (only
        // group-local shuffles follow)
        const int d0 = drp[row], d1 = drp[row + 1];
        if (!FILL) {
            if (g.gl == 0) cnt[row] = d1 - d0;
        } else {
            const int o = crp[row] - d0;
            for (int q = d0 + g.gl; q < d1; q += G) {
                cci[o + q] = dci[q];
                cv[o + q] = dv[q];
            }
        }
        return;
    }
    // numeric pass with brep: the slot this lane's first column went to in
    // the previous entry of A (the same column when both select rows of B of
    // one pattern)
    int hprev = -1;
    for (int base = 0; base < wl; base += G) {
        // lane t holds entry base + t of the row of A
        int kb0 = 0, kb1 = 0;
        double ka = 0.0;
        bool same = false;
        if (a0 + base + g.gl < a1) {
            const int q = a0 + base + g.gl;
            int k = aci[q];
            // with brep, rows of B with equal brep have equal patterns: an
            // entry whose predecessor in A's row selects such a row adds no
            // column (the symbolic pass takes an empty row of B instead; the
            // numeric pass finds its slots where the predecessor put them)
            same = brep && q > a0 && brep[aci[q - 1]] == brep[k];
            if (FILL || !same) {
                kb0 = brp[k];
                kb1 = brp[k + 1];
            }
            if (FILL) ka = av[q];
        }
        const int lim = min(G, wl - base);   // the same for the whole wavefront
        // The first G entries of the rows of B that the next D entries of A
        // select are loaded together (independent loads, one memory latency),
        // then inserted one row after another, in the order of A's entries.
        // Tables of 64 slots or more already limit the occupancy through LDS,
        // so eight rows of B in registers cost nothing there; small tables
        // take four.
        constexpr int D = CAP >= 64 ? (G < 8 ? G : 8) : (G < 4 ? G : 4);
        for (int t0 = 0; t0 < lim; t0 += D) {
            int hj[D];
            double hv[D];
#pragma unroll
            for (int d = 0; d < D; ++d) {
                const int b0 = __shfl(kb0, g.gbase + t0 + d, WAVE), b1 = __shfl(kb1, g.gbase + t0 + d, WAVE);
                const bool in = t0 + d < lim && b0 + g.gl < b1;
                hj[d] = in ? bci[b0 + g.gl] : -1;
                hv[d] = (FILL && in) ? bv[b0 + g.gl] : 0.0;
            }
#pragma unroll
            for (int d = 0; d < D; ++d) {
                if (t0 + d >= lim) break;
                const int b0 = __shfl(kb0, g.gbase + t0 + d, WAVE), b1 = __shfl(kb1, g.gbase + t0 + d, WAVE);
                const double a = __shfl(ka, g.gbase + t0 + d, WAVE);
                const bool sd = FILL && brep && __shfl((int)same, g.gbase + t0 + d, WAVE) != 0;
                for (int q = b0 + g.gl; q < b1; q += G) {
                    const bool first = q == b0 + g.gl;
                    const int j = first ? hj[d] : bci[q];
                    const double prod = FILL ? a * (first ? hv[d] : bv[q]) : 0.0;
                    int h;
                    if (first && sd && hprev >= 0) {
                        h = hprev;
                    } else {
                        // multiplicative hash: the top log2(CAP) bits of j * 2654435761
                        h = (int)(((unsigned)j * 2654435761u) >> (32 - log2_pow2(CAP)));
                        int probes = 0;
                        for (;;) {
                            int old = atomicCAS(&K[h], -1, j);
                            if (old == -1 || old == j) break;
                            h = (h + 1) & (CAP - 1);
                            if (++probes == CAP) { atomicMax(flag, FILL ? 1 : 2); h = -1; break; }
                        }
                    }
                    if (FILL && h >= 0) Vs[h] = Vs[h] + prod;
                    if (first) hprev = h;
                }
                if (FILL && brep && b0 + g.gl >= b1) hprev = -1;
            }
        }
    }
    if (ADD && valid) {
        // C = D + A B: the entries of D's row join the table after every
        // product, so a shared entry is d + (its Gustavson sum), as in a
        // separate sparse add of the finished product; a D-only entry is d
        for (int q = drp[row] + g.gl; q < drp[row + 1]; q += G) {
            const int j = dci[q];
            int h = (int)(((unsigned)j * 2654435761u) >> (32 - log2_pow2(CAP)));
            int probes = 0;
            int old;
            for (;;) {
                old = atomicCAS(&K[h], -1, j);
                if (old == -1 || old == j) break;
                h = (h + 1) & (CAP - 1);
                if (++probes == CAP) { atomicMax(flag, FILL ? 1 : 2); h = -1; break; }
            }
            if (FILL && h >= 0) Vs[h] = (old == -1) ? dv[q] : dv[q] + Vs[h];
        }
    }
    if (!FILL) {
        int mine = 0;
#pragma unroll
        for (int u = 0; u < PER; ++u) mine += (K[g.gl + G * u] >= 0) ? 1 : 0;
        mine = g.sum(mine);
        if (valid && g.gl == 0) cnt[row] = mine;
        return;
    }
    // gather this lane's filled slots, place them after those of the lanes before it
    int kk[PER];
    double vv[PER];
    int mine = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        kk[u] = K[g.gl + G * u];
        vv[u] = Vs[g.gl + G * u];
        mine += (kk[u] >= 0) ? 1 : 0;
    }
    int incl = mine;
    for (int off = 1; off < G; off <<= 1) {
        int t = __shfl_up(incl, off, G);
        if (g.gl >= off) incl += t;
    }
    const int L = __shfl(incl, g.gbase + G - 1, WAVE);
    int pos = incl - mine;
#pragma unroll
    for (int u = 0; u < PER; ++u)
        if (kk[u] >= 0) {
            K[pos] = kk[u];
            Vs[pos] = vv[u];
            ++pos;
        }
    // rank = number of smaller columns among the L gathered entries
    if (valid) {
        const int o = crp[row];
        for (int e = g.gl; e < L; e += G) {
            const int key = K[e];
            int rank = 0;
            for (int f = 0; f < L; ++f) rank += (K[f] < key) ? 1 : 0;
            cci[o + rank] = key;
            cv[o + rank] = sgn * Vs[e];
        }
    }
}

// Products with the block-diagonal F-relaxation operator M, whose blocks of at
// most four F-points store, in every row, the block's columns in order (a
// larger, failed block keeps one diagonal entry per row).  M's layout is
// known: row s0 + r of a block of bs <= 4 rows starts at mrp[s0] + r bs and
// holds columns s0 .. s0 + bs - 1; a failed block's row holds its diagonal.
//
// Symbolic pass of M B (P_F = -M A_FC), G lanes per block: every row of a
// block has the same pattern, the union of B's rows s0 .. s0 + bs - 1, formed
// once in an LDS hash table.  A failed block's rows are taken one by one.
// At most BDL_STAGE entries of B per block.
constexpr int BDL_STAGE = 64, BDL_CAP = 128;

template <int G>
__global__ __launch_bounds__(TPB) void k_bdiag_left_count(int nb, const int* __restrict__ bstart,
                                                          const int* __restrict__ brp, const int* __restrict__ bci,
                                                          int* __restrict__ cnt, int* __restrict__ flag) {
    constexpr int NG = TPB / G, PER = BDL_CAP / G;
    __shared__ int keys[NG][BDL_CAP];
    Grp<G> g;
    const int grp = threadIdx.x / G;
    const int b = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    int s0 = 0, bs = 0;
    if (b < nb) {
        s0 = bstart[b];
        bs = bstart[b + 1] - s0;
    }
    const bool whole = bs <= 4;
    const int nsets = whole ? (bs > 0 ? 1 : 0) : bs;
    const int nsub = wave_max_int(nsets);
    int* K = keys[grp];
    for (int sub = 0; sub < nsub; ++sub) {
        const bool act = sub < nsets;
        const int r0 = whole ? s0 : s0 + sub, nrow = whole ? bs : 1, nk = act ? nrow : 0;
        int rb[5];
#pragma unroll
        for (int t = 0; t < 5; ++t) rb[t] = (act && t <= nk) ? brp[r0 + t] : 0;
        int bk0[4] = {0, 0, 0, 0}, bkl[4] = {0, 0, 0, 0};
#pragma unroll
        for (int t = 0; t < 4; ++t)
            if (t < nk) {
                bk0[t] = rb[t];
                bkl[t] = rb[t + 1] - rb[t];
            }
        int total = bkl[0] + bkl[1] + bkl[2] + bkl[3];
        if (total > BDL_STAGE) {
            if (g.gl == 0) atomicMax(flag, 1);
            total = 0;
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) K[g.gl + G * u] = -1;
        __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup");
        __builtin_amdgcn_wave_barrier();
        for (int e = g.gl; e < total; e += G) {
            // entry e of the concatenated rows: row t, position q
            int q = e, t = 0, base = bk0[0];
#pragma unroll
            for (int u = 0; u < 3; ++u) {
                const bool adv = t == u && q >= bkl[u];
                q = adv ? q - bkl[u] : q;
                base = adv ? bk0[u + 1] : base;
                t = adv ? u + 1 : t;
            }
            const int j = bci[base + q];
            // at most BDL_STAGE distinct keys in BDL_CAP slots: a slot is found
            int h = (int)(((unsigned)j * 2654435761u) >> (32 - log2_pow2(BDL_CAP)));
            for (int probes = 0; probes < BDL_CAP; ++probes) {
                const int old = atomicCAS(&K[h], -1, j);
                if (old == -1 || old == j) break;
                h = (h + 1) & (BDL_CAP - 1);
            }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
        int mine = 0;
#pragma unroll
        for (int u = 0; u < PER; ++u) mine += K[g.gl + G * u] >= 0 ? 1 : 0;
        const int L = g.sum(mine);
        if (act)
            for (int r = g.gl; r < nrow; r += G) cnt[r0 + r] = L;
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "workgroup");
        __builtin_amdgcn_wave_barrier();
    }
}

// C = A M with M on the right (W = A_CF M), 32 lanes per row of A (rows of at
// most 32 entries, columns ascending): lane e holds entry e.  A block's columns
// are a range of indices, so its entries in the row are consecutive: a run of
// entries whose M rows start at the same column and have the same length.  A
// run contributes exactly its block's columns, and the run's first lane sums
// the run's products for each of them in entry order (M's rows hold
// consecutive columns, the first of them the block's).  A group takes BDR_ROWS
// consecutive rows, with the loads of all of them issued before any is used.
constexpr int BDR_ROWS = 4;

template <bool FILL>
__global__ __launch_bounds__(TPB) void k_bdiag_right(int nr, const int* __restrict__ arp,
                                                     const int* __restrict__ aci, const double* __restrict__ av,
                                                     const int* __restrict__ mrp, const int* __restrict__ mci,
                                                     const double* __restrict__ mv, const int* __restrict__ crp,
                                                     int* __restrict__ cci, double* __restrict__ cv,
                                                     int* __restrict__ cnt, int* __restrict__ flag) {
    constexpr int G = 32, R = BDR_ROWS;
    Grp<G> g;
    const int row0 = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G) * R;
    int rpv[R + 1];
#pragma unroll
    for (int r = 0; r <= R; ++r) rpv[r] = row0 + r <= nr ? arp[row0 + r] : 0;
    int len[R], k[R], m0[R], ml[R], first[R];
    double a[R], mvv[R][4];
#pragma unroll
    for (int r = 0; r < R; ++r) {
        len[r] = row0 + r < nr ? rpv[r + 1] - rpv[r] : 0;
        if (len[r] > G) {
            if (g.gl == 0) atomicMax(flag, 1);
            len[r] = 0;
        }
        k[r] = g.gl < len[r] ? aci[rpv[r] + g.gl] : -1;
        if (FILL) a[r] = g.gl < len[r] ? av[rpv[r] + g.gl] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        m0[r] = k[r] >= 0 ? mrp[k[r]] : 0;
        ml[r] = k[r] >= 0 ? min(mrp[k[r] + 1] - m0[r], 4) : 0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        first[r] = k[r] >= 0 ? mci[m0[r]] : -1;
        if (FILL)
#pragma unroll
            for (int t = 0; t < 4; ++t) mvv[r][t] = t < ml[r] ? mv[m0[r] + t] : 0.0;
    }
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const bool act = k[r] >= 0;
        const int pk = __shfl_up(k[r], 1, G), pf = __shfl_up(first[r], 1, G), pl = __shfl_up(ml[r], 1, G);
        if (act && g.gl > 0 && pk >= k[r]) atomicMax(flag, 1);   // columns not ascending
        const bool head = act && (g.gl == 0 || pf != first[r] || pl != ml[r]);
        const int contrib = head ? ml[r] : 0;
        int incl = contrib;
        for (int off = 1; off < G; off <<= 1) {
            const int tt = __shfl_up(incl, off, G);
            if (g.gl >= off) incl += tt;
        }
        if (!FILL) {
            const int tot = __shfl(incl, g.gbase + G - 1, WAVE);
            if (row0 + r < nr && g.gl == 0) cnt[row0 + r] = tot;
            continue;
        }
        double p[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) p[t] = a[r] * mvv[r][t];
        // the run ends at the next head (or the row's end)
        const unsigned long long later = g.bits(head) & ~((2ULL << g.gl) - 1ULL);
        const int runlen = later ? __ffsll((long long)later) - 1 - g.gl : len[r] - g.gl;
        double acc[4];
#pragma unroll
        for (int t = 0; t < 4; ++t) acc[t] = 0.0 + p[t];
#pragma unroll
        for (int u = 1; u < 4; ++u) {
            const int src = g.gbase + min(g.gl + u, G - 1);
#pragma unroll
            for (int t = 0; t < 4; ++t) {
                const double q = __shfl(p[t], src, WAVE);
                if (u < runlen) acc[t] = acc[t] + q;
            }
        }
        if (head) {
            const int o = crp[row0 + r] + incl - contrib;
#pragma unroll
            for (int t = 0; t < 4; ++t)
                if (t < ml[r]) {
                    cci[o + t] = first[r] + t;
                    cv[o + t] = acc[t];
                }
        }
    }
}

// Symbolic pass of C = A B (ADD: C = D + A B) with a lane per entry of a row
// of A, for rows of A long against those of B (A P in the AMG levels), where
// the hashed kernel above would take the row's entries one after another.
// 32 lanes per row take its entries 32 at a time; each lane walks the row of
// B its entry selects and inserts the columns into the row's LDS hash table
// (CAS linear probing) in any order: the keys are the output pattern, the
// count their number.  A full table sets flag[0] to 2.  (A numeric pass built
// the same way -- each slot's products chained and summed in Gustavson order
// -- measured twice as slow as the hashed fill, which walks A's entries in
// order; the fill stays with that kernel.)
template <int CAP, bool ADD>
__global__ __launch_bounds__(TPB) void k_spgemm_lanes_count(int nr, const int* __restrict__ arp,
                                                            const int* __restrict__ aci,
                                                            const int* __restrict__ brp,
                                                            const int* __restrict__ bci,
                                                            const int* __restrict__ drp,
                                                            const int* __restrict__ dci, int* __restrict__ cnt,
                                                            int* __restrict__ flag) {
    constexpr int G = 32, NG = TPB / G, PER = CAP / G;
    __shared__ int keys[NG][CAP];
    Grp<G> g;
    const int grp = threadIdx.x / G;
    const int row = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    const bool valid = row < nr;
    int* K = keys[grp];
#pragma unroll
    for (int u = 0; u < PER; ++u) K[g.gl + G * u] = -1;
    __syncthreads();
    int a0 = 0, a1 = 0;
    if (valid) {
        a0 = arp[row];
        a1 = arp[row + 1];
    }
    const int wl = wave_max_int(a1 - a0);
    auto insert = [&](int j) {
        int h = (int)(((unsigned)j * 2654435761u) >> (32 - log2_pow2(CAP)));
        for (int probes = 0;; ++probes) {
            const int old = atomicCAS(&K[h], -1, j);
            if (old == -1 || old == j) return;
            if (probes + 1 == CAP) {
                atomicMax(flag, 2);
                return;
            }
            h = (h + 1) & (CAP - 1);
        }
    };
    for (int base = 0; base < wl; base += G) {
        const int e = a0 + base + g.gl;
        if (e < a1) {
            const int k = aci[e];
            const int b0 = brp[k], b1 = brp[k + 1];
            for (int q = b0; q < b1; ++q) insert(bci[q]);
        }
    }
    if (ADD && valid)
        for (int q = drp[row] + g.gl; q < drp[row + 1]; q += G) insert(dci[q]);
    __syncthreads();
    int mine = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) mine += K[g.gl + G * u] >= 0 ? 1 : 0;
    mine = g.sum(mine);
    if (valid && g.gl == 0) cnt[row] = mine;
}

// Block extraction (Sec. 2, the partition of eq. (2)): each row i goes to
// A_FF / A_FC (F rows) or A_CF / A_CC (C rows) with local numbering lmap.
// With fblk (the F-relaxation block of each F-point), an F row keeps in A_FF
// only the columns of its own block: the part of A_FF that M is formed from
// (the one-sweep apply never reads the rest).  A null output array skips that
// output (the count stays to be written).
// Both kernels issue the index loads of EX_BATCH chunks of G entries, then
// the flag gathers of all of them, before using any (rows of up to
// EX_BATCH * G entries in one round of dependent loads).
constexpr int EX_BATCH = 4;

template <int G>
__global__ __launch_bounds__(TPB) void k_extract_count_g(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                         const int* __restrict__ isF, const int* __restrict__ lmap,
                                                         const int* __restrict__ fblk, int* cFF, int* cFC, int* cCF,
                                                         int* cCC) {
    Grp<G> g;
    int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    int f = 0, c = 0;
    if (i < n) {
        const bool rowF = isF[i] != 0;
        const int fi = (rowF && fblk) ? fblk[lmap[i]] : -1;
        const int pe = rp[i + 1];
        for (int p = rp[i] + g.gl; p < pe; p += G * EX_BATCH) {
            int jj[EX_BATCH], fl[EX_BATCH];
#pragma unroll
            for (int u = 0; u < EX_BATCH; ++u) jj[u] = p + u * G < pe ? ci[p + u * G] : -1;
#pragma unroll
            for (int u = 0; u < EX_BATCH; ++u) fl[u] = jj[u] >= 0 ? isF[jj[u]] : 0;
#pragma unroll
            for (int u = 0; u < EX_BATCH; ++u) {
                if (jj[u] < 0) continue;
                if (fl[u]) f += (fi < 0 || fblk[lmap[jj[u]]] == fi) ? 1 : 0;
                else ++c;
            }
        }
    }
    f = g.sum(f);
    c = g.sum(c);
    if (i < n && g.gl == 0) {
        int l = lmap[i];
        if (isF[i]) { if (cFF) cFF[l] = f; if (cFC) cFC[l] = c; }
        else { if (cCF) cCF[l] = f; if (cCC) cCC[l] = c; }
    }
}

template <int G>
__global__ __launch_bounds__(TPB) void k_extract_fill_g(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                        const double* __restrict__ v, const int* __restrict__ isF,
                                                        const int* __restrict__ lmap, const int* __restrict__ fblk,
                                                        const int* __restrict__ rpFF,
                                                        int* ciFF, double* vFF, const int* __restrict__ rpFC,
                                                        int* ciFC, double* vFC, const int* __restrict__ rpCF,
                                                        int* ciCF, double* vCF, const int* __restrict__ rpCC,
                                                        int* ciCC, double* vCC) {
    Grp<G> g;
    int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    bool valid = i < n;
    int p0 = valid ? rp[i] : 0, len = valid ? rp[i + 1] - p0 : 0;
    int maxlen = wave_max_int(len);
    int oF = 0, oC = 0, fi = -1;
    int *cF = nullptr, *cC = nullptr;
    double *vF = nullptr, *vC = nullptr;
    if (valid) {
        int l = lmap[i];
        if (isF[i]) {
            if (ciFF) { oF = rpFF[l]; cF = ciFF; vF = vFF; }
            if (ciFC) { oC = rpFC[l]; cC = ciFC; vC = vFC; }
            if (fblk) fi = fblk[l];
        } else {
            if (ciCF) { oF = rpCF[l]; cF = ciCF; vF = vCF; }
            if (ciCC) { oC = rpCC[l]; cC = ciCC; vC = vCC; }
        }
    }
    for (int base = 0; base < maxlen; base += G * EX_BATCH) {
        int jj[EX_BATCH], fl[EX_BATCH], lj[EX_BATCH];
        double vv[EX_BATCH];
#pragma unroll
        for (int u = 0; u < EX_BATCH; ++u) {
            const int q = base + u * G + g.gl;
            jj[u] = q < len ? ci[p0 + q] : -1;
            vv[u] = q < len ? v[p0 + q] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < EX_BATCH; ++u) {
            fl[u] = jj[u] >= 0 ? isF[jj[u]] : 0;
            lj[u] = jj[u] >= 0 ? lmap[jj[u]] : 0;
        }
#pragma unroll
        for (int u = 0; u < EX_BATCH; ++u) {
            const bool act = jj[u] >= 0;
            const bool f = act && fl[u] && (fi < 0 || fblk[lj[u]] == fi);
            const bool c = act && !fl[u];
            const unsigned long long bf = g.bits(f), bc = g.bits(c);
            if (f && cF) { int o = oF + g.below(bf); cF[o] = lj[u]; vF[o] = vv[u]; }
            if (c && cC) { int o = oC + g.below(bc); cC[o] = lj[u]; vC[o] = vv[u]; }
            oF += __popcll(bf);
            oC += __popcll(bc);
        }
    }
}

// The same extraction straight from the block-CSR input (b = B): G lanes per
// scalar row i = I B + r, one block of the block row per lane at a time (row r
// of its B x B values in one contiguous load, the F flags of its B columns
// together).  The B groups of one block row sit in the same wavefront, so each
// block's values come from memory once.  Entry (r, c) of block (I, J) is entry
// (I B + r, J B + c) of the scalar operator unless it is an exact zero off the
// diagonal (the scalar operator of the input leaves those out).  Lanes hold
// consecutive blocks, so the per-lane counts scanned in lane order place the
// entries in column order.  (A group per block row, holding whole blocks, took
// 114 registers and half the occupancy.)  With vcopy, the values read are also
// stored there (the library's copy of the input, made in the same pass).
template <int B>
struct BsrRowPart {
    double a[B];    // row r of the block
    bool cf[B];     // column J B + c is an F-point
    int cl[B];      // its local index
    unsigned mf = 0, mc = 0;   // bit c: a kept F entry (in A_FF's block when ffb >= 0) / a kept C entry
    __device__ void load(int p, int I, int r, int ffb, const int* __restrict__ bci, const double* __restrict__ bv,
                         const int* __restrict__ isF, const int* __restrict__ lmap, const int* __restrict__ fblk,
                         double* __restrict__ vcopy) {
        const int J = bci[p];
        const double* src = bv + ((long)p * B + r) * B;
#pragma unroll
        for (int c = 0; c < B; ++c) a[c] = src[c];
        if (vcopy)
#pragma unroll
            for (int c = 0; c < B; ++c) vcopy[((long)p * B + r) * B + c] = a[c];
#pragma unroll
        for (int c = 0; c < B; ++c) {
            cf[c] = isF[J * B + c] != 0;
            cl[c] = lmap[J * B + c];
        }
        int fb[B];
#pragma unroll
        for (int c = 0; c < B; ++c) fb[c] = (ffb >= 0 && cf[c]) ? fblk[cl[c]] : -1;
#pragma unroll
        for (int c = 0; c < B; ++c) {
            const bool keep = a[c] != 0.0 || (J == I && c == r);
            const bool inb = ffb < 0 || fb[c] == ffb;
            mf |= (keep && cf[c] && inb) ? 1u << c : 0u;
            mc |= (keep && !cf[c]) ? 1u << c : 0u;
        }
    }
};

template <int G>
__device__ inline int group_scan_incl(int v, int gl) {
#pragma unroll
    for (int off = 1; off < G; off <<= 1) {
        const int t = __shfl_up(v, off, G);
        if (gl >= off) v += t;
    }
    return v;
}

// The symbolic pass keeps a group per block row (whole blocks per lane, the
// counts of the B rows together): it holds fewer registers than the numeric
// pass, and a quarter of the wavefronts of a group per scalar row ran faster.
template <int B>
struct BsrBlock {
    double a[B][B];
    int J;
    bool cf[B];     // column J B + c is an F-point
    int cl[B];      // its local index
    int fb[B];      // its F-relaxation block (with fblk; else -1)
    __device__ void load(int p, const int* __restrict__ bci, const double* __restrict__ bv,
                         const int* __restrict__ isF, const int* __restrict__ lmap, const int* __restrict__ fblk) {
        J = bci[p];
        const double* src = bv + (long)p * B * B;
#pragma unroll
        for (int r = 0; r < B; ++r)
#pragma unroll
            for (int c = 0; c < B; ++c) a[r][c] = src[r * B + c];
#pragma unroll
        for (int c = 0; c < B; ++c) {
            cf[c] = isF[J * B + c] != 0;
            cl[c] = lmap[J * B + c];
        }
#pragma unroll
        for (int c = 0; c < B; ++c) fb[c] = (fblk && cf[c]) ? fblk[cl[c]] : -1;
    }
    // kept F entries of row r (in A_FF's block when ffb >= 0) and kept C entries
    __device__ void row_counts(int I, int r, int ffb, int& nf, int& nc) const {
        nf = 0;
        nc = 0;
#pragma unroll
        for (int c = 0; c < B; ++c) {
            const bool keep = a[r][c] != 0.0 || (J == I && c == r);
            const bool inb = ffb < 0 || fb[c] == ffb;
            nf += (keep && cf[c] && inb) ? 1 : 0;
            nc += (keep && !cf[c]) ? 1 : 0;
        }
    }
};

template <int G, int B>
__global__ __launch_bounds__(TPB) void k_bsr_extract_count_g(int nbr, const int* __restrict__ brp,
                                                             const int* __restrict__ bci, const double* __restrict__ bv,
                                                             const int* __restrict__ isF, const int* __restrict__ lmap,
                                                             const int* __restrict__ fblk, int* cFF, int* cFC,
                                                             int* cCF, int* cCC) {
    Grp<G> g;
    const int I = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    const bool valid = I < nbr;
    int ffb[B], nf[B], nc[B];
#pragma unroll
    for (int r = 0; r < B; ++r) {
        nf[r] = nc[r] = 0;
        ffb[r] = (valid && fblk && isF[I * B + r]) ? fblk[lmap[I * B + r]] : -1;
    }
    if (valid) {
        BsrBlock<B> k;
        for (int p = brp[I] + g.gl; p < brp[I + 1]; p += G) {
            k.load(p, bci, bv, isF, lmap, fblk);
#pragma unroll
            for (int r = 0; r < B; ++r) {
                int f, c;
                k.row_counts(I, r, ffb[r], f, c);
                nf[r] += f;
                nc[r] += c;
            }
        }
    }
#pragma unroll
    for (int r = 0; r < B; ++r) {
        nf[r] = g.sum(nf[r]);
        nc[r] = g.sum(nc[r]);
    }
    if (valid && g.gl == 0) {
#pragma unroll
        for (int r = 0; r < B; ++r) {
            const int i = I * B + r, l = lmap[i];
            if (isF[i]) { if (cFF) cFF[l] = nf[r]; if (cFC) cFC[l] = nc[r]; }
            else { if (cCF) cCF[l] = nf[r]; if (cCC) cCC[l] = nc[r]; }
        }
    }
}

template <int G, int B>
__global__ __launch_bounds__(TPB) void k_bsr_extract_fill_g(int nbr, const int* __restrict__ brp,
                                                            const int* __restrict__ bci, const double* __restrict__ bv,
                                                            const int* __restrict__ isF, const int* __restrict__ lmap,
                                                            const int* __restrict__ fblk,
                                                            const int* __restrict__ rpFF, int* ciFF, double* vFF,
                                                            const int* __restrict__ rpFC, int* ciFC, double* vFC,
                                                            const int* __restrict__ rpCF, int* ciCF, double* vCF,
                                                            const int* __restrict__ rpCC, int* ciCC, double* vCC,
                                                            double* __restrict__ vcopy) {
    Grp<G> g;
    const int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    const bool valid = i < nbr * B;
    const int I = i / B, r = i - I * B;
    const int p0 = valid ? brp[I] : 0, nb = valid ? brp[I + 1] - p0 : 0;
    const int maxnb = wave_max_int(nb);
    int oF = 0, oC = 0, ffb = -1;
    int* cF = nullptr;
    int* cC = nullptr;
    double* vF = nullptr;
    double* vC = nullptr;
    if (valid) {
        const int l = lmap[i];
        if (isF[i]) {
            if (ciFF) { oF = rpFF[l]; cF = ciFF; vF = vFF; }
            if (ciFC) { oC = rpFC[l]; cC = ciFC; vC = vFC; }
            if (fblk) ffb = fblk[l];
        } else {
            if (ciCF) { oF = rpCF[l]; cF = ciCF; vF = vCF; }
            if (ciCC) { oC = rpCC[l]; cC = ciCC; vC = vCC; }
        }
    }
    for (int base = 0; base < maxnb; base += G) {
        const int q = base + g.gl;
        BsrRowPart<B> k;
        if (q < nb) k.load(p0 + q, I, r, ffb, bci, bv, isF, lmap, fblk, vcopy);
        const int f = __popc(k.mf), c = __popc(k.mc);
        const int fi = group_scan_incl<G>(f, g.gl), ci = group_scan_incl<G>(c, g.gl);
        int wf = oF + fi - f, wc = oC + ci - c;
#pragma unroll
        for (int cc = 0; cc < B; ++cc) {
            const bool tf = (k.mf >> cc) & 1u, tc = (k.mc >> cc) & 1u;
            if (tf && cF) { cF[wf] = k.cl[cc]; vF[wf] = k.a[cc]; }
            if (tc && cC) { cC[wc] = k.cl[cc]; vC[wc] = k.a[cc]; }
            wf += tf ? 1 : 0;
            wc += tc ? 1 : 0;
        }
        oF += __shfl(fi, g.gbase + G - 1, WAVE);
        oC += __shfl(ci, g.gbase + G - 1, WAVE);
    }
}

// scalar row i = I*b + r of a block row: G lanes take the row's blocks
// Scalar CSR of the block-CSR input without the exact zeros inside blocks
// (the diagonal is always kept): per scalar row, a count pass, then a fill pass
// in which each lane takes one block and places its kept entries after those of
// the lanes before it (a segmented prefix sum over the group).
template <int G>
__global__ __launch_bounds__(TPB) void k_bsr_count_g(int b, int nbr, const int* __restrict__ brp,
                                                     const int* __restrict__ bci, const double* __restrict__ bv,
                                                     int* __restrict__ cnt) {
    Grp<G> g;
    const int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    const int n = nbr * b;
    int k = 0;
    if (i < n) {
        const int I = i / b, r = i - I * b;
        for (int p = brp[I] + g.gl; p < brp[I + 1]; p += G) {
            const int J = bci[p];
            const double* blk = bv + (long)p * b * b + r * b;
            for (int c = 0; c < b; ++c) k += (blk[c] != 0.0 || J * b + c == i) ? 1 : 0;
        }
    }
    k = g.sum(k);
    if (i < n && g.gl == 0) cnt[i] = k;
}

template <int G>
__global__ __launch_bounds__(TPB) void k_bsr_fill_g(int b, int nbr, const int* __restrict__ brp,
                                                    const int* __restrict__ bci, const double* __restrict__ bv,
                                                    const int* __restrict__ rp, int* __restrict__ ci,
                                                    double* __restrict__ v) {
    Grp<G> g;
    const int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    const int n = nbr * b;
    const bool valid = i < n;
    int p0 = 0, p1 = 0, o = 0, I = 0, r = 0;
    if (valid) {
        I = i / b;
        r = i - I * b;
        p0 = brp[I];
        p1 = brp[I + 1];
        o = rp[i];
    }
    const int wl = wave_max_int(p1 - p0);
    for (int base = 0; base < wl; base += G) {
        const int p = p0 + base + g.gl;
        const bool act = valid && p < p1;
        int J = 0, keep = 0;
        const double* blk = bv;
        if (act) {
            J = bci[p];
            blk = bv + (long)p * b * b + r * b;
            for (int c = 0; c < b; ++c) keep += (blk[c] != 0.0 || J * b + c == i) ? 1 : 0;
        }
        int incl = keep;
        for (int off = 1; off < G; off <<= 1) {
            int t = __shfl_up(incl, off, G);
            if (g.gl >= off) incl += t;
        }
        if (act) {
            int q = o + incl - keep;
            for (int c = 0; c < b; ++c)
                if (blk[c] != 0.0 || J * b + c == i) {
                    ci[q] = J * b + c;
                    v[q] = blk[c];
                    ++q;
                }
        }
        o += __shfl(incl, g.gbase + G - 1, WAVE);
    }
}

// Strength of connection per entry, the number of strong entries of each row
// (scnt) and, by atomic increments, the number of rows that strongly depend
// on each column (lam, which must start at zero); with dinv, also the L1
// Jacobi diagonal 1 / (a_ii + sum_{j != i} |a_ij|) as l1_dinv forms it.
template <int G>
__global__ __launch_bounds__(TPB) void k_strength_g(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                    const double* __restrict__ v, double theta,
                                                    const int* __restrict__ label, unsigned char* __restrict__ strong,
                                                    int* __restrict__ scnt, int* __restrict__ lam,
                                                    double* __restrict__ dinv, int* __restrict__ flag) {
    Grp<G> g;
    int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    bool valid = i < n;
    int li = (valid && label) ? label[i] : 0;
    double mx = 0.0, sabs = 0.0, aii = 0.0;
    int have = 0;
    if (valid)
        for (int p = rp[i] + g.gl; p < rp[i + 1]; p += G) {
            int j = ci[p];
            if (j == i) aii = v[p];
            else sabs += fabs(v[p]);
            if (j == i || (label && label[j] != li)) continue;
            double t = -v[p];
            if (!have || t > mx) { mx = t; have = 1; }
        }
    if (dinv) {
        sabs = g.sumd(sabs);
        aii = g.sumd(aii);
        if (valid && g.gl == 0) {
            double d = aii + sabs;
            if (!(d > 0.0)) { set_flag(flag, 6); d = 1.0; }
            dinv[i] = 1.0 / d;
        }
    }
    for (int off = G / 2; off > 0; off >>= 1) {
        double om = __shfl_xor(mx, off, WAVE);
        int oh = __shfl_xor(have, off, WAVE);
        if (oh && (!have || om > mx)) mx = om;
        have |= oh;
    }
    int c = 0;
    if (valid) {
        double thr = theta * mx;
        for (int p = rp[i] + g.gl; p < rp[i + 1]; p += G) {
            int j = ci[p];
            unsigned char sflag = 0;
            if (have && mx > 0.0 && j != i && !(label && label[j] != li) && -v[p] >= thr) sflag = 1;
            strong[p] = sflag;
            c += sflag;
            if (sflag) atomicAdd(&lam[j], 1);
        }
    }
    c = g.sum(c);
    if (valid && g.gl == 0) scnt[i] = c;
}

template <int G>
__global__ __launch_bounds__(TPB) void k_sfill_g(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                 const unsigned char* __restrict__ strong, const int* __restrict__ srp,
                                                 int* __restrict__ sci) {
    Grp<G> g;
    int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    bool valid = i < n;
    int p0 = valid ? rp[i] : 0, len = valid ? rp[i + 1] - p0 : 0;
    int maxlen = wave_max_int(len);
    int o = valid ? srp[i] : 0;
    for (int base = 0; base < maxlen; base += G) {
        int q = base + g.gl;
        bool st = q < len && strong[p0 + q];
        unsigned long long bs = g.bits(st);
        if (st) sci[o + g.below(bs)] = ci[p0 + q];
        o += __popcll(bs);
    }
}

template <int G>
__global__ __launch_bounds__(TPB) void k_interp_count_g(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                        const unsigned char* __restrict__ strong,
                                                        const int* __restrict__ cf, int* __restrict__ cnt) {
    Grp<G> g;
    int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    bool valid = i < n;
    int c = 0;
    if (valid && cf[i] != 1)
        for (int p = rp[i] + g.gl; p < rp[i + 1]; p += G)
            if (strong[p] && cf[ci[p]] == 1) ++c;
    c = g.sum(c);
    if (valid && g.gl == 0) cnt[i] = (cf[i] == 1) ? 1 : c;
}

// Direct interpolation of one F row from its entries: kind bit 0 = diagonal,
// bit 1 = same-label off-diagonal, bit 2 = strong C neighbour (with bit 1).
// The sums run strictly left to right, as in the oracle; a term that does not
// belong to a sum is added as +0.0, which leaves it unchanged (none of the sums
// can be -0.0), and keeps the sums in registers.
struct InterpRow {
    double aii = 0.0, neg = 0.0, pos = 0.0, cs = 0.0;
    __device__ void add(int kind, double a) {
        if (kind & 1) aii = a;
        const bool off = (kind & 2) != 0;
        neg = neg + ((off && a < 0.0) ? a : 0.0);
        pos = pos + ((off && a > 0.0) ? a : 0.0);
        cs = cs + ((kind & 4) ? a : 0.0);
    }
};

// One workgroup per row block of A (the CSR-stream partition).  The block's
// values and columns are staged in LDS with coalesced loads, each entry marked
// when it is a strong C neighbour (strength already excludes the diagonal and
// other labels), whose slot then holds its P column instead, or when it has
// another label than its row; then one thread per row forms the sums and
// writes the row of P.  A block beyond the LDS
// stage is done thread per row from global memory.
constexpr int IF_LDS = 2048, IF_ROWS = 1024;
// rows longer than this on average use the lane-group kernel below instead
constexpr int INTERP_LDS_MAX_AVG = 45;
__global__ __launch_bounds__(TPB) void k_interp_fill_blk(const int* __restrict__ blk, const int* __restrict__ rp,
                                                         const int* __restrict__ ci, const double* __restrict__ v,
                                                         const unsigned char* __restrict__ strong,
                                                         const int* __restrict__ cf, const int* __restrict__ cidx,
                                                         const int* __restrict__ label, const int* __restrict__ prp,
                                                         int* __restrict__ pci, double* __restrict__ pv,
                                                         int* __restrict__ flag) {
    __shared__ double sv[IF_LDS];
    __shared__ int sc[IF_LDS];
    __shared__ unsigned char sk[IF_LDS];
    __shared__ int srp[IF_ROWS + 1];
    const int tid = threadIdx.x;
    const int r0 = blk[blockIdx.x], r1 = blk[blockIdx.x + 1];
    if (r0 >= r1) return;
    const int p0 = rp[r0], nnz = rp[r1] - p0, nrows = r1 - r0;
    const bool staged = nnz <= IF_LDS && nrows <= IF_ROWS;
    if (staged) {
        for (int t = tid; t <= nrows; t += TPB) srp[t] = rp[r0 + t] - p0;
        if (label) __syncthreads();
        for (int q = tid; q < nnz; q += TPB) {
            const int k = ci[p0 + q];
            const bool sc4 = strong[p0 + q] && cf[k] == 1;
            int mark = sc4 ? 1 : 0;
            if (label && !sc4) {
                // another label than the row's: the row is the last one that
                // starts at or before q
                int lo = 0, hi = nrows - 1;
                while (lo < hi) {
                    const int mid = (lo + hi + 1) >> 1;
                    if (srp[mid] <= q) lo = mid;
                    else hi = mid - 1;
                }
                if (label[k] != label[r0 + lo]) mark = 2;
            }
            sk[q] = (unsigned char)mark;
            sc[q] = sc4 ? cidx[k] : k;
            sv[q] = v[p0 + q];
        }
        __syncthreads();
    }
    for (int t = tid; t < nrows; t += TPB) {
        const int i = r0 + t;
        const int o0 = prp[i], o1 = prp[i + 1];
        if (cf[i] == 1) {
            pci[o0] = cidx[i];
            pv[o0] = 1.0;
            continue;
        }
        if (o1 <= o0) continue;
        const int li = label ? label[i] : 0;
        const int qb = staged ? srp[t] : rp[i] - p0, qe = staged ? srp[t + 1] : rp[i + 1] - p0;
        InterpRow s;
        for (int q = qb; q < qe; ++q) {
            bool s4;
            int k;
            double a;
            bool other;
            if (staged) { const int mk = sk[q]; s4 = mk == 1; other = mk == 2; k = sc[q]; a = sv[q]; }
            else {
                k = ci[p0 + q];
                s4 = strong[p0 + q] && cf[k] == 1;
                other = label && label[k] != li;
                a = v[p0 + q];
            }
            const int kind = s4 ? 6 : (k == i ? 1 : (other ? 0 : 2));
            s.add(kind, a);
        }
        const double atil = s.aii + s.pos, alpha = s.neg / s.cs;
        if (!(atil > 0.0)) set_flag(flag, 6);
        int o = o0;
        for (int q = qb; q < qe; ++q) {
            bool s4;
            int pc;
            double a;
            if (staged) { s4 = sk[q] == 1; pc = sc[q]; a = sv[q]; }
            else {
                const int k = ci[p0 + q];
                s4 = strong[p0 + q] && cf[k] == 1;
                pc = s4 ? cidx[k] : 0;
                a = v[p0 + q];
            }
            if (s4) {
                pci[o] = pc;
                pv[o] = -(alpha * a) / atil;
                ++o;
            }
        }
    }
}

// Direct interpolation for long rows, G lanes per row: the row sums are formed
// strictly left to right (each chunk's values are broadcast lane by lane), as
// the oracle does.
template <int G>
__global__ __launch_bounds__(TPB) void k_interp_fill_g(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                       const double* __restrict__ v,
                                                       const unsigned char* __restrict__ strong,
                                                       const int* __restrict__ cf, const int* __restrict__ cidx,
                                                       const int* __restrict__ label, const int* __restrict__ prp,
                                                       int* __restrict__ pci, double* __restrict__ pv,
                                                       int* __restrict__ flag) {
    Grp<G> g;
    int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    bool valid = i < n;
    bool frow = valid && cf[i] != 1 && prp[i + 1] > prp[i];
    if (valid && cf[i] == 1 && g.gl == 0) { pci[prp[i]] = cidx[i]; pv[prp[i]] = 1.0; }
    int p0 = valid ? rp[i] : 0, len = frow ? rp[i + 1] - p0 : 0;
    int maxlen = wave_max_int(len);
    int li = (frow && label) ? label[i] : 0;
    double aii = 0.0, neg = 0.0, pos = 0.0, cs = 0.0;
    for (int base = 0; base < maxlen; base += G) {
        int q = base + g.gl;
        bool act = q < len;
        int k = act ? ci[p0 + q] : -1;
        double a = act ? v[p0 + q] : 0.0;
        int kind = 0;  // 1 diag, 2 same-label off-diagonal, 0 other / inactive
        bool sc = false;
        if (act) {
            if (k == i) kind = 1;
            else if (!(label && label[k] != li)) {
                kind = 2;
                sc = strong[p0 + q] && cf[k] == 1;
            }
        }
        const int lim = min(G, maxlen - base);
        for (int t = 0; t < lim; ++t) {
            double at = __shfl(a, g.gbase + t, WAVE);
            int kt = __shfl(kind, g.gbase + t, WAVE);
            int st = __shfl((int)sc, g.gbase + t, WAVE);
            if (kt == 1) aii = at;
            else if (kt == 2) {
                if (at < 0.0) neg = neg + at;
                else if (at > 0.0) pos = pos + at;
                if (st) cs = cs + at;
            }
        }
    }
    double atil = aii + pos;
    if (frow && g.gl == 0 && !(atil > 0.0)) set_flag(flag, 6);
    double alpha = neg / cs;
    int o = frow ? prp[i] : 0;
    for (int base = 0; base < maxlen; base += G) {
        int q = base + g.gl;
        bool act = q < len;
        int k = act ? ci[p0 + q] : 0;
        bool w = act && strong[p0 + q] && cf[k] == 1;
        unsigned long long bw = g.bits(w);
        if (w) {
            int oo = o + g.below(bw);
            pci[oo] = cidx[k];
            pv[oo] = -(alpha * v[p0 + q]) / atil;
        }
        o += __popcll(bw);
    }
}

// ------------------------------------------------------------ extended+i interpolation
// Distance-two interpolation (De Sterck, Falgout, Nolting and Yang, Numer.
// Linear Algebra Appl. 15 (2008)).  A lane group of G lanes per row keeps the
// row's interpolatory set -- its strong C-neighbours and the strong
// C-neighbours of its strong F-neighbours -- as the keys of an LDS hash table
// (linear probing, as in the hashed SpGEMM).  The counts use tables of 512
// slots; a set that fills its table sets *flag.
constexpr int INTERP_EXT_COUNT_CAP = 512;

template <int CAP>
__device__ inline void ext_insert(int* K, int j, int* flag) {
    int h = (int)(((unsigned)j * 2654435761u) >> (32 - log2_pow2(CAP)));
    for (int probes = 0; probes < CAP; ++probes) {
        const int old = atomicCAS(&K[h], -1, j);
        if (old == -1 || old == j) return;
        h = (h + 1) & (CAP - 1);
    }
    set_flag(flag, 6);
}

template <int CAP>
__device__ inline int ext_find(const int* K, int j) {
    int h = (int)(((unsigned)j * 2654435761u) >> (32 - log2_pow2(CAP)));
    for (int probes = 0; probes < CAP; ++probes) {
        const int key = K[h];
        if (key == j) return h;
        if (key == -1) return -1;
        h = (h + 1) & (CAP - 1);
    }
    return -1;
}

// Inserts the interpolatory set of the group's row (entries p0 .. p0+len of A;
// len = 0 for C-rows); maxlen is the longest len of the wavefront.
template <int G, int CAP>
__device__ inline void ext_gather_set(const Grp<G>& g, int p0, int len, int maxlen, const int* __restrict__ rp,
                                      const int* __restrict__ ci, const unsigned char* __restrict__ strong,
                                      const int* __restrict__ cf, int* K, int* flag) {
    for (int base = 0; base < maxlen; base += G) {
        const int q = base + g.gl;
        const bool act = q < len;
        const int k = act ? ci[p0 + q] : 0;
        const bool st = act && strong[p0 + q];
        const bool isc = st && cf[k] == 1;
        if (isc) ext_insert<CAP>(K, k, flag);
        int kb0 = 0, kb1 = 0;
        if (st && !isc) {
            kb0 = rp[k];
            kb1 = rp[k + 1];
        }
        // the strong C-neighbours of each strong F-neighbour, one row after another
        const int lim = min(G, maxlen - base);
        for (int t = 0; t < lim; ++t) {
            const int b0 = __shfl(kb0, g.gbase + t, WAVE), b1 = __shfl(kb1, g.gbase + t, WAVE);
            for (int r = b0 + g.gl; r < b1; r += G) {
                const int l = ci[r];
                if (strong[r] && cf[l] == 1) ext_insert<CAP>(K, l, flag);
            }
        }
    }
}

template <int G>
__global__ __launch_bounds__(TPB) void k_interp_ext_count(int n, const int* __restrict__ rp,
                                                          const int* __restrict__ ci,
                                                          const unsigned char* __restrict__ strong,
                                                          const int* __restrict__ cf, int* __restrict__ cnt,
                                                          int* __restrict__ flag) {
    constexpr int CAP = INTERP_EXT_COUNT_CAP, NG = TPB / G, PER = CAP / G;
    __shared__ int keys[NG][CAP];
    Grp<G> g;
    const int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    const bool valid = i < n;
    const bool frow = valid && cf[i] != 1;
    int* K = keys[threadIdx.x / G];
#pragma unroll
    for (int u = 0; u < PER; ++u) K[g.gl + G * u] = -1;
    const int p0 = valid ? rp[i] : 0, len = frow ? rp[i + 1] - p0 : 0;
    const int maxlen = wave_max_int(len);
    ext_gather_set<G, CAP>(g, p0, len, maxlen, rp, ci, strong, cf, K, flag);
    int mine = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) mine += (K[g.gl + G * u] >= 0) ? 1 : 0;
    mine = g.sum(mine);
    if (valid && g.gl == 0) cnt[i] = frow ? mine : 1;
}

// The weights, summed exactly as the oracle does: a_ii, then the weak couplings
// outside the set in row order (every lane of the group adds the same terms,
// broadcast one at a time); each set member's numerator starts from a_ij; for
// every strong F-neighbour k in row order, d_k (row k's negative couplings to
// the set and to i, in row order) is formed the same way, then the lanes add
// (a_ik a_kl) / d_k to the numerators of the distinct columns l of row k (or
// to the diagonal for l = i; d_k = 0 lumps a_ik into the diagonal).  The row is
// written in column order (rank among its keys), w_ij = -num_j / atilde_ii.
template <int G, int CAP>
__global__ __launch_bounds__(TPB) void k_interp_ext_fill(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                         const double* __restrict__ v,
                                                         const unsigned char* __restrict__ strong,
                                                         const int* __restrict__ cf, const int* __restrict__ cidx,
                                                         const int* __restrict__ label, const int* __restrict__ prp,
                                                         int* __restrict__ pci, double* __restrict__ pv,
                                                         int* __restrict__ flag) {
    constexpr int NG = TPB / G, PER = CAP / G;
    __shared__ int keys[NG][CAP];
    __shared__ double vals[NG][CAP];
    Grp<G> g;
    const int grp = threadIdx.x / G;
    const int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    const bool valid = i < n;
    if (valid && cf[i] == 1 && g.gl == 0) {
        pci[prp[i]] = cidx[i];
        pv[prp[i]] = 1.0;
    }
    const bool frow = valid && cf[i] != 1 && prp[i + 1] > prp[i];
    int* K = keys[grp];
    double* Vs = vals[grp];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        K[g.gl + G * u] = -1;
        Vs[g.gl + G * u] = 0.0;
    }
    const int p0 = valid ? rp[i] : 0, len = frow ? rp[i + 1] - p0 : 0;
    const int maxlen = wave_max_int(len);
    ext_gather_set<G, CAP>(g, p0, len, maxlen, rp, ci, strong, cf, K, flag);
    const int li = (frow && label) ? label[i] : 0;
    double aii = 0.0;
    for (int base = 0; base < maxlen; base += G) {
        const int q = base + g.gl;
        const bool isd = q < len && ci[p0 + q] == i;
        const double a = isd ? v[p0 + q] : 0.0;
        const unsigned long long m = g.bits(isd);
        const double at = __shfl(a, g.gbase + (m ? __ffsll((unsigned long long)m) - 1 : 0), WAVE);
        if (m) aii = at;
    }
    double atil = aii;
    for (int base = 0; base < maxlen; base += G) {
        const int q = base + g.gl;
        const bool act = q < len;
        const int j = act ? ci[p0 + q] : i;
        const double a = act ? v[p0 + q] : 0.0;
        bool weak = false;
        if (act && j != i && !(label && label[j] != li)) {
            const int h = ext_find<CAP>(K, j);
            if (h >= 0) Vs[h] = a;
            else weak = !strong[p0 + q];
        }
        const int lim = min(G, maxlen - base);
        for (int t = 0; t < lim; ++t) {
            const double x = __shfl(a, g.gbase + t, WAVE);
            const int wk = __shfl((int)weak, g.gbase + t, WAVE);
            if (wk) atil = atil + x;
        }
    }
    for (int base = 0; base < maxlen; base += G) {
        const int q = base + g.gl;
        const bool act = q < len;
        const int k = act ? ci[p0 + q] : 0;
        const bool isf = act && strong[p0 + q] && cf[k] != 1;
        const double aik = isf ? v[p0 + q] : 0.0;
        int kb0 = 0, kb1 = 0;
        if (isf) {
            kb0 = rp[k];
            kb1 = rp[k + 1];
        }
        const int lim = min(G, maxlen - base);
        for (int t = 0; t < lim; ++t) {
            const int src = g.gbase + t;
            const int ft = __shfl((int)isf, src, WAVE);
            const int kt = __shfl(k, src, WAVE);
            const double at = __shfl(aik, src, WAVE);
            const int b0 = __shfl(kb0, src, WAVE), b1 = __shfl(kb1, src, WAVE);
            const int kmax = wave_max_int(b1 - b0);
            double d = 0.0;
            for (int kb = 0; kb < kmax; kb += G) {
                const int r = b0 + kb + g.gl;
                bool mem = false;
                double a2 = 0.0;
                if (r < b1) {
                    const int l = ci[r];
                    a2 = v[r];
                    if (a2 < 0.0 && l != kt) mem = (l == i) || ext_find<CAP>(K, l) >= 0;
                }
                const int lim2 = min(G, kmax - kb);
                for (int u = 0; u < lim2; ++u) {
                    const double x = __shfl(a2, g.gbase + u, WAVE);
                    const int mu = __shfl((int)mem, g.gbase + u, WAVE);
                    if (mu) d = d + x;
                }
            }
            double dterm = 0.0;
            bool dhas = false;
            if (ft && d != 0.0) {
                for (int r = b0 + g.gl; r < b1; r += G) {
                    const int l = ci[r];
                    const double a2 = v[r];
                    if (!(a2 < 0.0) || l == kt) continue;
                    if (l == i) {
                        dterm = (at * a2) / d;
                        dhas = true;
                    } else {
                        const int h = ext_find<CAP>(K, l);
                        if (h >= 0) Vs[h] = Vs[h] + (at * a2) / d;
                    }
                }
            }
            const unsigned long long dm = g.bits(dhas);
            const double dv = __shfl(dterm, g.gbase + (dm ? __ffsll((unsigned long long)dm) - 1 : 0), WAVE);
            if (ft) {
                if (d == 0.0) atil = atil + at;
                else if (dm) atil = atil + dv;
            }
        }
    }
    if (frow && g.gl == 0 && !(atil > 0.0)) set_flag(flag, 6);
    // gather the filled slots, place them after those of the lanes before
    int kk[PER];
    double vv[PER];
    int mine = 0;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        kk[u] = K[g.gl + G * u];
        vv[u] = Vs[g.gl + G * u];
        mine += (kk[u] >= 0) ? 1 : 0;
    }
    int incl = mine;
    for (int off = 1; off < G; off <<= 1) {
        int t = __shfl_up(incl, off, G);
        if (g.gl >= off) incl += t;
    }
    const int L = __shfl(incl, g.gbase + G - 1, WAVE);
    int pos = incl - mine;
#pragma unroll
    for (int u = 0; u < PER; ++u)
        if (kk[u] >= 0) {
            K[pos] = kk[u];
            Vs[pos] = vv[u];
            ++pos;
        }
    if (frow) {
        const int o = prp[i];
        for (int e = g.gl; e < L; e += G) {
            const int key = K[e];
            int rank = 0;
            for (int f = 0; f < L; ++f) rank += (K[f] < key) ? 1 : 0;
            pci[o + rank] = cidx[key];
            pv[o + rank] = -Vs[e] / atil;
        }
    }
}

template <int G>
__global__ __launch_bounds__(TPB) void k_l1_dinv_g(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                   const double* __restrict__ v, double* __restrict__ dinv,
                                                   int* __restrict__ flag) {
    Grp<G> g;
    int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    bool valid = i < n;
    double s = 0.0, aii = 0.0;
    if (valid)
        for (int p = rp[i] + g.gl; p < rp[i + 1]; p += G) {
            if (ci[p] == i) aii = v[p];
            else s += fabs(v[p]);
        }
    s = g.sumd(s);
    aii = g.sumd(aii);
    if (valid && g.gl == 0) {
        double d = aii + s;
        if (!(d > 0.0)) { set_flag(flag, 6); d = 1.0; }
        dinv[i] = 1.0 / d;
    }
}

// ------------------------------------------------------------------ aggressive coarsening
// Second-order strength on the first C-points (C1; isC1 flags, e1 their exclusive
// prefix = C1 index): the graph is the pattern of L * Rt without its diagonal,
// with L = the strong rows of the C1 points (global columns) and Rt = S
// restricted to C1 columns plus a unit entry (k, C1 index of k) for every C1
// point k, so that row i of L * Rt holds every C1 point one or two strong
// connections away from i.  All values are 1 (the products count paths).
__global__ void k_agg_rt_count(int n, const int* __restrict__ srp, const int* __restrict__ sci,
                               const int* __restrict__ isC1, int* __restrict__ cnt) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int c = isC1[k];
    for (int q = srp[k]; q < srp[k + 1]; ++q) c += isC1[sci[q]];
    cnt[k] = c;
}

__global__ void k_agg_rt_fill(int n, const int* __restrict__ srp, const int* __restrict__ sci,
                              const int* __restrict__ isC1, const int* __restrict__ e1, const int* __restrict__ rp,
                              int* __restrict__ ci, double* __restrict__ v) {
    int k = blockIdx.x * blockDim.x + threadIdx.x;
    if (k >= n) return;
    int o = rp[k];
    bool own = isC1[k] != 0;
    for (int q = srp[k]; q < srp[k + 1]; ++q) {
        int j = sci[q];
        if (own && j > k) {          // the unit entry in column order (e1 grows with the point index)
            ci[o] = e1[k]; v[o] = 1.0; ++o;
            own = false;
        }
        if (isC1[j]) { ci[o] = e1[j]; v[o] = 1.0; ++o; }
    }
    if (own) { ci[o] = e1[k]; v[o] = 1.0; }
}

// rows of L: the strong row of the C1 point pts[r]
__global__ void k_agg_l_count(int n1, const int* __restrict__ pts, const int* __restrict__ srp,
                              int* __restrict__ cnt) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n1) return;
    int i = pts[r];
    cnt[r] = srp[i + 1] - srp[i];
}

__global__ void k_agg_l_fill(int n1, const int* __restrict__ pts, const int* __restrict__ srp,
                             const int* __restrict__ sci, const int* __restrict__ rp, int* __restrict__ ci,
                             double* __restrict__ v) {
    int r = blockIdx.x * blockDim.x + threadIdx.x;
    if (r >= n1) return;
    int i = pts[r], o = rp[r];
    for (int q = srp[i]; q < srp[i + 1]; ++q, ++o) { ci[o] = sci[q]; v[o] = 1.0; }
}

// the pattern of a square CSR without its diagonal entries
__global__ void k_nodiag_count(int n, const int* __restrict__ rp, const int* __restrict__ ci, int* __restrict__ cnt) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int c = 0;
    for (int p = rp[i]; p < rp[i + 1]; ++p) c += (ci[p] != i);
    cnt[i] = c;
}

__global__ void k_nodiag_fill(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                              const int* __restrict__ orp, int* __restrict__ oci) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    int o = orp[i];
    for (int p = rp[i]; p < rp[i + 1]; ++p)
        if (ci[p] != i) oci[o++] = ci[p];
}

// lam[j] = number of entries in column j (the PMIS measure of a strength graph)
__global__ void k_col_count(long nnz, const int* __restrict__ ci, int* __restrict__ lam) {
    long p = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (p < nnz) atomicAdd(lam + ci[p], 1);
}

// final split: C where the point is a C1 point chosen again by the second PMIS
__global__ void k_agg_final(int n, const int* __restrict__ isC1, const int* __restrict__ e1,
                            const int* __restrict__ cf2, int* __restrict__ cf) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    cf[i] = (isC1[i] && cf2[e1[i]] == 1) ? 1 : -1;
}

// multi-pass interpolation: points interpolated so far (C-points and the rows
// of P that are not empty) count as C in the next pass
__global__ void k_mp_assigned(int n, const int* __restrict__ cf, const int* __restrict__ prp,
                              int* __restrict__ cfm) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= n) return;
    cfm[i] = (cf[i] == 1 || prp[i + 1] > prp[i]) ? 1 : -1;
}

// number of points the next pass reaches (not yet interpolated, with a strong
// neighbour that is), one atomic per wavefront
__global__ void k_mp_reach(int n, const int* __restrict__ cfm, const int* __restrict__ wcnt,
                           unsigned long long* __restrict__ reach) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    bool r = i < n && cfm[i] != 1 && wcnt[i] > 0;
    unsigned long long m = __ballot(r);
    if ((threadIdx.x & (WAVE - 1)) == 0 && m) atomicAdd(reach, (unsigned long long)__popcll(m));
}

// Diagonal of the hybrid L1 Gauss-Seidel smoother: d_i = a_ii plus the l1 norm
// of row i's entries outside its chunk [i - i % chunk, + chunk) (*flag set
// where it is not positive).
template <int G>
__global__ __launch_bounds__(TPB) void k_hgs_diag_g(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                    const double* __restrict__ v, int chunk, double* __restrict__ d,
                                                    int* __restrict__ flag) {
    Grp<G> g;
    int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    bool valid = i < n;
    double s = 0.0, aii = 0.0;
    if (valid) {
        const int c0 = i - i % chunk, c1 = c0 + chunk;
        for (int p = rp[i] + g.gl; p < rp[i + 1]; p += G) {
            const int j = ci[p];
            if (j == i) aii = v[p];
            else if (j < c0 || j >= c1) s += fabs(v[p]);
        }
    }
    s = g.sumd(s);
    aii = g.sumd(aii);
    if (valid && g.gl == 0) {
        double di = aii + s;
        if (!(di > 0.0)) { set_flag(flag, 6); di = 1.0; }
        d[i] = di;
    }
}

// The entries a_ij with label[i] == label[j] (the separate-component
// approximation of a block whose unknowns carry field labels): G lanes per
// row, counts, then the kept entries in their order (ballot compaction).
template <int G, bool FILL>
__global__ __launch_bounds__(TPB) void k_label_filter_g(int n, const int* __restrict__ rp,
                                                        const int* __restrict__ ci, const double* __restrict__ v,
                                                        const int* __restrict__ label, int* __restrict__ cnt,
                                                        const int* __restrict__ orp, int* __restrict__ oci,
                                                        double* __restrict__ ov) {
    Grp<G> g;
    const int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    const bool valid = i < n;
    int p0 = 0, p1 = 0, li = 0, o = 0;
    if (valid) {
        p0 = rp[i];
        p1 = rp[i + 1];
        li = label[i];
        if (FILL) o = orp[i];
    }
    const int wl = wave_max_int(p1 - p0);
    int kept = 0;
    for (int base = 0; base < wl; base += G) {
        const int p = p0 + base + g.gl;
        const bool act = p < p1;
        int j = 0;
        bool keep = false;
        if (act) {
            j = ci[p];
            keep = label[j] == li;
        }
        const unsigned long long bits = g.bits(keep);
        if (FILL && keep) {
            const int q = o + kept + g.below(bits);
            oci[q] = j;
            ov[q] = v[p];
        }
        kept += __popcll(bits);
    }
    if (!FILL && valid && g.gl == 0) cnt[i] = kept;
}

// In-chunk entries of row i of the hybrid Gauss-Seidel sweep (columns sorted,
// diagonal at dpos[i]): below the diagonal down to the chunk start (forward
// sweeps) and above it up to the chunk end (backward sweeps).
__device__ inline void hgs_tri_span(int i, int chunk, int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                    int pd, int& lo0, int& nlo, int& nup) {
    const int c0 = i - i % chunk, c1 = min(n, c0 + chunk);
    int p = pd;
    while (p > rp[i] && ci[p - 1] >= c0) --p;
    lo0 = p;
    nlo = pd - p;
    int q = pd + 1;
    const int pe = rp[i + 1];
    while (q < pe && ci[q] < c1) ++q;
    nup = q - pd - 1;
}

// Widest row of each in-chunk triangle: w[0] = lower, w[1] = upper (two ints
// of one zeroed slot; integer maxima, so the result is deterministic).
__global__ void k_hgs_tri_count(int n, int chunk, const int* __restrict__ rp, const int* __restrict__ ci,
                                const int* __restrict__ dpos, int* __restrict__ w) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    int nlo = 0, nup = 0;
    if (i < n && dpos[i] >= 0) {
        int lo0;
        hgs_tri_span(i, chunk, n, rp, ci, dpos[i], lo0, nlo, nup);
    }
    nlo = wave_max_int(nlo);
    nup = wave_max_int(nup);
    if ((threadIdx.x & (WAVE - 1)) == 0) {
        if (nlo > 0) atomicMax(w, nlo);
        if (nup > 0) atomicMax(w + 1, nup);
    }
}

// Slot tables of the in-chunk triangles, slot k of chunk position t of chunk c
// at (t * W + k) * nchp + c (consecutive chunks adjacent, so the sweep's loads
// coalesce): the local column (0..chunk-1) and the value, lower entries in
// column order, then padding (value 0, column t).  dT[t * nchp + c] = 1 / d of
// that row (1 for rows past n).  One thread per (t, c), c fastest.
__global__ void k_hgs_tri_fill(int n, int chunk, int nchp, const int* __restrict__ rp, const int* __restrict__ ci,
                               const double* __restrict__ v, const int* __restrict__ dpos,
                               const double* __restrict__ d, int wl, unsigned char* __restrict__ lc,
                               double* __restrict__ lv, int wu, unsigned char* __restrict__ uc,
                               double* __restrict__ uv, double* __restrict__ dT) {
    const long q = (long)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (long)nchp * chunk) return;
    const int t = (int)(q / nchp), c = (int)(q % nchp);
    const long il = (long)c * chunk + t;
    int lo0 = 0, nlo = 0, nup = 0, pd = -1;
    const bool row = il < n;
    if (row) {
        pd = dpos[il];
        if (pd >= 0) hgs_tri_span((int)il, chunk, n, rp, ci, pd, lo0, nlo, nup);
    }
    const int c0 = c * chunk;
    for (int k = 0; k < wl; ++k) {
        const size_t o = ((size_t)t * wl + k) * nchp + c;
        const bool e = k < nlo;
        lc[o] = (unsigned char)(e ? ci[lo0 + k] - c0 : t);
        lv[o] = e ? v[lo0 + k] : 0.0;
    }
    for (int k = 0; k < wu; ++k) {
        const size_t o = ((size_t)t * wu + k) * nchp + c;
        const bool e = k < nup;
        uc[o] = (unsigned char)(e ? ci[pd + 1 + k] - c0 : t);
        uv[o] = e ? v[pd + 1 + k] : 0.0;
    }
    if (dT) dT[(size_t)t * nchp + c] = row ? 1.0 / d[il] : 1.0;
}

// Scatter of A's entries into the rows of its transpose: row j of the
// transpose has cnt[j] slots from trp[j]; each entry takes one by decrementing
// cnt[j] (which ends at zero), so the order inside a row is arbitrary.
template <int G>
__global__ __launch_bounds__(TPB) void k_transpose_scatter_g(int nr, const int* __restrict__ rp,
                                                             const int* __restrict__ ci, const double* __restrict__ v,
                                                             const int* __restrict__ trp, int* __restrict__ cnt,
                                                             int* __restrict__ tci, double* __restrict__ tv) {
    Grp<G> g;
    int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    if (i >= nr) return;
    for (int p = rp[i] + g.gl; p < rp[i + 1]; p += G) {
        int j = ci[p];
        int q = trp[j] + atomicSub(&cnt[j], 1) - 1;
        tci[q] = i;
        if (tv) tv[q] = v[p];
    }
}

// Coarsest-level inverse for n <= 128, kept in registers: 256 threads, thread
// (tr, tc) = (t / 16, t % 16) holds the entries (tr + 16 i, tc + 16 k), i, k < 8.
// In-place Gauss-Jordan with partial pivoting and no row exchanges: the pivot
// of column c is the largest |entry| among the rows not yet used as pivots
// (ties to the lower row).  Step (p, c) scales row p by 1/a_pc and removes
// column c from every other row.  Column c of the left half of [A | I] is the
// unit vector e_p from then on, while column p of the right half starts to
// differ from e_p, so the slot of column c stores that right-half column: the
// pivot row gets 1/a_pc there and row r gets -a_rc/a_pc.  At the end slot
// (r, c) holds entry (r, p(c)) of the right half, whose row p(c') is row c' of
// the inverse: inv[c'][p(c)] = slot (p(c'), c).  Two barriers per step: one
// publishes the per-wave pivot candidates, one the scaled pivot row; the
// multipliers of a row travel by shuffles inside its 16-lane group.
__global__ __launch_bounds__(256) void k_dense_inverse_small(int n, const double* __restrict__ a,
                                                             double* __restrict__ inv, int* __restrict__ flag) {
    // the inverse is compared with the oracle's to a tolerance, not bit for
    // bit, so the update may use fused multiply-adds
#pragma clang fp contract(fast)
    __shared__ double cand_v[4];
    __shared__ int cand_i[4];
    __shared__ double prow[128];
    __shared__ int pc[128], pos[128];
    const int t = threadIdx.x, tr = t >> 4, tc = t & 15, w = t >> 6;
    double m[8][8];
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int r = tr + 16 * i;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int c = tc + 16 * k;
            m[i][k] = (r < n && c < n) ? a[(long)r * n + c] : 0.0;
        }
    }
    unsigned used = 0;  // bit i: row tr + 16 i has been a pivot row
#pragma unroll
    for (int KC = 0; KC < 8; ++KC) {
        if (16 * KC >= n) break;
        for (int cl = 0; cl < 16; ++cl) {
            const int c = 16 * KC + cl;
            if (c >= n) break;
            // candidates: the best unused row of column c among this thread's
            // rows, then among the four row groups of the wave
            double bv = -1.0;
            int bi = n;
            if (tc == cl) {
#pragma unroll
                for (int i = 0; i < 8; ++i) {
                    const int r = tr + 16 * i;
                    const double ax = fabs(m[i][KC]);
                    if (r < n && !((used >> i) & 1u) && ax > bv) { bv = ax; bi = r; }
                }
            }
#pragma unroll
            for (int off = 16; off <= 32; off <<= 1) {
                const double ov = __shfl_xor(bv, off, WAVE);
                const int oi = __shfl_xor(bi, off, WAVE);
                if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
            }
            if ((t & (WAVE - 1)) == cl) { cand_v[w] = bv; cand_i[w] = bi; }
            __syncthreads();
            double pvv = cand_v[0];
            int pl = cand_i[0];
#pragma unroll
            for (int q = 1; q < 4; ++q) {
                const double ov = cand_v[q];
                const int oi = cand_i[q];
                if (ov > pvv || (ov == pvv && oi < pl)) { pvv = ov; pl = oi; }
            }
            // every thread read the same candidates: the pivot row is uniform,
            // which turns the row selections below into scalar branches
            const int p = __builtin_amdgcn_readfirstlane(pl);
            if (!(pvv > 0.0) || !isfinite(pvv)) {
                if (t == 0) set_flag(flag, 3);
                return;
            }
            if (t == 0) { pc[c] = p; pos[p] = c; }
            const int pi = p >> 4;
            if (tr == (p & 15)) {
                used |= 1u << pi;
                double x[8];
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    if (i == pi) {
#pragma unroll
                        for (int k = 0; k < 8; ++k) x[k] = m[i][k];
                    }
                const double ip = 1.0 / __shfl(x[KC], cl, 16);
#pragma unroll
                for (int k = 0; k < 8; ++k) x[k] = (k == KC && tc == cl) ? ip : x[k] * ip;
#pragma unroll
                for (int i = 0; i < 8; ++i)
                    if (i == pi) {
#pragma unroll
                        for (int k = 0; k < 8; ++k) m[i][k] = x[k];
                    }
#pragma unroll
                for (int k = 0; k < 8; ++k) prow[tc + 16 * k] = x[k];
            }
            __syncthreads();
            double pr[8];
#pragma unroll
            for (int k = 0; k < 8; ++k) pr[k] = prow[tc + 16 * k];
#pragma unroll
            for (int i = 0; i < 8; ++i) {
                const double f = __shfl(m[i][KC], cl, 16);
                if (tr + 16 * i != p) {
#pragma unroll
                    for (int k = 0; k < 8; ++k) {
                        const double base = (k == KC && tc == cl) ? 0.0 : m[i][k];
                        m[i][k] = base - f * pr[k];
                    }
                }
            }
        }
    }
    __syncthreads();
#pragma unroll
    for (int i = 0; i < 8; ++i) {
        const int r = tr + 16 * i;
        if (r >= n) continue;
        const long row = (long)pos[r] * n;
#pragma unroll
        for (int k = 0; k < 8; ++k) {
            const int c = tc + 16 * k;
            if (c < n) inv[row + pc[c]] = m[i][k];
        }
    }
}

// ------------------------------------------------------------------ fused-apply operators
// R = [X (F columns mapped to global) | I at cmap[i]], X scaled by `scale`.
__global__ void k_rj_count(int nC, const int* __restrict__ xrp, int* __restrict__ len) {
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i < nC) len[i] = xrp[i + 1] - xrp[i] + 1;
}

// P = [[Y (coarse columns) , M (columns nC + fmap)] on F rows ; unit rows on C rows]
__global__ void k_pj_count(int n, const int* __restrict__ isF, const int* __restrict__ lmap,
                           const int* __restrict__ yrp, const int* __restrict__ mrp, int* __restrict__ len) {
    int g = blockIdx.x * blockDim.x + threadIdx.x;
    if (g >= n) return;
    if (!isF[g]) { len[g] = 1; return; }
    int k = lmap[g];
    len[g] = (yrp[k + 1] - yrp[k]) + (mrp[k + 1] - mrp[k]);
}

// Lane-group versions of the two fills above (with the FP32 copy of the values
// too when the output has one allocated), each lane taking FILL_BATCH
// entries of its row with every load of the batch issued before any is used
// (a row's loads form a chain of three or four dependent steps).  In a row of
// R the unit entry goes before the first column above g, so entry p of X lands
// at (p - row start) + (col > g) and the unit after the columns below g.
constexpr int FILL_BATCH = 4;

template <int G>
__global__ __launch_bounds__(TPB) void k_rj_fill_g(int nC, const int* __restrict__ xrp, const int* __restrict__ xci,
                                                   const double* __restrict__ xv, double scale,
                                                   const int* __restrict__ fmap, const int* __restrict__ cmap,
                                                   const int* __restrict__ rrp, int* __restrict__ rci,
                                                   double* __restrict__ rv, float* __restrict__ rvf) {
    Grp<G> g;
    const int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    const bool valid = i < nC;
    int p0 = 0, len = 0, o = 0, gc = 0;
    if (valid) {
        p0 = xrp[i];
        len = xrp[i + 1] - p0;
        o = rrp[i];
        gc = cmap[i];
    }
    const int wl = wave_max_int(len);
    int nless = 0;
    for (int base = 0; base < wl; base += G * FILL_BATCH) {
        int col[FILL_BATCH];
        double val[FILL_BATCH];
#pragma unroll
        for (int u = 0; u < FILL_BATCH; ++u) {
            const int q = base + u * G + g.gl;
            col[u] = q < len ? xci[p0 + q] : -1;
            val[u] = q < len ? xv[p0 + q] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < FILL_BATCH; ++u) col[u] = col[u] >= 0 ? fmap[col[u]] : -1;
#pragma unroll
        for (int u = 0; u < FILL_BATCH; ++u) {
            const int q = base + u * G + g.gl;
            const bool act = q < len;
            if (act) {
                const int pos = o + q + (col[u] > gc ? 1 : 0);
                const double x = scale * val[u];
                rci[pos] = col[u];
                rv[pos] = x;
                if (rvf) rvf[pos] = (float)x;
            }
            nless += __popcll(g.bits(act && col[u] < gc));
        }
    }
    if (valid && g.gl == 0) {
        rci[o + nless] = gc;
        rv[o + nless] = 1.0;
        if (rvf) rvf[o + nless] = 1.0f;
    }
}

template <int G>
__global__ __launch_bounds__(TPB) void k_pj_fill_g(int n, int nC, const int* __restrict__ isF,
                                                   const int* __restrict__ lmap, const int* __restrict__ yrp,
                                                   const int* __restrict__ yci, const double* __restrict__ yv,
                                                   double yscale, const int* __restrict__ mrp,
                                                   const int* __restrict__ mci, const double* __restrict__ mv,
                                                   double mscale, const int* __restrict__ fmap,
                                                   const int* __restrict__ prp, int* __restrict__ pci,
                                                   double* __restrict__ pv, float* __restrict__ pvf) {
    Grp<G> g;
    const int r = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    if (r >= n) return;
    const int o = prp[r];
    const int k = lmap[r];
    if (!isF[r]) {
        if (g.gl == 0) {
            pci[o] = k;
            pv[o] = 1.0;
            if (pvf) pvf[o] = 1.0f;
        }
        return;
    }
    // the row is [Y row k | M row k]: entry q < ylen from Y, the rest from M
    const int y0 = yrp[k], ylen = yrp[k + 1] - y0;
    const int m0 = mrp[k], len = ylen + mrp[k + 1] - m0;
    for (int base = 0; base < len; base += G * FILL_BATCH) {
        int col[FILL_BATCH];
        double val[FILL_BATCH];
#pragma unroll
        for (int u = 0; u < FILL_BATCH; ++u) {
            const int q = base + u * G + g.gl;
            const bool iny = q < ylen, inm = !iny && q < len;
            col[u] = iny ? yci[y0 + q] : (inm ? mci[m0 + q - ylen] : -1);
            val[u] = iny ? yscale * yv[y0 + q] : (inm ? mscale * mv[m0 + q - ylen] : 0.0);
        }
#pragma unroll
        for (int u = 0; u < FILL_BATCH; ++u) {
            const int q = base + u * G + g.gl;
            if (q >= ylen && q < len) col[u] = nC + fmap[col[u]];
        }
#pragma unroll
        for (int u = 0; u < FILL_BATCH; ++u) {
            const int q = base + u * G + g.gl;
            if (q < len) {
                pci[o + q] = col[u];
                pv[o + q] = val[u];
                if (pvf) pvf[o + q] = (float)val[u];
            }
        }
    }
}

// ---------------------------------------------------------------- composed two-grid operators
// For one L1-Jacobi V(1,1) level (pre-sweep from zero, restriction, coarse
// correction, post-sweep) the output is linear in the level's right-hand side b
// and the coarse correction x_c:  b_c = G b  and  x = W b + Q x_c  with
//   W = 2 D^-1 - D^-1 A D^-1,  Q = P - D^-1 (A P),  G = R - (R A) D^-1.
// These kernels form W, Q, G on the patterns of A, A P and R A; every entry of
// P (of R) must appear in the pattern of A P (of R A), which holds when every
// row of A stores its diagonal.  A missing diagonal or entry sets *bad.

// W on the pattern of A.
template <int G>
__global__ __launch_bounds__(TPB) void k_compose_w_g(int n, const int* __restrict__ rp, const int* __restrict__ ci,
                                                     const double* __restrict__ v, const double* __restrict__ dinv,
                                                     double* __restrict__ w, int* __restrict__ bad) {
    Grp<G> g;
    int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    bool valid = i < n;
    int diag = 0;
    if (valid) {
        double di = dinv[i];
        for (int p = rp[i] + g.gl; p < rp[i + 1]; p += G) {
            int j = ci[p];
            double t = di * v[p];
            t = t * dinv[j];
            double o = -t;
            if (j == i) {
                o = 2.0 * di - t;
                ++diag;
            }
            w[p] = o;
        }
    }
    diag = g.sum(diag);
    if (valid && g.gl == 0 && diag != 1) atomicMax(bad, 1);
}

// out = X - S Y on the pattern of Y, with S = diag(rs) from the left (rs != null)
// or diag(cs) from the right.  Row i of X must be contained in row i of Y.
template <int G>
__global__ __launch_bounds__(TPB) void k_compose_sub_g(int nr, const int* __restrict__ xrp, const int* __restrict__ xci,
                                                       const double* __restrict__ xv, const int* __restrict__ yrp,
                                                       const int* __restrict__ yci, const double* __restrict__ yv,
                                                       const double* __restrict__ rs, const double* __restrict__ cs,
                                                       double* __restrict__ out, int* __restrict__ bad) {
    Grp<G> g;
    int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    bool valid = i < nr;
    int found = 0, xlen = 0;
    if (valid) {
        int x0 = xrp[i], x1 = xrp[i + 1];
        xlen = x1 - x0;
        double ri = rs ? rs[i] : 0.0;
        for (int p = yrp[i] + g.gl; p < yrp[i + 1]; p += G) {
            int j = yci[p];
            double t = (rs ? ri : cs[j]) * yv[p];
            // binary search for column j in row i of X (columns ascending)
            int lo = x0, hi = x1;
            while (lo < hi) {
                int mid = (lo + hi) >> 1;
                if (xci[mid] < j) lo = mid + 1;
                else hi = mid;
            }
            double o = -t;
            if (lo < x1 && xci[lo] == j) {
                o = xv[lo] - t;
                ++found;
            }
            out[p] = o;
        }
    }
    found = g.sum(found);
    if (valid && g.gl == 0 && found != xlen) atomicMax(bad, 1);
}

// C = [A | B] row by row (columns of B shifted by off); C's row pointers are
// the sums of A's and B's.
template <int G>
__global__ __launch_bounds__(TPB) void k_concat_g(int nr, const int* __restrict__ arp, const int* __restrict__ aci,
                                                  const double* __restrict__ av, const int* __restrict__ brp,
                                                  const int* __restrict__ bci, const double* __restrict__ bv, int off,
                                                  int* __restrict__ crp, int* __restrict__ cci,
                                                  double* __restrict__ cv) {
    Grp<G> g;
    int i = (int)(((long)blockIdx.x * TPB + threadIdx.x) / G);
    if (i > nr) return;
    int a0 = arp[i], b0 = brp[i];
    int o = a0 + b0;
    if (g.gl == 0) crp[i] = o;
    if (i == nr) return;
    int la = arp[i + 1] - a0, lb = brp[i + 1] - b0;
    for (int q = g.gl; q < la; q += G) {
        cci[o + q] = aci[a0 + q];
        cv[o + q] = av[a0 + q];
    }
    for (int q = g.gl; q < lb; q += G) {
        cci[o + la + q] = bci[b0 + q] + off;
        cv[o + la + q] = bv[b0 + q];
    }
}

}  // namespace

// ====================================================================== launchers
static int group_for(int max_row) {
    if (max_row < 0) return 64;
    int G = 4;
    while (G < max_row && G < 64) G <<= 1;
    return G;
}

// Lane groups for streaming row kernels that are bound by memory latency:
// about four chunks per row, so a wavefront covers several rows and keeps
// more loads in flight than one lane per entry of the longest row would.
static int group_rows(int max_row) { return max_row < 0 ? 64 : group_for((max_row + 3) / 4); }

#define MGR_DISPATCH_G4(G, ...)                                  \
    switch (G) {                                                 \
        case 4: { constexpr int GG = 4; __VA_ARGS__; } break;    \
        case 8: { constexpr int GG = 8; __VA_ARGS__; } break;    \
        case 16: { constexpr int GG = 16; __VA_ARGS__; } break;  \
        case 32: { constexpr int GG = 32; __VA_ARGS__; } break;  \
        default: { constexpr int GG = 64; __VA_ARGS__; } break;  \
    }

static int grid_for(long rows, int G) { return (int)((rows * G + TPB - 1) / TPB); }

void scan_async(const int* in, int* out, int n, long long* slot, hipStream_t s) {
    if (n <= SCAN_SMALL) {
        k_scan_small<<<1, SCAN_SMALL_T, 0, s>>>(in, n < 0 ? 0 : n, out, slot);
        MGR_LAUNCH_CHECK();
        return;
    }
    int nb = ceil_div(n > 0 ? n : 1, SCAN_B);
    DArr<long long> tmp((size_t)2 * nb + 2, s);
    k_scan_reduce<<<nb, SCAN_T, 0, s>>>(in, n, tmp.p, tmp.p + nb);
    k_scan_apply<<<nb, SCAN_T, 0, s>>>(in, n, tmp.p, tmp.p + nb, nb, out, slot);
    MGR_LAUNCH_CHECK();
}

void scan_exclusive_async(const int* in, int* out, int n, hipStream_t s) { scan_async(in, out, n, nullptr, s); }


void fill_ll(long long* p, long long v, int n, hipStream_t s) {
    if (n <= 0) return;
    k_fill_ll<<<nblk(n), TPB, 0, s>>>(p, v, n);
    MGR_LAUNCH_CHECK();
}

int read_int(const int* dptr, hipStream_t s) {
    int h = 0;
    MGR_HIP(hipMemcpyAsync(&h, dptr, sizeof(int), hipMemcpyDeviceToHost, s));
    MGR_HIP(hipStreamSynchronize(s));
    return h;
}


void field_hist(int n, const int* field, int* hist, int* flag, hipStream_t s) {
    k_fill_int<<<1, 32, 0, s>>>(hist, 0, 32);
    if (n > 0) k_field_hist<<<std::min(nblk(n), 1024), TPB, 0, s>>>(n, field, hist, flag);
    MGR_LAUNCH_CHECK();
}

void fill_bytes(unsigned char* p, unsigned char v, long n, hipStream_t s) {
    if (n <= 0) return;
    k_fill_u8<<<nblk(n), TPB, 0, s>>>(p, v, n);
    MGR_LAUNCH_CHECK();
}

void fill_int(int* p, int v, long n, hipStream_t s) {
    if (n <= 0) return;
    k_fill_int<<<nblk(n), TPB, 0, s>>>(p, v, n);
    MGR_LAUNCH_CHECK();
}

void to_float(const double* src, float* dst, long n, hipStream_t s) {
    if (n <= 0) return;
    k_to_float<<<nblk(n), TPB, 0, s>>>(src, dst, n);
    MGR_LAUNCH_CHECK();
}

void to_float_batch(int k, const double* const* src, float* const* dst, const long* n, hipStream_t s) {
    if (k <= 0) return;
    if (k > F32_SEGS) throw Error(MGR_ERR_ARG, "internal: too many FP32 conversion segments");
    F32Segs sg{};
    sg.k = k;
    long blocks = 0;
    for (int q = 0; q < k; ++q) {
        sg.src[q] = src[q];
        sg.dst[q] = dst[q];
        sg.n[q] = n[q];
        sg.boff[q] = (int)blocks;
        blocks += (n[q] + (long)TPB * F32_PER - 1) / ((long)TPB * F32_PER);
    }
    sg.boff[k] = (int)blocks;
    if (blocks <= 0) return;
    if (blocks > INT_MAX) throw Error(MGR_ERR_UNSUPPORTED, "FP32 conversion too large");
    k_to_float_batch<<<(unsigned)blocks, TPB, 0, s>>>(sg);
    MGR_LAUNCH_CHECK();
}

void negate(double* v, long n, hipStream_t s) {
    if (n <= 0) return;
    k_negate<<<nblk(n), TPB, 0, s>>>(v, n);
    MGR_LAUNCH_CHECK();
}

void gather_int(int n, const int* map, const int* src, int* dst, hipStream_t s) {
    if (n <= 0) return;
    k_gather_int<<<nblk(n), TPB, 0, s>>>(n, map, src, dst);
    MGR_LAUNCH_CHECK();
}

void iota_div(int n, int b, int* out, hipStream_t s) {
    if (n <= 0) return;
    k_iota_div<<<nblk(n), TPB, 0, s>>>(n, b, out);
    MGR_LAUNCH_CHECK();
}

void bsr_count(int b, int nbr, long nnzb, const int* brp, const int* bci, const double* bv, int* cnt,
               hipStream_t s) {
    if (nbr <= 0) return;
    long n = (long)nbr * b;
    int G = group_for((int)((nnzb + nbr - 1) / nbr));
    MGR_DISPATCH_G4(G, (k_bsr_count_g<GG><<<grid_for(n, GG), TPB, 0, s>>>(b, nbr, brp, bci, bv, cnt)));
    MGR_LAUNCH_CHECK();
}

void bsr_fill(int b, int nbr, long nnzb, const int* brp, const int* bci, const double* bv, DCsr& A, hipStream_t s) {
    if (nbr <= 0) return;
    long n = (long)nbr * b;
    int G = group_for((int)((nnzb + nbr - 1) / nbr));
    MGR_DISPATCH_G4(G, (k_bsr_fill_g<GG><<<grid_for(n, GG), TPB, 0, s>>>(b, nbr, brp, bci, bv, A.rp.p, A.ci.p,
                                                                           A.v.p)));
    MGR_LAUNCH_CHECK();
}

void bsr_transpose_blocks(int b, int nbr, const int* rp, const int* ci, const double* v, int* trp, int* tci,
                          double* tv, hipStream_t s) {
    int nnzb = read_int(rp + nbr, s);
    DArr<int> cnt((size_t)nbr + 1, s), cursor((size_t)nbr + 1, s), src((size_t)(nnzb > 0 ? nnzb : 1), s);
    fill_int(cnt.p, 0, nbr + 1, s);
    if (nnzb > 0) k_bsr_tcount<<<nblk(nnzb), TPB, 0, s>>>(nnzb, ci, cnt.p);
    scan_exclusive_async(cnt.p, trp, nbr, s);
    MGR_HIP(hipMemcpyAsync(cursor.p, trp, sizeof(int) * (nbr + 1), hipMemcpyDeviceToDevice, s));
    k_bsr_tscatter<<<nblk(nbr), TPB, 0, s>>>(nbr, rp, ci, cursor.p, tci, src.p);
    k_bsr_tsort<<<nblk(nbr), TPB, 0, s>>>(nbr, trp, tci, src.p);
    if (nnzb > 0) k_bsr_tvalues<<<nblk(nnzb), TPB, 0, s>>>(nnzb, b, src.p, v, tv);
    MGR_LAUNCH_CHECK();
}

void cf_flags(int n, const int* field, uint32_t mask, int* isF, int* flag, hipStream_t s) {
    if (n <= 0) return;
    k_cf_flags<<<nblk(n), TPB, 0, s>>>(n, field, mask, isF, flag);
    MGR_LAUNCH_CHECK();
}

void cf_maps(int n, const int* isF, const int* fpos, int* lmap, int* fmap, int* cmap, hipStream_t s) {
    if (n <= 0) return;
    k_cf_maps<<<nblk(n), TPB, 0, s>>>(n, isF, fpos, lmap, fmap, cmap);
    MGR_LAUNCH_CHECK();
}

void extract_count(const DCsr& A, const int* isF, const int* lmap, const int* fblk, int* cFF, int* cFC, int* cCF,
                   int* cCC, hipStream_t s) {
    if (A.nr <= 0) return;
    int G = group_rows(A.max_row);
    MGR_DISPATCH_G4(G, (k_extract_count_g<GG><<<grid_for(A.nr, GG), TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, isF, lmap, fblk,
                                                                                   cFF, cFC, cCF, cCC)));
    MGR_LAUNCH_CHECK();
}

// the arrays of an output CSR, or nulls when it is not produced (nr == 0 and no rows)
static inline const int* orp(const DCsr* M) { return M ? M->rp.p : nullptr; }
static inline int* oci(DCsr* M) { return M ? M->ci.p : nullptr; }
static inline double* ov(DCsr* M) { return M ? M->v.p : nullptr; }

void extract_fill(const DCsr& A, const int* isF, const int* lmap, const int* fblk, DCsr* FF, DCsr* FC, DCsr* CF,
                  DCsr* CC, hipStream_t s) {
    if (A.nr <= 0) return;
    int G = group_rows(A.max_row);
    MGR_DISPATCH_G4(G, (k_extract_fill_g<GG><<<grid_for(A.nr, GG), TPB, 0, s>>>(
                           A.nr, A.rp.p, A.ci.p, A.v.p, isF, lmap, fblk, orp(FF), oci(FF), ov(FF), orp(FC), oci(FC),
                           ov(FC), orp(CF), oci(CF), ov(CF), orp(CC), oci(CC), ov(CC))));
    MGR_LAUNCH_CHECK();
}

#define MGR_DISPATCH_B(B, ...)                                    \
    switch (B) {                                                  \
        case 2: { constexpr int BB = 2; __VA_ARGS__; } break;     \
        case 3: { constexpr int BB = 3; __VA_ARGS__; } break;     \
        default: { constexpr int BB = 4; __VA_ARGS__; } break;    \
    }

// lanes per block row: about one block per lane
static int bsr_group(int nbr, long nnzb) {
    const int avg = (int)((nnzb + nbr - 1) / nbr);
    return avg <= 4 ? 4 : avg <= 8 ? 8 : avg <= 16 ? 16 : avg <= 32 ? 32 : 64;
}

void bsr_extract_count(int b, int nbr, long nnzb, const int* brp, const int* bci, const double* bv, const int* isF,
                       const int* lmap, const int* fblk, int* cFF, int* cFC, int* cCF, int* cCC, hipStream_t s) {
    if (nbr <= 0) return;
    const int G = bsr_group(nbr, nnzb);
    MGR_DISPATCH_B(b, MGR_DISPATCH_G4(G, (k_bsr_extract_count_g<GG, BB><<<grid_for(nbr, GG), TPB, 0, s>>>(
                                             nbr, brp, bci, bv, isF, lmap, fblk, cFF, cFC, cCF, cCC))));
    MGR_LAUNCH_CHECK();
}

void bsr_extract_fill(int b, int nbr, long nnzb, const int* brp, const int* bci, const double* bv, const int* isF,
                      const int* lmap, const int* fblk, DCsr* FF, DCsr* FC, DCsr* CF, DCsr* CC, double* vcopy,
                      hipStream_t s) {
    if (nbr <= 0) return;
    const int G = bsr_group(nbr, nnzb);
    MGR_DISPATCH_B(b, MGR_DISPATCH_G4(G, (k_bsr_extract_fill_g<GG, BB><<<grid_for((long)nbr * BB, GG), TPB, 0, s>>>(
                                             nbr, brp, bci, bv, isF, lmap, fblk, orp(FF), oci(FF), ov(FF), orp(FC),
                                             oci(FC), ov(FC), orp(CF), oci(CF), ov(CF), orp(CC), oci(CC), ov(CC),
                                             vcopy))));
    MGR_LAUNCH_CHECK();
}

void frelax_block_flags(int nF, const int* bid, int* flagk, hipStream_t s) {
    if (nF <= 0) return;
    k_frelax_flags<<<nblk(nF), TPB, 0, s>>>(nF, bid, flagk);
    MGR_LAUNCH_CHECK();
}

void frelax_block_starts(int nF, const int* flagk, const int* excl, int* bstart, int* bnum, hipStream_t s) {
    if (nF <= 0) return;
    k_frelax_starts<<<nblk(nF), TPB, 0, s>>>(nF, flagk, excl, bstart, bnum);
    MGR_LAUNCH_CHECK();
}

void frelax_row_len(int nF, const int* bnum, const int* bstart, int* len, int* flag, hipStream_t s) {
    if (nF <= 0) return;
    k_frelax_len<<<nblk(nF), TPB, 0, s>>>(nF, bnum, bstart, len, flag);
    MGR_LAUNCH_CHECK();
}

void frelax_fill(int nb, const int* bstart, const DCsr& AFF, DCsr& M, int* flag, hipStream_t s) {
    if (nb <= 0) return;
    k_frelax_fill<<<grid_for(nb, 4), TPB, 0, s>>>(nb, bstart, AFF.rp.p, AFF.ci.p, AFF.v.p, M.rp.p, M.ci.p, M.v.p,
                                                  flag);
    MGR_LAUNCH_CHECK();
}


template <bool FILL>
static void spgemm_launch(const DCsr& A, const DCsr& B, int max_row, const int* crp, int* cci, double* cv, int* cnt,
                          int* flag, hipStream_t s) {
    // max_row selects the variant: <= 64 entries per row of A -> one head per lane
    if (A.nr <= 0) return;
    if (B.nc <= SPGEMM_DENSE && A.nr <= SPGEMM_DENSE_ROWS && (long)A.nr * B.nc <= SPGEMM_DENSE_WORK) {
        const size_t lds = (size_t)B.nc * (FILL ? sizeof(double) + 1 : 1);
        k_spgemm_dw<FILL><<<A.nr, WAVE, lds, s>>>(A.nr, A.rp.p, A.ci.p, A.v.p, B.rp.p, B.ci.p, B.v.p, B.nc, crp, cci,
                                                cv, cnt);
        MGR_LAUNCH_CHECK();
        return;
    }
    int grid = ceil_div(A.nr, TPB / WAVE);
    if (max_row <= 32) {
        int G = 1;
        while (G < max_row) G <<= 1;
        int g2 = ceil_div((long)A.nr * G, TPB);
#define MGR_SPGEMM_G(GG)                                                                                         \
    k_spgemm_g<GG, FILL><<<g2, TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, A.v.p, B.rp.p, B.ci.p, B.v.p, crp, cci, cv, cnt, \
                                           flag)
        switch (G) {
            case 1: MGR_SPGEMM_G(1); break;
            case 2: MGR_SPGEMM_G(2); break;
            case 4: MGR_SPGEMM_G(4); break;
            case 8: MGR_SPGEMM_G(8); break;
            case 16: MGR_SPGEMM_G(16); break;
            default: MGR_SPGEMM_G(32); break;
        }
#undef MGR_SPGEMM_G
    } else if (max_row <= WAVE)
        k_spgemm<1, FILL><<<grid, TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, A.v.p, B.rp.p, B.ci.p, B.v.p, crp, cci, cv,
                                                cnt, flag);
    else if (max_row <= 4 * WAVE)
        k_spgemm<4, FILL><<<grid, TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, A.v.p, B.rp.p, B.ci.p, B.v.p, crp, cci, cv,
                                                cnt, flag);
    else if (max_row <= 16 * WAVE)
        k_spgemm<16, FILL><<<grid, TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, A.v.p, B.rp.p, B.ci.p, B.v.p, crp, cci, cv,
                                                 cnt, flag);
    else
        throw Error(-6, "SpGEMM: a row of the left factor has more than 1024 entries");
    MGR_LAUNCH_CHECK();
}


static bool spgemm_dense_ok(const DCsr& A, const DCsr& B) {
    return B.nc <= SPGEMM_DENSE && A.nr <= SPGEMM_DENSE_ROWS && (long)A.nr * B.nc <= SPGEMM_DENSE_WORK;
}

// Hashed rows with tables of cap slots (cap >= 32, a power of two <= 512);
// with D, C = D + A B.
// lanes per row of A: enough for the rows of B, and for TPB / G tables of cap
// slots to take at most 64 KB of LDS
static int hash_group(const DCsr& B, int cap) {
    int gb = 4;
    while (gb < B.max_row && gb < 32) gb <<= 1;
    int gl = (int)((long)cap * 12 * TPB / 65536);
    int G = gb;
    while (G < gl) G <<= 1;
    return G > 32 ? 32 : G;
}

template <bool FILL, bool ADD>
static void spgemm_hash_launch(const DCsr& A, const DCsr& B, const DCsr* D, int cap, const int* crp, int* cci,
                               double* cv, int* cnt, int* flag, hipStream_t s, int lo = -1, int hi = INT_MAX,
                               double sgn = 1.0, const int* brep = nullptr) {
    const int* drp = ADD ? D->rp.p : nullptr;
    const int* dci = ADD ? D->ci.p : nullptr;
    const double* dvv = ADD ? D->v.p : nullptr;
    const int G = hash_group(B, cap);
#define MGR_HASH(GG, CC)                                                                                          \
    k_spgemm_hash<GG, CC, FILL, ADD><<<grid_for(A.nr, GG), TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, A.v.p, B.rp.p,     \
                                                                       B.ci.p, B.v.p, drp, dci, dvv, crp, cci, cv, \
                                                                       cnt, flag, lo, hi, sgn, brep)
    switch (cap) {
        case 32: if (G <= 4) MGR_HASH(4, 32); else if (G == 8) MGR_HASH(8, 32); else if (G == 16) MGR_HASH(16, 32); else MGR_HASH(32, 32); break;
        case 64: if (G <= 4) MGR_HASH(4, 64); else if (G == 8) MGR_HASH(8, 64); else if (G == 16) MGR_HASH(16, 64); else MGR_HASH(32, 64); break;
        case 128: if (G <= 8) MGR_HASH(8, 128); else if (G == 16) MGR_HASH(16, 128); else MGR_HASH(32, 128); break;
        case 256: if (G <= 16) MGR_HASH(16, 256); else MGR_HASH(32, 256); break;
        default: MGR_HASH(32, 512); break;
    }
#undef MGR_HASH
    MGR_LAUNCH_CHECK();
}

// The lane-per-entry symbolic kernel: rows of A of 24 entries or more and at
// least twice as long as those of B (shorter rows keep more lanes busy in the
// hashed kernel: measured on the MGR products A_CF M, A_CC + A_CF P_F).
static bool lanes_ok(const DCsr& A, const DCsr& B) {
    return A.nr > 0 && A.max_row >= 24 && B.max_row >= 0 && 2 * B.max_row <= A.max_row;
}

template <bool ADD>
static void spgemm_lanes_count(const DCsr& A, const DCsr& B, const DCsr* D, int cap, int* cnt, int* flag,
                               hipStream_t s) {
    const int* drp = ADD ? D->rp.p : nullptr;
    const int* dci = ADD ? D->ci.p : nullptr;
    const int grid = grid_for(A.nr, 32);
#define MGR_LANES(CC) \
    k_spgemm_lanes_count<CC, ADD><<<grid, TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, B.rp.p, B.ci.p, drp, dci, cnt, flag)
    switch (cap) {
        case 32: MGR_LANES(32); break;
        case 64: MGR_LANES(64); break;
        case 128: MGR_LANES(128); break;
        case 256: MGR_LANES(256); break;
        default: MGR_LANES(512); break;
    }
#undef MGR_LANES
    MGR_LAUNCH_CHECK();
}

bool bdiag_left_ok(const DCsr& M, const DCsr& B) {
    return M.max_row >= 0 && M.max_row <= 4 && B.max_row >= 0 && 4 * B.max_row <= BDL_STAGE;
}
// rows of A of 8 entries or more on average: a mostly empty A (A_CF of a
// level whose few F-points couple to few C-points) keeps the hashed product,
// whose small lane groups skip empty rows at less cost
bool bdiag_right_ok(const DCsr& A, const DCsr& M) {
    return A.max_row >= 0 && A.max_row <= 32 && M.max_row >= 0 && M.max_row <= 4 && A.nnz >= 8L * A.nr;
}

void bdiag_left_count(int nb, const int* bstart, const DCsr& B, int* cnt, int* flag, hipStream_t s) {
    if (nb <= 0) return;
    k_bdiag_left_count<16><<<grid_for(nb, 16), TPB, 0, s>>>(nb, bstart, B.rp.p, B.ci.p, cnt, flag);
    MGR_LAUNCH_CHECK();
}
void bdiag_right_count(const DCsr& A, const DCsr& M, int* cnt, int* flag, hipStream_t s) {
    if (A.nr <= 0) return;
    const int grid = grid_for((A.nr + BDR_ROWS - 1) / BDR_ROWS, 32);
    k_bdiag_right<false><<<grid, TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, A.v.p, M.rp.p, M.ci.p, M.v.p, nullptr, nullptr,
                                               nullptr, cnt, flag);
    MGR_LAUNCH_CHECK();
}
void bdiag_right_fill(const DCsr& A, const DCsr& M, DCsr& C, int* flag, hipStream_t s) {
    if (A.nr <= 0) return;
    const int grid = grid_for((A.nr + BDR_ROWS - 1) / BDR_ROWS, 32);
    k_bdiag_right<true><<<grid, TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, A.v.p, M.rp.p, M.ci.p, M.v.p, C.rp.p, C.ci.p,
                                              C.v.p, nullptr, flag);
    MGR_LAUNCH_CHECK();
}

// Numeric hashed pass.  Where the tables of a workgroup take 40 KB of LDS or
// more, the LDS bounds the rows in flight per CU; on a large product whose
// average row is at most a sixth of cap (the longest rows of a Galerkin
// product sit next to wells or boundaries), the rows of at most a quarter of
// cap entries then take tables of half the size in a first launch, the rest
// a second one (measured: the level-0 A P of the pressure AMG, 864 -> 565 +
// 99 us; on small levels, with smaller tables or longer average rows the
// second launch costs more than it saves).
template <bool ADD>
static void spgemm_fill_split(const DCsr& A, const DCsr& B, const DCsr* D, DCsr& C, int cap, int* flag,
                              hipStream_t s, double sgn = 1.0, const int* brep = nullptr) {
    const long lds = (long)(TPB / hash_group(B, cap)) * cap * 12;
    const bool short_rows = C.nr > 0 && 6 * C.nnz <= (long)C.nr * cap;   // average row <= cap / 6
    if (cap >= 64 && lds >= 40960 && A.nr >= 262144 && short_rows) {
        spgemm_hash_launch<true, ADD>(A, B, D, cap / 2, C.rp.p, C.ci.p, C.v.p, nullptr, flag, s, -1, cap / 4, sgn,
                                      brep);
        spgemm_hash_launch<true, ADD>(A, B, D, cap, C.rp.p, C.ci.p, C.v.p, nullptr, flag, s, cap / 4, INT_MAX,
                                      sgn, brep);
    } else {
        spgemm_hash_launch<true, ADD>(A, B, D, cap, C.rp.p, C.ci.p, C.v.p, nullptr, flag, s, -1, INT_MAX, sgn,
                                      brep);
    }
}

static int pow2_at_least(long v, int lo) {
    int c = lo;
    while (c < v) c <<= 1;
    return c;
}

void spgemm_count(const DCsr& A, const DCsr& B, int max_row, int* cnt, int* flag, hipStream_t s, bool loose) {
    // hashed rows when the right factor is too wide for the dense LDS row and
    // every output row is bounded by A.max_row * B.max_row <= 256 distinct
    // columns; with `loose`, also up to a bound of SPGEMM_HASH_LOOSE with
    // tables of 512 slots, a full table then setting *flag to 2
    if (!spgemm_dense_ok(A, B) && A.nr > 0 && B.max_row >= 0 && max_row >= 0) {
        const long bound = (long)max_row * B.max_row;
        if (bound <= 256 || (loose && bound <= SPGEMM_HASH_LOOSE)) {
            const int cap = pow2_at_least(bound < 512 ? bound : 512, 32);
            if (lanes_ok(A, B))
                spgemm_lanes_count<false>(A, B, nullptr, cap, cnt, flag, s);
            else
                spgemm_hash_launch<false, false>(A, B, nullptr, cap, nullptr, nullptr, nullptr, cnt, flag, s);
            return;
        }
    }
    spgemm_launch<false>(A, B, max_row, nullptr, nullptr, nullptr, cnt, flag, s);
}

void spgemm_fill(const DCsr& A, const DCsr& B, int max_row, DCsr& C, int* flag, hipStream_t s, bool neg) {
    // hashed rows when the right factor is too wide for the dense LDS row and the
    // output rows (known from the symbolic pass) fit a table of at most 512 slots
    if (!spgemm_dense_ok(A, B) && A.nr > 0 && C.max_row >= 0 && C.max_row <= 256 && B.max_row >= 0) {
        const int cap = pow2_at_least(2L * C.max_row, 32);
        spgemm_fill_split<false>(A, B, nullptr, C, cap, flag, s, neg ? -1.0 : 1.0);
        return;
    }
    spgemm_launch<true>(A, B, max_row, C.rp.p, C.ci.p, C.v.p, nullptr, nullptr, s);
    if (neg) negate(C.v.p, C.nnz, s);
}

bool spgemm_add_fusable(const DCsr& A, const DCsr& B, const DCsr& D) {
    return D.nr == A.nr && D.nc == B.nc && A.max_row >= 0 && B.max_row >= 0 && D.max_row >= 0 &&
           (long)A.max_row * B.max_row + D.max_row <= 256;
}

void spgemm_add_count(const DCsr& A, const DCsr& B, const DCsr& D, int* cnt, int* flag, hipStream_t s, bool loose,
                      const int* brep) {
    if (!spgemm_add_fusable(A, B, D)) throw Error(-1, "spgemm_add: rows may exceed 256 entries");
    if (A.nr <= 0) return;
    const long bound = (long)A.max_row * B.max_row + D.max_row;
    int cap = pow2_at_least(bound, 32);
    if (loose) {
        // a row of C holds D's row: tables of at least twice that
        const int lc = std::max(SPGEMM_ADD_LOOSE_CAP, pow2_at_least(2L * D.max_row, 32));
        cap = std::min(cap, lc);
    }
    if (lanes_ok(A, B) && !brep)
        spgemm_lanes_count<true>(A, B, &D, cap, cnt, flag, s);
    else
        spgemm_hash_launch<false, true>(A, B, &D, cap, nullptr, nullptr, nullptr, cnt, flag, s, -1, INT_MAX, 1.0,
                                        brep);
}

void spgemm_add_fill(const DCsr& A, const DCsr& B, const DCsr& D, DCsr& C, int* flag, hipStream_t s,
                     const int* brep) {
    if (A.nr <= 0) return;
    const int cap = pow2_at_least(2L * C.max_row, 32);
    spgemm_fill_split<true>(A, B, &D, C, cap, flag, s, 1.0, brep);
}

static int add_group(const DCsr& A, const DCsr& B) {
    if (A.max_row < 0 || B.max_row < 0) return 64;
    return group_for(A.max_row > B.max_row ? A.max_row : B.max_row);
}

void add_count(const DCsr& A, const DCsr& B, int* cnt, hipStream_t s) {
    if (A.nr <= 0) return;
    int G = add_group(A, B);
    MGR_DISPATCH_G4(G, (k_add_g<GG, false><<<grid_for(A.nr, GG), TPB, 0, s>>>(
                           A.nr, A.rp.p, A.ci.p, A.v.p, B.rp.p, B.ci.p, B.v.p, nullptr, nullptr, nullptr, cnt)));
    MGR_LAUNCH_CHECK();
}

void add_fill(const DCsr& A, const DCsr& B, DCsr& C, hipStream_t s) {
    if (A.nr <= 0) return;
    int G = add_group(A, B);
    MGR_DISPATCH_G4(G, (k_add_g<GG, true><<<grid_for(A.nr, GG), TPB, 0, s>>>(
                           A.nr, A.rp.p, A.ci.p, A.v.p, B.rp.p, B.ci.p, B.v.p, C.rp.p, C.ci.p, C.v.p, nullptr)));
    MGR_LAUNCH_CHECK();
}

void transpose_count(const DCsr& A, int* cnt, hipStream_t s) {
    if (A.nnz <= 0) return;
    k_transpose_count<<<nblk(A.nnz), TPB, 0, s>>>(A.nnz, A.ci.p, cnt);
    MGR_LAUNCH_CHECK();
}

void transpose_fill(const DCsr& A, DCsr& T, int* cnt, hipStream_t s) {
    if (A.nnz <= 0) return;
    // scatter into temporaries, then order each row while copying it out
    DArr<int> tci((size_t)A.nnz, s);
    DArr<double> tv(A.v.p ? (size_t)A.nnz : 0, s);
    if (A.nr > 0) {
        int G = group_for(A.max_row);
        MGR_DISPATCH_G4(G, (k_transpose_scatter_g<GG><<<grid_for(A.nr, GG), TPB, 0, s>>>(
                               A.nr, A.rp.p, A.ci.p, A.v.p, T.rp.p, cnt, tci.p, A.v.p ? tv.p : nullptr)));
    }
    if (T.nr > 0)
        k_transpose_rank<<<grid_for(T.nr, WAVE), TPB, 0, s>>>(T.nr, T.rp.p, tci.p, tv.p, T.ci.p,
                                                              A.v.p ? T.v.p : nullptr);
    MGR_LAUNCH_CHECK();
}

void amg_strength(const DCsr& A, double theta, const int* label, unsigned char* strong, int* scnt, int* lam,
                  double* dinv, int* flag, hipStream_t s) {
    if (A.nr <= 0) return;
    int G = group_rows(A.max_row);
    MGR_DISPATCH_G4(G, (k_strength_g<GG><<<grid_for(A.nr, GG), TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, A.v.p, theta, label,
                                                                              strong, scnt, lam, dinv, flag)));
    MGR_LAUNCH_CHECK();
}


void strength_compact_fill(const DCsr& A, const unsigned char* strong, const int* srp, int* sci, hipStream_t s) {
    if (A.nr <= 0) return;
    int G = group_rows(A.max_row);
    MGR_DISPATCH_G4(G, (k_sfill_g<GG><<<grid_for(A.nr, GG), TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, strong, srp, sci)));
    MGR_LAUNCH_CHECK();
}


void pmis_init(int n, const int* lam, uint64_t seed, int level, double* w, int* cf, hipStream_t s) {
    if (n <= 0) return;
    k_pmis_init<<<nblk(n), TPB, 0, s>>>(n, lam, seed, level, w, cf);
    MGR_LAUNCH_CHECK();
}

void pmis_select(int n, const int* srp, const int* sci, const double* w, const int* cf, unsigned char* beaten,
                 int avg_row, hipStream_t s) {
    if (n <= 0) return;
    if (avg_row <= PMIS_GROUP_MIN || n > PMIS_GROUP_MAX_N) {
        k_pmis_select_g<1><<<grid_for(n, 1), TPB, 0, s>>>(n, srp, sci, w, cf, beaten);
    } else {
        int G = group_for(avg_row);
        MGR_DISPATCH_G4(G, (k_pmis_select_g<GG><<<grid_for(n, GG), TPB, 0, s>>>(n, srp, sci, w, cf, beaten)));
    }
    MGR_LAUNCH_CHECK();
}

void pmis_update(int n, const int* srp, const int* sci, const int* cf, const unsigned char* beaten, int* cf_next,
                 unsigned char* beaten_next, int* undecided, int avg_row, hipStream_t s) {
    if (n <= 0) return;
    if (avg_row <= PMIS_GROUP_MIN || n > PMIS_GROUP_MAX_N) {
        k_pmis_update_g<1><<<grid_for(n, 1), TPB, 0, s>>>(n, srp, sci, cf, beaten, cf_next, beaten_next, undecided);
    } else {
        int G = group_for(avg_row);
        MGR_DISPATCH_G4(G, (k_pmis_update_g<GG><<<grid_for(n, GG), TPB, 0, s>>>(n, srp, sci, cf, beaten, cf_next,
                                                                                 beaten_next, undecided)));
    }
    MGR_LAUNCH_CHECK();
}

void cf_is_c(int n, const int* cf, int* isC, hipStream_t s) {
    if (n <= 0) return;
    k_is_c<<<nblk(n), TPB, 0, s>>>(n, cf, isC);
    MGR_LAUNCH_CHECK();
}

void interp_count(const DCsr& A, const unsigned char* strong, const int* cf, int* cnt, hipStream_t s) {
    if (A.nr <= 0) return;
    int G = group_rows(A.max_row);
    MGR_DISPATCH_G4(G, (k_interp_count_g<GG><<<grid_for(A.nr, GG), TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, strong, cf, cnt)));
    MGR_LAUNCH_CHECK();
}

void interp_fill(const DCsr& A, const unsigned char* strong, const int* cf, const int* cidx, const int* label,
                 DCsr& P, int* flag, hipStream_t s) {
    if (A.nr <= 0) return;
    const int avg = (int)((A.nnz + A.nr - 1) / A.nr);
    if (avg > INTERP_LDS_MAX_AVG) {
        // the row sums run lane by lane through each chunk of G entries, so
        // the group is sized to the average row, not the longest
        int G = group_for(avg);
        MGR_DISPATCH_G4(G, (k_interp_fill_g<GG><<<grid_for(A.nr, GG), TPB, 0, s>>>(
                               A.nr, A.rp.p, A.ci.p, A.v.p, strong, cf, cidx, label, P.rp.p, P.ci.p, P.v.p, flag)));
    } else {
        if (!A.blk.p) throw Error(-1, "interp_fill: operator without row blocks");
        k_interp_fill_blk<<<A.nblk, TPB, 0, s>>>(A.blk.p, A.rp.p, A.ci.p, A.v.p, strong, cf, cidx, label, P.rp.p,
                                                 P.ci.p, P.v.p, flag);
    }
    MGR_LAUNCH_CHECK();
}

void interp_ext_count(const DCsr& A, const unsigned char* strong, const int* cf, int* cnt, int* flag, hipStream_t s) {
    if (A.nr <= 0) return;
    if (A.max_row <= 16)
        k_interp_ext_count<16><<<grid_for(A.nr, 16), TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, strong, cf, cnt, flag);
    else
        k_interp_ext_count<32><<<grid_for(A.nr, 32), TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, strong, cf, cnt, flag);
    MGR_LAUNCH_CHECK();
}

void interp_ext_fill(const DCsr& A, const unsigned char* strong, const int* cf, const int* cidx, const int* label,
                     DCsr& P, int* flag, hipStream_t s) {
    if (A.nr <= 0) return;
    if (P.max_row > INTERP_EXT_COUNT_CAP / 2)
        throw Error(-6, "extended+i interpolation: an interpolatory set exceeds 256 points");
    int cap = 64;
    while (cap < 2 * P.max_row) cap <<= 1;
    // 48 KB of LDS per workgroup at most: 16 rows of 256 slots or 8 of 512
    const bool g32 = A.max_row > 16 || cap == 512;
#define MGR_EXT_FILL(GG, CC)                                                                                     \
    k_interp_ext_fill<GG, CC><<<grid_for(A.nr, GG), TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, A.v.p, strong, cf, cidx, \
                                                                label, P.rp.p, P.ci.p, P.v.p, flag)
    switch (cap) {
        case 64: if (g32) MGR_EXT_FILL(32, 64); else MGR_EXT_FILL(16, 64); break;
        case 128: if (g32) MGR_EXT_FILL(32, 128); else MGR_EXT_FILL(16, 128); break;
        case 256: if (g32) MGR_EXT_FILL(32, 256); else MGR_EXT_FILL(16, 256); break;
        default: MGR_EXT_FILL(32, 512); break;
    }
#undef MGR_EXT_FILL
    MGR_LAUNCH_CHECK();
}

void l1_dinv(const DCsr& A, double* dinv, int* flag, hipStream_t s) {
    if (A.nr <= 0) return;
    int G = group_rows(A.max_row);
    MGR_DISPATCH_G4(G, (k_l1_dinv_g<GG><<<grid_for(A.nr, GG), TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, A.v.p, dinv, flag)));
    MGR_LAUNCH_CHECK();
}

void agg_rt_count(int n, const int* srp, const int* sci, const int* isC1, int* cnt, hipStream_t s) {
    if (n <= 0) return;
    k_agg_rt_count<<<nblk(n), TPB, 0, s>>>(n, srp, sci, isC1, cnt);
    MGR_LAUNCH_CHECK();
}
void agg_rt_fill(int n, const int* srp, const int* sci, const int* isC1, const int* e1, DCsr& Rt, hipStream_t s) {
    if (n <= 0) return;
    k_agg_rt_fill<<<nblk(n), TPB, 0, s>>>(n, srp, sci, isC1, e1, Rt.rp.p, Rt.ci.p, Rt.v.p);
    MGR_LAUNCH_CHECK();
}
void agg_l_count(int n1, const int* pts, const int* srp, int* cnt, hipStream_t s) {
    if (n1 <= 0) return;
    k_agg_l_count<<<nblk(n1), TPB, 0, s>>>(n1, pts, srp, cnt);
    MGR_LAUNCH_CHECK();
}
void agg_l_fill(int n1, const int* pts, const int* srp, const int* sci, DCsr& L, hipStream_t s) {
    if (n1 <= 0) return;
    k_agg_l_fill<<<nblk(n1), TPB, 0, s>>>(n1, pts, srp, sci, L.rp.p, L.ci.p, L.v.p);
    MGR_LAUNCH_CHECK();
}
void nodiag_count(const DCsr& A, int* cnt, hipStream_t s) {
    if (A.nr <= 0) return;
    k_nodiag_count<<<nblk(A.nr), TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, cnt);
    MGR_LAUNCH_CHECK();
}
void nodiag_fill(const DCsr& A, DCsr& B, hipStream_t s) {
    if (A.nr <= 0) return;
    k_nodiag_fill<<<nblk(A.nr), TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, B.rp.p, B.ci.p);
    MGR_LAUNCH_CHECK();
}
void col_count(long nnz, const int* ci, int* lam, hipStream_t s) {
    if (nnz <= 0) return;
    k_col_count<<<nblk(nnz), TPB, 0, s>>>(nnz, ci, lam);
    MGR_LAUNCH_CHECK();
}
void agg_final(int n, const int* isC1, const int* e1, const int* cf2, int* cf, hipStream_t s) {
    if (n <= 0) return;
    k_agg_final<<<nblk(n), TPB, 0, s>>>(n, isC1, e1, cf2, cf);
    MGR_LAUNCH_CHECK();
}
void mp_assigned(int n, const int* cf, const int* prp, int* cfm, hipStream_t s) {
    if (n <= 0) return;
    k_mp_assigned<<<nblk(n), TPB, 0, s>>>(n, cf, prp, cfm);
    MGR_LAUNCH_CHECK();
}
void mp_reach(int n, const int* cfm, const int* wcnt, long long* reach, hipStream_t s) {
    if (n <= 0) return;
    k_mp_reach<<<nblk(n), TPB, 0, s>>>(n, cfm, wcnt, reinterpret_cast<unsigned long long*>(reach));
    MGR_LAUNCH_CHECK();
}

void hgs_diag(const DCsr& A, int chunk, double* d, int* flag, hipStream_t s) {
    if (A.nr <= 0) return;
    int G = group_rows(A.max_row);
    MGR_DISPATCH_G4(G, (k_hgs_diag_g<GG><<<grid_for(A.nr, GG), TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, A.v.p, chunk, d,
                                                                              flag)));
    MGR_LAUNCH_CHECK();
}

void label_filter_count(const DCsr& A, const int* label, int* cnt, hipStream_t s) {
    if (A.nr <= 0) return;
    int G = group_rows(A.max_row);
    MGR_DISPATCH_G4(G, (k_label_filter_g<GG, false><<<grid_for(A.nr, GG), TPB, 0, s>>>(
                           A.nr, A.rp.p, A.ci.p, A.v.p, label, cnt, nullptr, nullptr, nullptr)));
    MGR_LAUNCH_CHECK();
}

void label_filter_fill(const DCsr& A, const int* label, DCsr& B, hipStream_t s) {
    if (A.nr <= 0) return;
    int G = group_rows(A.max_row);
    MGR_DISPATCH_G4(G, (k_label_filter_g<GG, true><<<grid_for(A.nr, GG), TPB, 0, s>>>(
                           A.nr, A.rp.p, A.ci.p, A.v.p, label, nullptr, B.rp.p, B.ci.p, B.v.p)));
    MGR_LAUNCH_CHECK();
}

void hgs_tri_count(const DCsr& A, const int* dpos, int chunk, int* w, hipStream_t s) {
    if (A.nr <= 0) return;
    k_hgs_tri_count<<<nblk(A.nr), TPB, 0, s>>>(A.nr, chunk, A.rp.p, A.ci.p, dpos, w);
    MGR_LAUNCH_CHECK();
}

void hgs_tri_fill(const DCsr& A, const int* dpos, const double* d, int chunk, int nchp, int wl, unsigned char* lc,
                  double* lv, int wu, unsigned char* uc, double* uv, double* dT, hipStream_t s) {
    if (A.nr <= 0) return;
    k_hgs_tri_fill<<<nblk((long)nchp * chunk), TPB, 0, s>>>(A.nr, chunk, nchp, A.rp.p, A.ci.p, A.v.p, dpos, d, wl,
                                                            lc, lv, wu, uc, uv, dT);
    MGR_LAUNCH_CHECK();
}

void densify(const DCsr& A, double* dense, hipStream_t s) {
    if (A.nr <= 0) return;
    k_densify<<<A.nr, 128, 0, s>>>(A.nc, A.rp.p, A.ci.p, A.v.p, dense);
    MGR_LAUNCH_CHECK();
}

void dense_gemm(int m, int k, int n, const double* a, const double* b, double* c, hipStream_t s) {
    if ((long)m * n <= 0) return;
    k_dense_gemm<<<nblk((long)m * n), TPB, 0, s>>>(m, k, n, a, b, c);
    MGR_LAUNCH_CHECK();
}

void sparse_dense_add(const DCsr& Q, const double* x, int n, double* t, hipStream_t s) {
    if (Q.nr <= 0 || n <= 0) return;
    k_sparse_dense_add<<<Q.nr, TPB, 0, s>>>(n, Q.rp.p, Q.ci.p, Q.v.p, x, t);
    MGR_LAUNCH_CHECK();
}

void dense_transpose(int n, const double* a, double* t, hipStream_t s) {
    if (n <= 0) return;
    k_dense_transpose<<<nblk((long)n * n), TPB, 0, s>>>(n, a, t);
    MGR_LAUNCH_CHECK();
}

void dense_inverse(int n, double* a, double* inv, int* flag, hipStream_t s) {
    if (n <= 0) return;
    if (n <= 128) {
        k_dense_inverse_small<<<1, 256, 0, s>>>(n, a, inv, flag);
        MGR_LAUNCH_CHECK();
        return;
    }
    DArr<double> fcol((size_t)n, s);
    k_dense_inverse<<<1, 1024, 0, s>>>(n, a, inv, fcol.p, flag);
    MGR_LAUNCH_CHECK();
}

void level_sweep(const DCsr& A, bool fwd, int* lev, int* changed, hipStream_t s) {
    if (A.nr <= 0) return;
    k_level_sweep<<<nblk(A.nr), TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, fwd ? 1 : 0, lev, changed);
    MGR_LAUNCH_CHECK();
}

void level_max(int n, const int* lev, int* out, hipStream_t s) {
    if (n <= 0) return;
    k_level_max<<<nblk(n), TPB, 0, s>>>(n, lev, out);
    MGR_LAUNCH_CHECK();
}

void level_bucket(int n, const int* lev, int* cnt, int* cursor, int* order, hipStream_t s, bool scatter) {
    if (n <= 0) return;
    if (!scatter) k_level_count<<<nblk(n), TPB, 0, s>>>(n, lev, cnt);
    else k_level_scatter<<<nblk(n), TPB, 0, s>>>(n, lev, cursor, order);
    MGR_LAUNCH_CHECK();
}

void diag_pos(const DCsr& A, int* dpos, int* flag, hipStream_t s) {
    if (A.nr <= 0) return;
    k_diag_pos<<<nblk(A.nr), TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, dpos, flag);
    MGR_LAUNCH_CHECK();
}

void ilu_level(int cnt, const int* rows, DCsr& LU, const int* dpos, int* flag, hipStream_t s) {
    if (cnt <= 0) return;
    k_ilu_level<<<nblk(cnt), TPB, 0, s>>>(cnt, rows, LU.rp.p, LU.ci.p, dpos, LU.v.p, flag);
    MGR_LAUNCH_CHECK();
}

void split_count(const DCsr& A, int* nl, int* nu, hipStream_t s) {
    if (A.nr <= 0) return;
    k_split_count<<<nblk(A.nr), TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, nl, nu);
    MGR_LAUNCH_CHECK();
}

void split_fill(const DCsr& A, DCsr& L, DCsr& U, hipStream_t s) {
    if (A.nr <= 0) return;
    k_split_fill<<<nblk(A.nr), TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, A.v.p, L.rp.p, L.ci.p, L.v.p, U.rp.p, U.ci.p, U.v.p);
    MGR_LAUNCH_CHECK();
}

void rj_count(int nC, const DCsr& X, int* len, hipStream_t s) {
    if (nC <= 0) return;
    k_rj_count<<<nblk(nC), TPB, 0, s>>>(nC, X.rp.p, len);
    MGR_LAUNCH_CHECK();
}

void rj_fill(int nC, const DCsr& X, double scale, const int* fmap, const int* cmap, DCsr& R, hipStream_t s) {
    if (nC <= 0) return;
    int G = group_for((X.max_row + FILL_BATCH - 1) / FILL_BATCH);
    MGR_DISPATCH_G4(G, (k_rj_fill_g<GG><<<grid_for(nC, GG), TPB, 0, s>>>(nC, X.rp.p, X.ci.p, X.v.p, scale, fmap,
                                                                          cmap, R.rp.p, R.ci.p, R.v.p, R.vf.p)));
    MGR_LAUNCH_CHECK();
}

void pj_count(int n, const int* isF, const int* lmap, const DCsr& Y, const DCsr& M, int* len, hipStream_t s) {
    if (n <= 0) return;
    k_pj_count<<<nblk(n), TPB, 0, s>>>(n, isF, lmap, Y.rp.p, M.rp.p, len);
    MGR_LAUNCH_CHECK();
}

void pj_fill(int n, int nC, const int* isF, const int* lmap, const DCsr& Y, double yscale, const DCsr& M,
             double mscale, const int* fmap, DCsr& P, hipStream_t s) {
    if (n <= 0) return;
    int G = group_for(Y.max_row < 0 || M.max_row < 0 ? -1 : (Y.max_row + M.max_row + FILL_BATCH - 1) / FILL_BATCH);
    MGR_DISPATCH_G4(G, (k_pj_fill_g<GG><<<grid_for(n, GG), TPB, 0, s>>>(n, nC, isF, lmap, Y.rp.p, Y.ci.p, Y.v.p,
                                                                         yscale, M.rp.p, M.ci.p, M.v.p, mscale,
                                                                         fmap, P.rp.p, P.ci.p, P.v.p, P.vf.p)));
    MGR_LAUNCH_CHECK();
}

void compose_w(const DCsr& A, const double* dinv, double* w, int* bad, hipStream_t s) {
    if (A.nr <= 0) return;
    int G = group_for(A.max_row);
    MGR_DISPATCH_G4(G, (k_compose_w_g<GG><<<grid_for(A.nr, GG), TPB, 0, s>>>(A.nr, A.rp.p, A.ci.p, A.v.p, dinv, w,
                                                                             bad)));
    MGR_LAUNCH_CHECK();
}

void compose_sub(const DCsr& X, const DCsr& Y, const double* rs, const double* cs, double* out, int* bad,
                 hipStream_t s) {
    if (Y.nr <= 0) return;
    if (X.nr != Y.nr || X.nc != Y.nc) throw Error(-6, "internal: composed operator shapes differ");
    int G = group_for(Y.max_row);
    MGR_DISPATCH_G4(G, (k_compose_sub_g<GG><<<grid_for(Y.nr, GG), TPB, 0, s>>>(
                           Y.nr, X.rp.p, X.ci.p, X.v.p, Y.rp.p, Y.ci.p, Y.v.p, rs, cs, out, bad)));
    MGR_LAUNCH_CHECK();
}

void concat_rows(const DCsr& A, const DCsr& B, DCsr& C, hipStream_t s) {
    if (A.nr != B.nr) throw Error(-6, "internal: concatenated operators differ in rows");
    C.alloc(A.nr, A.nc + B.nc, A.nnz + B.nnz, s);
    C.max_row = A.max_row + B.max_row;
    int G = group_for(C.max_row);
    MGR_DISPATCH_G4(G, (k_concat_g<GG><<<grid_for((long)A.nr + 1, GG), TPB, 0, s>>>(
                           A.nr, A.rp.p, A.ci.p, A.v.p, B.rp.p, B.ci.p, B.v.p, A.nc, C.rp.p, C.ci.p, C.v.p)));
    MGR_LAUNCH_CHECK();
}

}  // namespace mgr
