// common.hpp -- device buffers, device CSR container and error handling shared
// by the host orchestration and the kernel launchers of libmgrhip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <utility>

namespace mgr {

// Errors carry one of the MGR_ERR_* codes of mgr.h.
struct Error : public std::runtime_error {
    int code;
    Error(int c, const std::string& m) : std::runtime_error(m), code(c) {}
};

#define MGR_HIP(call)                                                                                 \
    do {                                                                                              \
        hipError_t e_ = (call);                                                                       \
        if (e_ != hipSuccess)                                                                         \
            throw ::mgr::Error(e_ == hipErrorOutOfMemory ? -4 : -2,                                   \
                               std::string(#call) + ": " + hipGetErrorString(e_) + " at " + __FILE__ + \
                                   ":" + std::to_string(__LINE__));                                   \
    } while (0)

#define MGR_LAUNCH_CHECK() MGR_HIP(hipGetLastError())

// Stream-ordered device array (hipMallocAsync / hipFreeAsync on one stream).
template <typename T>
struct DArr {
    T* p = nullptr;
    size_t n = 0;
    hipStream_t s = nullptr;
    DArr() = default;
    DArr(size_t count, hipStream_t st) { alloc(count, st); }
    DArr(const DArr&) = delete;
    DArr& operator=(const DArr&) = delete;
    DArr(DArr&& o) noexcept : p(o.p), n(o.n), s(o.s) { o.p = nullptr; o.n = 0; }
    DArr& operator=(DArr&& o) noexcept {
        if (this != &o) { reset(); p = o.p; n = o.n; s = o.s; o.p = nullptr; o.n = 0; }
        return *this;
    }
    ~DArr() { reset(); }
    void alloc(size_t count, hipStream_t st) {
        reset();
        s = st;
        n = count;
        if (count) MGR_HIP(hipMallocAsync(reinterpret_cast<void**>(&p), count * sizeof(T), st));
    }
    void reset() {
        if (p) (void)hipFreeAsync(p, s);
        p = nullptr;
        n = 0;
    }
    T* get() const { return p; }
    size_t bytes() const { return n * sizeof(T); }
};

// Device CSR matrix (int32 indices).  v holds FP64 values; vf an optional FP32
// copy used by the single-precision apply.
struct DCsr {
    int nr = 0, nc = 0;
    long nnz = 0;
    DArr<int> rp, ci;
    DArr<double> v;
    DArr<float> vf;
    DArr<int> blk;   // row-block boundaries of the CSR-stream SpMV
    int nblk = 0;
    int max_row = -1;  // longest row (-1 = not known yet)
    bool empty() const { return nr == 0 && nnz == 0; }
    void alloc(int rows, int cols, long nz, hipStream_t s) {
        nr = rows;
        nc = cols;
        nnz = nz;
        rp.alloc((size_t)rows + 1, s);
        ci.alloc((size_t)(nz > 0 ? nz : 1), s);
        v.alloc((size_t)(nz > 0 ? nz : 1), s);
        vf.reset();
        blk.reset();
        nblk = 0;
        max_row = -1;
    }
};

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace mgr
