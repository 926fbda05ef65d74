// common.hpp -- device buffers, device CSR container and error handling shared
// by the host orchestration and the kernel launchers of libmgrhip.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <map>
#include <stdexcept>
#include <string>
#include <utility>
#include <vector>

#include "mgr.h"

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

// Set for the duration of a call that must not allocate device memory (the
// no-allocation apply): an allocation then fails with an error instead of
// reaching the runtime.
inline thread_local bool tl_noalloc = false;
inline void check_may_allocate() {
    if (tl_noalloc) throw Error(-1, "internal: a device allocation was requested by a call that allocates nothing");
}

// Stream-ordered block cache of one solver context.  A setup makes hundreds of
// short-lived device arrays; handing their blocks back to a free list (by size
// class) and out again to later allocations on the same stream costs a map
// lookup instead of a runtime call.  Reuse needs no synchronisation because all
// of a context's device work is ordered on its one stream.  The blocks stay
// with the context until it is destroyed.
struct BlockCache {
    hipStream_t s = nullptr;
    // the caller's device memory provider, if one was given to mgr_create
    mgr_alloc_fn af = nullptr;
    mgr_free_fn ff = nullptr;
    void* actx = nullptr;
    std::multimap<size_t, void*> free_;
    std::vector<void*> owned_;
    // 256-byte granules up to 4 KiB, then four classes per power of two
    static size_t size_class(size_t bytes) {
        if (bytes <= 4096) return (bytes + 255) & ~size_t(255);
        size_t p = 4096;
        while (p * 2 < bytes) p *= 2;
        size_t step = p / 4;
        return (bytes + step - 1) / step * step;
    }
    void* get(size_t bytes, size_t& cls) {
        check_may_allocate();
        cls = size_class(bytes);
        auto it = free_.find(cls);
        if (it != free_.end()) {
            void* q = it->second;
            free_.erase(it);
            return q;
        }
        void* q = nullptr;
        if (af) {
            q = af(cls, (void*)s, actx);
            if (!q) throw Error(MGR_ERR_OOM, "the caller's allocator returned no memory for " + std::to_string(cls) +
                                                 " bytes");
        } else {
            MGR_HIP(hipMallocAsync(&q, cls, s));
        }
        owned_.push_back(q);
        return q;
    }
    void put(void* q, size_t cls) { free_.emplace(cls, q); }
    // every block goes back to where it came from (the caller has synchronised s)
    void release() {
        for (void* q : owned_) {
            if (ff) ff(q, (void*)s, actx);
            else (void)hipFreeAsync(q, s);
        }
        owned_.clear();
        free_.clear();
    }
    ~BlockCache() { release(); }
};

// The cache that device arrays allocated by the current thread draw from (set
// for the duration of a library call on a context; null elsewhere).
inline thread_local BlockCache* tl_cache = nullptr;

// Stream-ordered device array: from the current context's block cache when one
// is active on this stream, else hipMallocAsync / hipFreeAsync.
template <typename T>
struct DArr {
    T* p = nullptr;
    size_t n = 0;
    hipStream_t s = nullptr;
    BlockCache* cache = nullptr;
    size_t cls = 0;
    DArr() = default;
    DArr(size_t count, hipStream_t st) { alloc(count, st); }
    DArr(const DArr&) = delete;
    DArr& operator=(const DArr&) = delete;
    DArr(DArr&& o) noexcept : p(o.p), n(o.n), s(o.s), cache(o.cache), cls(o.cls) {
        o.p = nullptr;
        o.n = 0;
        o.cache = nullptr;
    }
    DArr& operator=(DArr&& o) noexcept {
        if (this != &o) {
            reset();
            p = o.p; n = o.n; s = o.s; cache = o.cache; cls = o.cls;
            o.p = nullptr; o.n = 0; o.cache = nullptr;
        }
        return *this;
    }
    ~DArr() { reset(); }
    void alloc(size_t count, hipStream_t st) {
        reset();
        s = st;
        n = count;
        if (!count) return;
        check_may_allocate();
        if (tl_cache && tl_cache->s == st) {
            cache = tl_cache;
            p = static_cast<T*>(cache->get(count * sizeof(T), cls));
        } else {
            MGR_HIP(hipMallocAsync(reinterpret_cast<void**>(&p), count * sizeof(T), st));
        }
    }
    void reset() {
        if (p) {
            if (cache) cache->put(p, cls);
            else (void)hipFreeAsync(p, s);
        }
        p = nullptr;
        n = 0;
        cache = nullptr;
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
    DArr<int> bpos;  // the entry offset of each boundary (rp[blk[b]])
    int nblk = 0;
    // sliced ELL copy for SpMVs on operators with short, fairly uniform rows:
    // slices of one workgroup's rows, each slot-major with the slice's own
    // width (esw, in slots) and a fixed stride of ew slots per row; ew = the
    // longest row (0 = no copy)
    DArr<int> eci, esw;
    DArr<double> ev;
    DArr<float> evf;
    int ew = 0;
    int ell_state = 0;   // 0 = not decided, 1 = the copy pays, -1 = it does not
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
        bpos.reset();
        nblk = 0;
        eci.reset();
        esw.reset();
        ev.reset();
        evf.reset();
        ew = 0;
        ell_state = 0;
        max_row = -1;
    }
};

inline int ceil_div(long a, long b) { return (int)((a + b - 1) / b); }

}  // namespace mgr
