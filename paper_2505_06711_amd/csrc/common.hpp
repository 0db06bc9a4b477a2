// Runtime plumbing shared by the library's translation units: status codes carried by
// exceptions inside the library (never across the C ABI), device buffers, launch checks.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <cstdio>
#include <stdexcept>
#include <string>
#include <vector>

#include "reann.h"

namespace reann {

struct Error : std::runtime_error {
    reann_status code;
    Error(reann_status c, const std::string &m) : std::runtime_error(m), code(c) {}
};

[[noreturn]] inline void fail(reann_status c, const std::string &m) { throw Error(c, m); }

inline void hip_check(hipError_t e, const char *what, const char *file, int line) {
    if (e != hipSuccess) {
        char buf[512];
        std::snprintf(buf, sizeof buf, "%s failed at %s:%d: %s", what, file, line, hipGetErrorString(e));
        if (e == hipErrorOutOfMemory) throw Error(REANN_E_NOMEM, buf);
        throw Error(REANN_E_DEVICE, buf);
    }
}
#define HIP_OK(x) ::reann::hip_check((x), #x, __FILE__, __LINE__)
#define LAUNCH_OK(name) ::reann::hip_check(hipGetLastError(), name, __FILE__, __LINE__)

// Bump allocator over device memory the library does not allocate (the static scratch of the
// allocation-free entry point).  While one is installed on a thread, every DevBuf that grows on
// that thread takes its memory from it, 256-byte aligned, instead of hipMalloc, and never frees
// it; running out throws REANN_E_CAPACITY.
struct Arena {
    char *base = nullptr;
    size_t cap = 0, used = 0;
};
inline Arena *&current_arena() {
    static thread_local Arena *a = nullptr;
    return a;
}

// Owning device allocation that only grows.  A buffer that has to grow again takes a quarter
// more than asked for: sizes that follow a moving system (ghost and pair counts after a list
// rebuild) then stop reallocating after a few rebuilds, and hipFree, which waits for the whole
// device, stays out of the steady state.
struct DevBuf {
    void *p = nullptr;
    size_t bytes = 0;
    bool owned = true;   // false: memory of an Arena, not freed here
    DevBuf() = default;
    DevBuf(const DevBuf &) = delete;
    DevBuf &operator=(const DevBuf &) = delete;
    DevBuf(DevBuf &&o) noexcept : p(o.p), bytes(o.bytes), owned(o.owned) { o.p = nullptr; o.bytes = 0; }
    DevBuf &operator=(DevBuf &&o) noexcept {
        if (this != &o) {
            release();
            p = o.p; bytes = o.bytes; owned = o.owned;
            o.p = nullptr; o.bytes = 0;
        }
        return *this;
    }
    ~DevBuf() { release(); }
    void release() {
        if (p && owned) (void)hipFree(p);
        p = nullptr;
        bytes = 0;
        owned = true;
    }
    void *ensure(size_t n) {
        if (n == 0) n = 256;
        if (n > bytes) {
            const bool regrow = p != nullptr;
            release();
            if (Arena *a = current_arena()) {
                const size_t off = (a->used + 255) & ~(size_t)255;
                if (off > a->cap || n > a->cap - off)
                    throw Error(REANN_E_CAPACITY, "the evaluation needs more device memory than the " +
                                                      std::to_string(a->cap >> 20) + " MiB of static scratch");
                p = a->base + off;
                a->used = off + n;
                owned = false;
            } else {
                if (regrow) n += n / 4;
                HIP_OK(hipMalloc(&p, n));
            }
            bytes = n;
        }
        return p;
    }
    template <class T> T *as() const { return static_cast<T *>(p); }
};

// A pinned host word that device-to-host copies write (a device-side check read later, once
// the stream has been waited for anyway).
struct PinnedWord {
    int32_t *p = nullptr;
    PinnedWord() = default;
    PinnedWord(const PinnedWord &) = delete;
    PinnedWord &operator=(const PinnedWord &) = delete;
    ~PinnedWord() {
        if (p) (void)hipHostFree(p);
    }
    int32_t *get() {
        if (!p) HIP_OK(hipHostMalloc((void **)&p, 64, hipHostMallocDefault));
        return p;
    }
    double *get_double() { return reinterpret_cast<double *>(get()); }   // the 64 bytes as doubles
};

template <class T> struct DArr {
    DevBuf b;
    size_t n = 0;
    T *resize(size_t count) {
        b.ensure(count * sizeof(T));
        n = count;
        return b.as<T>();
    }
    T *ptr() const { return b.as<T>(); }
    size_t bytes() const { return b.bytes; }
};

inline int grid_for(int64_t n, int block) { return (int)((n + block - 1) / block); }

// Parameters of the (L, K) pairs the kernels are compiled for.
constexpr int n_lambda(int L) { return (L + 1) * (L + 2) * (L + 3) / 6; }
constexpr int n_feat(int L, int K) { return (L + 1) * K * (K + 1) / 2; }

}  // namespace reann
