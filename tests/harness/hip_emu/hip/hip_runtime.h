// Host emulation of the part of the HIP device and runtime surface that the
// batched-tube kernels use (test infrastructure only; never linked into the
// library).  A kernel launch runs its blocks one after another; the threads of
// a block are fibers (ucontext) of one host thread, switched at every barrier:
//   - __syncthreads is a barrier of the block's live threads;
//   - the wave operations (__ballot, __shfl, __shfl_xor) exchange values
//     through a barrier of the wave's live threads (64 per wave), so a wave
//     operation that some live lane of the wave does not reach is reported
//     instead of silently reading a stale value;
//   - emu::wave_sync() marks a point where a kernel relies on the lanes of a
//     wave running in lockstep (a test inserts it into its copy of a kernel);
//   - dynamic LDS is a heap buffer of exactly the launch's size and device
//     allocations are heap buffers of exactly their size, so AddressSanitizer
//     reports any access past either; both start filled with 0xff bytes (NaN
//     doubles), as uninitialised memory;
//   - a launch with more dynamic LDS than the 64 KB a block may use, or more
//     than 1024 threads, is refused with a message.
// When no fiber of a block can run and some have not finished (a barrier
// that not every live thread reaches), the emulation stops with the name and
// arrival count of each waiting barrier.
#pragma once

#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <functional>
#include <vector>

#include <ucontext.h>
#if defined(__SANITIZE_ADDRESS__)
#include <sanitizer/common_interface_defs.h>
#endif

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __constant__
#define __shared__
#define __launch_bounds__(...)
// the device's reciprocal and reciprocal square root estimates; the kernels
// refine or certify every use, so a correctly rounded value serves
#define __builtin_amdgcn_rcp(x) (1.0 / (x))
#define __builtin_amdgcn_rsq(x) (1.0 / sqrt(x))

typedef int hipError_t;
enum {
    hipSuccess = 0,
    hipErrorInvalidValue = 1,
    hipErrorOutOfMemory = 2,
    hipErrorInvalidConfiguration = 9,
    hipErrorNotSupported = 801
};
typedef void* hipStream_t;
typedef void* hipEvent_t;
typedef void* hipGraph_t;
typedef void* hipGraphExec_t;
enum hipMemcpyKind {
    hipMemcpyHostToHost,
    hipMemcpyHostToDevice,
    hipMemcpyDeviceToHost,
    hipMemcpyDeviceToDevice,
    hipMemcpyDefault
};
#define hipStreamNonBlocking 1u
#define hipStreamCaptureModeThreadLocal 1

struct hipDeviceProp_t {
    int multiProcessorCount;
    char gcnArchName[256];
};

struct dim3 {
    unsigned x, y, z;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

namespace emu {

// launch parameters the emulated device reports
inline int g_cus = 4;
inline int g_occ = 2;
inline hipError_t g_last_error = hipSuccess;
constexpr size_t kFiberStack = 64 * 1024;

enum FiberState { RUNNABLE, BLOCKED, DONE };
struct Fiber {
    ucontext_t uc;
    char* stack = nullptr;
    FiberState st = RUNNABLE;
};

struct Barrier {
    int expected = 0, count = 0;
    const char* what = "";
    std::vector<int> waiters;
    void init(int n, const char* w) {
        expected = n;
        count = 0;
        what = w;
        waiters.clear();
    }
};

struct Wave {
    Barrier bar;
    uint64_t slot[64];
    bool live[64];
};

struct Block {
    unsigned bid;
    dim3 grid, block;
    Barrier bar;
    std::vector<Wave> waves;
    void* smem;
    std::vector<Fiber> fibers;
    ucontext_t main;
    int cur = -1;
    std::function<void()> body;
#if defined(__SANITIZE_ADDRESS__)
    void* fake = nullptr;
    const void* main_bottom = nullptr;
    size_t main_size = 0;
#endif
};
inline Block* blk_ = nullptr;

// fiber stacks, allocated once and reused by every block of every launch
struct StackPool {
    std::vector<char*> s;
    ~StackPool() {
        for (char* p : s) free(p);
    }
};
inline char* fiber_stack(unsigned t) {
    static StackPool pool;
    while (pool.s.size() <= t) pool.s.push_back((char*)malloc(kFiberStack));
    return pool.s[t];
}

inline void switch_to_fiber(Block* b, int i) {
    b->cur = i;
#if defined(__SANITIZE_ADDRESS__)
    __sanitizer_start_switch_fiber(&b->fake, b->fibers[i].stack, kFiberStack);
#endif
    swapcontext(&b->main, &b->fibers[i].uc);
#if defined(__SANITIZE_ADDRESS__)
    __sanitizer_finish_switch_fiber(b->fake, nullptr, nullptr);
#endif
}

// the running fiber gives the host thread back to its block's scheduler
inline void yield_fiber() {
    Block* b = blk_;
    Fiber& me = b->fibers[b->cur];
#if defined(__SANITIZE_ADDRESS__)
    void* fake = nullptr;
    __sanitizer_start_switch_fiber(me.st == DONE ? nullptr : &fake, b->main_bottom, b->main_size);
#endif
    swapcontext(&me.uc, &b->main);
#if defined(__SANITIZE_ADDRESS__)
    __sanitizer_finish_switch_fiber(fake, &b->main_bottom, &b->main_size);
#endif
}

inline void release(Barrier& bar) {
    for (int w : bar.waiters) blk_->fibers[w].st = RUNNABLE;
    bar.waiters.clear();
    bar.count = 0;
}

inline void barrier_wait(Barrier& bar) {
    Block* b = blk_;
    if (++bar.count == bar.expected) {
        release(bar);
        return;
    }
    b->fibers[b->cur].st = BLOCKED;
    bar.waiters.push_back(b->cur);
    yield_fiber();
}

// a thread left the kernel: later barriers wait for one thread fewer
inline void barrier_drop(Barrier& bar) {
    --bar.expected;
    if (bar.count > 0 && bar.count == bar.expected) release(bar);
}

struct Idx3 {
    unsigned x, y, z;
};
inline unsigned tid_() { return (unsigned)blk_->cur; }
inline Idx3 thread_idx() { return {tid_(), 0u, 0u}; }
inline Idx3 block_idx() { return {blk_->bid, 0u, 0u}; }
inline Idx3 block_dim() { return {blk_->block.x, 1u, 1u}; }
inline Idx3 grid_dim() { return {blk_->grid.x, 1u, 1u}; }
inline void* dyn_smem() { return blk_->smem; }

inline Wave& wave() { return blk_->waves[tid_() / 64]; }
inline int lane() { return (int)(tid_() % 64); }

// every live lane of the wave deposits v; returns after all have
inline void deposit(uint64_t v) {
    Wave& w = wave();
    w.slot[lane()] = v;
    barrier_wait(w.bar);
}
inline void release_wave() { barrier_wait(wave().bar); }

// a point where the kernel relies on the lanes of a wave running in
// lockstep (every lane's earlier LDS operations precede any lane's later
// ones): all live lanes of the wave meet here
inline void wave_sync() { barrier_wait(wave().bar); }

inline uint64_t fetch(int src) {
    Wave& w = wave();
    if (!w.live[src]) {
        fprintf(stderr, "emulation: lane %d of block %u reads lane %d, which has left the kernel\n",
                lane(), blk_->bid, src);
        abort();
    }
    return w.slot[src];
}

template <class T>
uint64_t to_bits(T v) {
    static_assert(sizeof(T) <= 8, "wave exchange of at most 8 bytes");
    uint64_t r = 0;
    memcpy(&r, &v, sizeof(T));
    return r;
}
template <class T>
T from_bits(uint64_t r) {
    T v;
    memcpy(&v, &r, sizeof(T));
    return v;
}

template <class T>
T atomic_max(T* p, T v) {
    const T old = *p;
    if (old < v) *p = v;
    return old;
}

inline void fiber_entry() {
    Block* b = blk_;
#if defined(__SANITIZE_ADDRESS__)
    __sanitizer_finish_switch_fiber(nullptr, &b->main_bottom, &b->main_size);
#endif
    const int t = b->cur;
    b->body();
    Wave& w = b->waves[t / 64];
    w.live[t % 64] = false;
    barrier_drop(w.bar);
    barrier_drop(b->bar);
    b->fibers[t].st = DONE;
    yield_fiber();  // never resumed
}

template <class... KArgs, class... Args>
void launch(void (*k)(KArgs...), dim3 g, dim3 b, size_t shm, Args... args) {
    if (b.x == 0 || b.x > 1024 || b.y != 1 || b.z != 1 || g.y != 1 || g.z != 1 || g.x == 0 ||
        shm > 64 * 1024) {
        fprintf(stderr, "emulation: launch refused (grid %u, block %u, dynamic LDS %zu B)\n", g.x,
                b.x, shm);
        g_last_error = hipErrorInvalidConfiguration;
        return;
    }
    for (unsigned bid = 0; bid < g.x; ++bid) {
        Block blk;
        blk.bid = bid;
        blk.grid = g;
        blk.block = b;
        blk.bar.init((int)b.x, "__syncthreads");
        const unsigned nw = (b.x + 63) / 64;
        blk.waves = std::vector<Wave>(nw);
        for (unsigned w = 0; w < nw; ++w) {
            const unsigned nt = (w + 1) * 64 <= b.x ? 64 : b.x - w * 64;
            blk.waves[w].bar.init((int)nt, "wave operation");
            for (unsigned l = 0; l < 64; ++l) blk.waves[w].live[l] = l < nt;
        }
        blk.smem = shm ? malloc(shm) : nullptr;
        if (shm) memset(blk.smem, 0xff, shm);
        blk.body = [k, args...]() { k(args...); };
        blk.fibers = std::vector<Fiber>(b.x);
        blk_ = &blk;
        for (unsigned t = 0; t < b.x; ++t) {
            Fiber& f = blk.fibers[t];
            f.stack = fiber_stack(t);
            getcontext(&f.uc);
            f.uc.uc_stack.ss_sp = f.stack;
            f.uc.uc_stack.ss_size = kFiberStack;
            f.uc.uc_link = nullptr;
            makecontext(&f.uc, fiber_entry, 0);
        }
        // round-robin over the runnable fibers until every one has finished
        for (;;) {
            bool all_done = true, ran = false;
            for (unsigned t = 0; t < b.x; ++t) {
                if (blk.fibers[t].st == DONE) continue;
                all_done = false;
                if (blk.fibers[t].st != RUNNABLE) continue;
                ran = true;
                switch_to_fiber(&blk, (int)t);
            }
            if (all_done) break;
            if (!ran) {
                fprintf(stderr, "emulation: block %u cannot proceed: %s %d of %d arrived",
                        bid, blk.bar.what, blk.bar.count, blk.bar.expected);
                for (unsigned w = 0; w < nw; ++w)
                    fprintf(stderr, "; wave %u %s %d of %d", w, blk.waves[w].bar.what,
                            blk.waves[w].bar.count, blk.waves[w].bar.expected);
                fprintf(stderr, "\n");
                abort();
            }
        }
        free(blk.smem);
        blk_ = nullptr;
    }
}

}  // namespace emu

#define threadIdx (emu::thread_idx())
#define blockIdx (emu::block_idx())
#define blockDim (emu::block_dim())
#define gridDim (emu::grid_dim())

inline void __syncthreads() { emu::barrier_wait(emu::blk_->bar); }

inline unsigned long long __ballot(int pred) {
    emu::deposit(pred ? 1u : 0u);
    emu::Wave& w = emu::wave();
    unsigned long long m = 0;
    for (int l = 0; l < 64; ++l)
        if (w.live[l] && w.slot[l]) m |= 1ull << l;
    emu::release_wave();
    return m;
}

template <class T>
T __shfl(T var, int src, int width = 64) {
    emu::deposit(emu::to_bits(var));
    const int base = emu::lane() / width * width;
    const T r = emu::from_bits<T>(emu::fetch(base + ((src % width) + width) % width));
    emu::release_wave();
    return r;
}

template <class T>
T __shfl_xor(T var, int mask, int width = 64) {
    emu::deposit(emu::to_bits(var));
    const int src = emu::lane() ^ mask;
    const int base = emu::lane() / width * width;
    const T r = emu::from_bits<T>(emu::fetch(src < base + width ? src : emu::lane()));
    emu::release_wave();
    return r;
}

inline int __ffsll(long long x) { return __builtin_ffsll(x); }
inline int __ffsll(unsigned long long x) { return __builtin_ffsll((long long)x); }
inline long long __double_as_longlong(double x) { return emu::from_bits<long long>(emu::to_bits(x)); }
inline double __longlong_as_double(long long x) { return emu::from_bits<double>(emu::to_bits(x)); }

inline unsigned long long atomicMax(unsigned long long* p, unsigned long long v) {
    return emu::atomic_max(p, v);
}
inline int atomicMax(int* p, int v) { return emu::atomic_max(p, v); }

#define hipLaunchKernelGGL(K, G, B, S, ST, ...) \
    emu::launch(K, dim3(G), dim3(B), (size_t)(S), __VA_ARGS__)

// ---- runtime ---------------------------------------------------------------
inline hipError_t hipMalloc(void** p, size_t n) {
    *p = malloc(n ? n : 1);
    if (*p == nullptr) return hipErrorOutOfMemory;
    memset(*p, 0xff, n);
    return hipSuccess;
}
template <class T>
hipError_t hipMalloc(T** p, size_t n) {
    return hipMalloc((void**)p, n);
}
inline hipError_t hipFree(void* p) {
    free(p);
    return hipSuccess;
}
inline hipError_t hipMemcpy(void* d, const void* s, size_t n, hipMemcpyKind) {
    memmove(d, s, n);
    return hipSuccess;
}
inline hipError_t hipGetLastError() {
    const hipError_t e = emu::g_last_error;
    emu::g_last_error = hipSuccess;
    return e;
}
inline hipError_t hipDeviceSynchronize() { return hipSuccess; }
inline hipError_t hipGetDevice(int* d) {
    *d = 0;
    return hipSuccess;
}
inline hipError_t hipGetDeviceProperties(hipDeviceProp_t* p, int) {
    p->multiProcessorCount = emu::g_cus;
    strcpy(p->gcnArchName, "host-emulation");
    return hipSuccess;
}
template <class F>
hipError_t hipOccupancyMaxActiveBlocksPerMultiprocessor(int* occ, F, int, size_t) {
    *occ = emu::g_occ;
    return hipSuccess;
}
inline hipError_t hipStreamCreateWithFlags(hipStream_t* s, unsigned) {
    *s = nullptr;
    return hipSuccess;
}
inline hipError_t hipStreamDestroy(hipStream_t) { return hipSuccess; }
// graph capture is not emulated (launches run at once): refuse it
inline hipError_t hipStreamBeginCapture(hipStream_t, int) { return hipErrorNotSupported; }
inline hipError_t hipStreamEndCapture(hipStream_t, hipGraph_t*) { return hipErrorNotSupported; }
inline hipError_t hipGraphInstantiate(hipGraphExec_t*, hipGraph_t, void*, void*, size_t) {
    return hipErrorNotSupported;
}
inline hipError_t hipGraphLaunch(hipGraphExec_t, hipStream_t) { return hipErrorNotSupported; }
inline hipError_t hipGraphExecDestroy(hipGraphExec_t) { return hipSuccess; }
inline hipError_t hipGraphDestroy(hipGraph_t) { return hipSuccess; }
inline hipError_t hipEventCreate(hipEvent_t* e) {
    *e = nullptr;
    return hipSuccess;
}
inline hipError_t hipEventDestroy(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventRecord(hipEvent_t, hipStream_t) { return hipSuccess; }
inline hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
inline hipError_t hipEventElapsedTime(float* ms, hipEvent_t, hipEvent_t) {
    *ms = 1.0f;
    return hipSuccess;
}
