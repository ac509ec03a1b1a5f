// Host stand-in for the HIP runtime: TEST INFRASTRUCTURE ONLY.
//
// The library's kernel and runtime sources are compiled unchanged for the CPU against this header
// (it shadows <hip/hip_runtime.h> on the include path of the host build) and run under
// AddressSanitizer, so that every global-memory and LDS access of every kernel is bounds-checked
// on the host before a kernel reaches the GPU:
//   - device allocations sit in their own mappings with inaccessible guard regions on both sides
//     and a poisoned tail, so an access outside a buffer faults or is reported by ASan;
//   - the dynamic LDS of each launch is such an allocation of exactly the launch's byte count;
//   - every block runs its threads as cooperative fibers (one OS thread): __syncthreads is a
//     block barrier, the DPP lane shifts and __shfl_xor exchange values within a wave of 64;
//   - streams and events are sequential: work runs when it is enqueued, which is one valid order
//     of what the library enqueues (it orders its two streams with events).
// Numerics follow the host's IEEE arithmetic; cosine and reciprocal use the libm forms.
#pragma once

#include <sanitizer/asan_interface.h>
#include <sanitizer/common_interface_defs.h>
#include <sys/mman.h>

#include <algorithm>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <functional>
#include <vector>

#define __global__
#define __device__
#define __host__
#define __forceinline__ inline
#define __noinline__ __attribute__((noinline))
#define __launch_bounds__(...)
#define __shared__ static
#define __align__(n) __attribute__((aligned(n)))

struct dim3 {
    unsigned x = 1, y = 1, z = 1;
    dim3(unsigned a = 1, unsigned b = 1, unsigned c = 1) : x(a), y(b), z(c) {}
};

typedef int hipError_t;
enum { hipSuccess = 0, hipErrorNotReady = 600, hipErrorInvalidValue = 1, hipErrorLaunchFailure = 719 };
typedef struct emu_stream *hipStream_t;
typedef struct emu_event *hipEvent_t;
enum hipMemcpyKind { hipMemcpyHostToHost = 0, hipMemcpyHostToDevice = 1, hipMemcpyDeviceToHost = 2,
                     hipMemcpyDeviceToDevice = 3, hipMemcpyDefault = 4 };
#define hipStreamNonBlocking 1u
#define hipEventDisableTiming 2u
#define hipEventDisableSystemFence 0x20000000u

using std::isfinite;
using std::fabs;
using std::ceil;
using std::floor;
using std::sqrt;

template <typename A, typename B>
inline auto min(A a, B b) -> decltype(a < b ? a : b) { return b < a ? b : a; }
template <typename A, typename B>
inline auto max(A a, B b) -> decltype(a < b ? a : b) { return a < b ? b : a; }

inline float __cosf(float x) { return std::cos(x); }
inline double cospi(double x) { return std::cos(M_PI * x); }
inline float cospif(float x) { return std::cos(float(M_PI) * x); }

namespace emu {

// ---- guarded allocations ----------------------------------------------------------------------
void *galloc(size_t bytes);
void gfree(void *p);

// ---- fibers ----------------------------------------------------------------------------------
struct Fiber {
    void *sp = nullptr;    // saved stack pointer while switched out
    char *stack = nullptr;
    size_t ssize = 0;
    dim3 tidx;
    int lane = 0, wave = 0;
    bool done = false;
    int wait = 0;          // 0 running, 1 block barrier, 2 wave barrier
    unsigned long gen = 0;
    void *fake = nullptr;
};

struct Block {
    std::vector<Fiber> f;
    int nthreads = 0, nwaves = 0;
    int active = 0, arrived = 0;
    unsigned long bgen = 0;
    std::vector<int> wactive, warrived;
    std::vector<unsigned long> wgen;
    std::vector<uint64_t> slot[2];   // wave exchange slots, double-buffered by generation parity
    std::vector<char> ldone;         // lane finished (reads as inactive)
};

extern Fiber *cur;
extern Block *blk;
extern dim3 cur_block, cur_grid, cur_dim;
extern unsigned char *cur_lds;
extern const void *sched_bottom;
extern size_t sched_size;

void yield();

inline void syncthreads() {
    Fiber *f = cur;
    f->wait = 1;
    f->gen = blk->bgen;
    if (++blk->arrived == blk->active) {
        blk->arrived = 0;
        blk->bgen++;
    }
    yield();
}

inline void wave_barrier() {
    Fiber *f = cur;
    const int w = f->wave;
    f->wait = 2;
    f->gen = blk->wgen[w];
    if (++blk->warrived[w] == blk->wactive[w]) {
        blk->warrived[w] = 0;
        blk->wgen[w]++;
    }
    yield();
}

// value of lane src (0 if src is off the wave or finished) after every active lane of the wave
// has published its own
inline uint64_t exchange(uint64_t mine, int src_lane, bool *valid) {
    Fiber *f = cur;
    const int w = f->wave, par = (int)(blk->wgen[w] & 1);
    blk->slot[par][f->wave * 64 + f->lane] = mine;
    wave_barrier();
    const int gl = f->wave * 64 + src_lane;
    const bool ok = src_lane >= 0 && src_lane < 64 && gl < blk->nthreads && !blk->ldone[gl];
    if (valid) *valid = ok;
    return ok ? blk->slot[par][gl] : 0;
}

inline unsigned char *dyn_lds() { return cur_lds; }

void run_launch(const std::function<void()> &body, dim3 grid, dim3 block, size_t shmem);

}  // namespace emu

#define threadIdx (emu::cur->tidx)
#define blockIdx (emu::cur_block)
#define gridDim (emu::cur_grid)
#define blockDim (emu::cur_dim)

inline void __syncthreads() { emu::syncthreads(); }

#define __builtin_amdgcn_readfirstlane(v) (v)
#define __builtin_amdgcn_rcpf(v) (1.0f / (v))
#define __builtin_amdgcn_update_dpp(...) emu::dpp(__VA_ARGS__)

namespace emu {
// DPP wave shifts used by the library: 0x138 wave_shr:1 (lane i reads lane i-1), 0x130
// wave_shl:1 (lane i reads lane i+1); a lane with no source reads 0 (bound_ctrl) or old
inline int dpp(int old, int v, int ctrl, int, int, bool bound_ctrl) {
    int src;
    if (ctrl == 0x138) src = cur->lane - 1;
    else if (ctrl == 0x130) src = cur->lane + 1;
    else {
        std::fprintf(stderr, "emu: unsupported DPP control 0x%x\n", ctrl);
        std::abort();
    }
    bool ok = false;
    const uint64_t r = exchange((uint32_t)v, src, &ok);
    if (!ok) return bound_ctrl ? 0 : old;
    return (int)(uint32_t)r;
}
}  // namespace emu

template <typename T>
inline T __shfl_xor(T v, int mask, int width = 64) {
    static_assert(sizeof(T) <= 8, "shfl of a wide type");
    uint64_t bits = 0;
    std::memcpy(&bits, &v, sizeof(T));
    const int lane = emu::cur->lane;
    const int src = (lane & ~(width - 1)) | ((lane ^ mask) & (width - 1));
    bool ok = false;
    const uint64_t r = emu::exchange(bits, src, &ok);
    T out;
    if (!ok) return v;
    std::memcpy(&out, &r, sizeof(T));
    return out;
}

// one OS thread runs every fiber: plain read-modify-write is atomic here
template <typename T> inline T atomicMin(T *p, T v) { T o = *p; if (v < o) *p = v; return o; }
template <typename T> inline T atomicMax(T *p, T v) { T o = *p; if (v > o) *p = v; return o; }
template <typename T> inline T atomicOr(T *p, T v) { T o = *p; *p = o | v; return o; }
template <typename T> inline T atomicAdd(T *p, T v) { T o = *p; *p = o + v; return o; }

// ---- runtime API ------------------------------------------------------------------------------
hipError_t hipGetLastError();
const char *hipGetErrorString(hipError_t e);
hipError_t hipGetDevice(int *d);
hipError_t hipDeviceSynchronize();
hipError_t hipMalloc(void **p, size_t bytes);
template <typename T> inline hipError_t hipMalloc(T **p, size_t bytes) { return hipMalloc((void **)p, bytes); }
hipError_t hipFree(void *p);
hipError_t hipHostMalloc(void **p, size_t bytes, unsigned flags = 0);
template <typename T> inline hipError_t hipHostMalloc(T **p, size_t bytes, unsigned flags = 0) {
    return hipHostMalloc((void **)p, bytes, flags);
}
hipError_t hipHostFree(void *p);
hipError_t hipMemset(void *p, int v, size_t bytes);
hipError_t hipMemsetAsync(void *p, int v, size_t bytes, hipStream_t s = nullptr);
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind k);
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind k, hipStream_t s = nullptr);
hipError_t hipMemcpy2DAsync(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width, size_t height,
                            hipMemcpyKind k, hipStream_t s = nullptr);
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned flags);
hipError_t hipStreamCreate(hipStream_t *s);
hipError_t hipStreamDestroy(hipStream_t s);
hipError_t hipStreamSynchronize(hipStream_t s);
hipError_t hipStreamWaitEvent(hipStream_t s, hipEvent_t e, unsigned flags);
hipError_t hipEventCreate(hipEvent_t *e);
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned flags);
hipError_t hipEventDestroy(hipEvent_t e);
hipError_t hipEventRecord(hipEvent_t e, hipStream_t s = nullptr);
hipError_t hipEventSynchronize(hipEvent_t e);
hipError_t hipEventQuery(hipEvent_t e);
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b);
#define HIP_SYMBOL(x) ((const void *)&(x))
hipError_t hipGetSymbolAddress(void **p, const void *symbol);

#define hipLaunchKernelGGL(kernel, grid, block, shmem, stream, ...)                                  \
    emu::run_launch([&]() { (kernel)(__VA_ARGS__); }, dim3(grid), dim3(block), (size_t)(shmem))
