// Host stand-in for the HIP runtime (see hip/hip_runtime.h): guarded allocations, the fiber
// scheduler that runs a launch block by block, and sequential streams and events.
// TEST INFRASTRUCTURE ONLY.
#include "hip/hip_runtime.h"

#include <map>
#include <unistd.h>

namespace emu {

Fiber *cur = nullptr;
Block *blk = nullptr;
dim3 cur_block, cur_grid, cur_dim;
unsigned char *cur_lds = nullptr;
const void *sched_bottom = nullptr;
size_t sched_size = 0;

// Context switch without a system call: save the callee-saved registers and the FP control words on
// the current stack, store its pointer in *save, continue on next (System V x86-64).
extern "C" void emu_swap(void **save, void *next);
asm(R"(
    .text
    .globl emu_swap
    .type emu_swap, @function
emu_swap:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    subq $8, %rsp
    stmxcsr (%rsp)
    fnstcw 4(%rsp)
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    ldmxcsr (%rsp)
    fldcw 4(%rsp)
    addq $8, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
    .size emu_swap, .-emu_swap
)");

static void *sched_sp = nullptr;
static const std::function<void()> *cur_body = nullptr;
static hipError_t last_error = hipSuccess;

// ---- guarded allocations: [guard][data, tail poisoned][guard] --------------------------------
static const size_t kGuard = size_t(64) << 20;
struct Region {
    char *base;
    size_t total;
};
static std::map<void *, Region> regions;

void *galloc(size_t bytes) {
    const size_t pg = (size_t)sysconf(_SC_PAGESIZE);
    const size_t body = ((bytes ? bytes : 1) + pg - 1) / pg * pg;
    const size_t total = kGuard + body + kGuard;
    char *base = (char *)mmap(nullptr, total, PROT_NONE, MAP_PRIVATE | MAP_ANONYMOUS | MAP_NORESERVE, -1, 0);
    if (base == MAP_FAILED) return nullptr;
    char *data = base + kGuard;
    if (mprotect(data, body, PROT_READ | PROT_WRITE) != 0) {
        munmap(base, total);
        return nullptr;
    }
    // device memory starts with unspecified contents: fill with a signalling pattern (0xFF bytes are
    // NaN in both float and double) so that a read of never-written memory is not silently zero
    std::memset(data, 0xFF, body);
    const size_t tail0 = (bytes + 7) / 8 * 8;
    if (body > tail0) ASAN_POISON_MEMORY_REGION(data + tail0, body - tail0);
    regions[data] = {base, total};
    return data;
}

void gfree(void *p) {
    if (!p) return;
    auto it = regions.find(p);
    if (it == regions.end()) {
        std::fprintf(stderr, "emu: free of an unknown device pointer %p\n", p);
        std::abort();
    }
    const size_t pg = (size_t)sysconf(_SC_PAGESIZE);
    ASAN_UNPOISON_MEMORY_REGION((char *)p, it->second.total - 2 * kGuard);
    (void)pg;
    munmap(it->second.base, it->second.total);
    regions.erase(it);
}

// ---- fibers ------------------------------------------------------------------------------------
void yield() {
    Fiber *f = cur;
    __sanitizer_start_switch_fiber(&f->fake, sched_bottom, sched_size);
    emu_swap(&f->sp, sched_sp);
    __sanitizer_finish_switch_fiber(f->fake, nullptr, nullptr);
}

static void fiber_entry() {
    Fiber *f = cur;
    __sanitizer_finish_switch_fiber(nullptr, &sched_bottom, &sched_size);
    (*cur_body)();
    f->done = true;
    Block *b = blk;
    b->ldone[f->wave * 64 + f->lane] = 1;
    // a finished thread no longer takes part in the barriers
    b->active--;
    if (b->arrived > 0 && b->arrived == b->active) {
        b->arrived = 0;
        b->bgen++;
    }
    b->wactive[f->wave]--;
    if (b->warrived[f->wave] > 0 && b->warrived[f->wave] == b->wactive[f->wave]) {
        b->warrived[f->wave] = 0;
        b->wgen[f->wave]++;
    }
    __sanitizer_start_switch_fiber(nullptr, sched_bottom, sched_size);
    void *dead;
    emu_swap(&dead, sched_sp);  // never resumed
    __builtin_unreachable();
}

// first frame of a fiber: the words emu_swap pops (FP control, six registers) and a return address
static void *fiber_stack_init(char *stack, size_t size) {
    // the last fiber on this stack ended inside fiber_entry, whose frame stays poisoned
    ASAN_UNPOISON_MEMORY_REGION(stack, size);
    uintptr_t top = ((uintptr_t)(stack + size)) & ~(uintptr_t)15;
    uint64_t *sp = (uint64_t *)top;
    *--sp = 0;                           // alignment: fiber_entry starts with rsp = 8 (mod 16)
    *--sp = (uint64_t)(uintptr_t)&fiber_entry;
    for (int i = 0; i < 6; ++i) *--sp = 0;
    uint32_t ctl[2];
    asm volatile("stmxcsr %0" : "=m"(ctl[0]));
    asm volatile("fnstcw %0" : "=m"(ctl[1]));
    *--sp = (uint64_t)ctl[0] | ((uint64_t)(ctl[1] & 0xffff) << 32);
    return sp;
}

static bool runnable(const Fiber &f, const Block &b) {
    if (f.done) return false;
    if (f.wait == 0) return true;
    if (f.wait == 1) return b.bgen != f.gen;
    return b.wgen[f.wave] != f.gen;
}

static std::vector<char *> stacks;
static const size_t kStack = size_t(512) << 10;

void run_launch(const std::function<void()> &body, dim3 grid, dim3 block, size_t shmem) {
    const int nt = (int)(block.x * block.y * block.z);
    if (block.y != 1 || block.z != 1 || nt > 1024 || nt < 1) {
        std::fprintf(stderr, "emu: unsupported block shape %u x %u x %u\n", block.x, block.y, block.z);
        std::abort();
    }
    while ((int)stacks.size() < nt) stacks.push_back((char *)std::malloc(kStack));
    cur_grid = grid;
    cur_dim = block;
    cur_body = &body;
    unsigned char *lds = shmem ? (unsigned char *)galloc(shmem) : nullptr;
    cur_lds = lds;
    Block b;
    b.nthreads = nt;
    b.nwaves = (nt + 63) / 64;
    b.f.resize(nt);
    b.wactive.assign(b.nwaves, 0);
    b.warrived.assign(b.nwaves, 0);
    b.wgen.assign(b.nwaves, 0);
    b.slot[0].assign(b.nwaves * 64, 0);
    b.slot[1].assign(b.nwaves * 64, 0);
    b.ldone.assign(b.nwaves * 64, 1);
    for (unsigned bz = 0; bz < grid.z; ++bz)
        for (unsigned by = 0; by < grid.y; ++by)
            for (unsigned bx = 0; bx < grid.x; ++bx) {
                cur_block = dim3(bx, by, bz);
                b.active = nt;
                b.arrived = 0;
                b.bgen = 0;
                std::fill(b.warrived.begin(), b.warrived.end(), 0);
                std::fill(b.wgen.begin(), b.wgen.end(), 0);
                std::fill(b.ldone.begin(), b.ldone.end(), 1);
                for (int w = 0; w < b.nwaves; ++w) b.wactive[w] = std::min(64, nt - 64 * w);
                for (int t = 0; t < nt; ++t) {
                    Fiber &f = b.f[t];
                    f.tidx = dim3((unsigned)t);
                    f.lane = t & 63;
                    f.wave = t >> 6;
                    f.done = false;
                    f.wait = 0;
                    f.gen = 0;
                    f.stack = stacks[t];
                    f.ssize = kStack;
                    b.ldone[t] = 0;
                    f.sp = fiber_stack_init(f.stack, kStack);
                }
                blk = &b;
                int left = nt;
                while (left > 0) {
                    bool progress = false;
                    for (int t = 0; t < nt; ++t) {
                        Fiber &f = b.f[t];
                        if (!runnable(f, b)) continue;
                        f.wait = 0;
                        cur = &f;
                        void *fake = nullptr;
                        __sanitizer_start_switch_fiber(&fake, f.stack, f.ssize);
                        emu_swap(&sched_sp, f.sp);
                        __sanitizer_finish_switch_fiber(fake, nullptr, nullptr);
                        progress = true;
                        if (f.done) --left;
                    }
                    if (!progress) {
                        std::fprintf(stderr,
                                     "emu: block (%u,%u,%u) deadlocked: %d threads wait at a barrier that the "
                                     "others never reach\n", bx, by, bz, left);
                        std::abort();
                    }
                }
                blk = nullptr;
                cur = nullptr;
            }
    if (lds) gfree(lds);
    cur_lds = nullptr;
}

}  // namespace emu

// ---- runtime API -------------------------------------------------------------------------------
struct emu_stream {
    int id;
};
struct emu_event {
    int recorded;
};

hipError_t hipGetLastError() {
    const hipError_t e = emu::last_error;
    emu::last_error = hipSuccess;
    return e;
}
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulated error"; }
hipError_t hipGetDevice(int *d) {
    *d = 0;
    return hipSuccess;
}
hipError_t hipDeviceSynchronize() { return hipSuccess; }
hipError_t hipMalloc(void **p, size_t bytes) {
    *p = emu::galloc(bytes);
    return *p ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipFree(void *p) {
    emu::gfree(p);
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t bytes, unsigned) {
    *p = std::malloc(bytes ? bytes : 1);
    return *p ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipHostFree(void *p) {
    std::free(p);
    return hipSuccess;
}
hipError_t hipMemset(void *p, int v, size_t bytes) {
    std::memset(p, v, bytes);
    return hipSuccess;
}
hipError_t hipMemsetAsync(void *p, int v, size_t bytes, hipStream_t) { return hipMemset(p, v, bytes); }
hipError_t hipMemcpy(void *dst, const void *src, size_t bytes, hipMemcpyKind) {
    std::memmove(dst, src, bytes);
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *dst, const void *src, size_t bytes, hipMemcpyKind k, hipStream_t) {
    return hipMemcpy(dst, src, bytes, k);
}
hipError_t hipMemcpy2DAsync(void *dst, size_t dpitch, const void *src, size_t spitch, size_t width, size_t height,
                            hipMemcpyKind, hipStream_t) {
    for (size_t r = 0; r < height; ++r)
        std::memmove((char *)dst + r * dpitch, (const char *)src + r * spitch, width);
    return hipSuccess;
}
hipError_t hipStreamCreateWithFlags(hipStream_t *s, unsigned) {
    *s = new emu_stream{1};
    return hipSuccess;
}
hipError_t hipStreamCreate(hipStream_t *s) { return hipStreamCreateWithFlags(s, 0); }
hipError_t hipStreamDestroy(hipStream_t s) {
    delete s;
    return hipSuccess;
}
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamWaitEvent(hipStream_t, hipEvent_t, unsigned) { return hipSuccess; }
hipError_t hipEventCreate(hipEvent_t *e) {
    *e = new emu_event{0};
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e) {
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t) {
    e->recorded = 1;
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t, hipEvent_t) {
    *ms = 0.0f;
    return hipSuccess;
}
hipError_t hipGetSymbolAddress(void **p, const void *symbol) {
    *p = const_cast<void *>(symbol);
    return hipSuccess;
}
