// Scheduler and host API of the SIMT emulation (see simt.h).
#include "simt.h"

#include <algorithm>
#include <vector>

#if defined(__SANITIZE_ADDRESS__)
extern "C" void __sanitizer_start_switch_fiber(void **fake_stack_save, const void *bottom, size_t size);
extern "C" void __sanitizer_finish_switch_fiber(void *fake_stack_save, const void **bottom_old,
                                                size_t *size_old);
#define SIMT_ASAN 1
#else
#define SIMT_ASAN 0
#endif

namespace simt {
namespace {

constexpr int kWave = 64;
constexpr size_t kStack = 256 * 1024;

enum State { kRun = 0, kLaneOp, kBarrier, kDone };

// Context switch without a system call (swapcontext saves the signal mask
// with one): push the callee-saved registers, swap stack pointers, pop.
extern "C" void simt_switch(void **save_sp, void *new_sp);
asm(R"(
    .text
    .globl simt_switch
    .type simt_switch, @function
simt_switch:
    pushq %rbp
    pushq %rbx
    pushq %r12
    pushq %r13
    pushq %r14
    pushq %r15
    movq %rsp, (%rdi)
    movq %rsi, %rsp
    popq %r15
    popq %r14
    popq %r13
    popq %r12
    popq %rbx
    popq %rbp
    ret
    .size simt_switch, .-simt_switch
)");

struct Fiber {
    void *sp = nullptr;   // saved stack pointer while not running
    char *stack = nullptr;
    unsigned tid = 0;
    int state = kRun;
    int kind = 0, param = 0, width = 64;
    uint64_t in = 0, out = 0;
};

void *g_sched_sp = nullptr;
std::vector<Fiber> g_fibers;
Fiber *g_cur = nullptr;
dim3 g_block, g_grid, g_bidx;
std::function<void()> g_body;
unsigned long long g_ops = 0;
void *g_fake = nullptr;
const void *g_sched_bottom = nullptr;
size_t g_sched_size = 0;

void fail(const char *what, unsigned b, int wave)
{
    fprintf(stderr, "simt: %s (block %u, wave %d)\n", what, b, wave);
    fflush(stderr);
    abort();
}

// switch from the scheduler into fiber f, and back when it parks or ends
void run_fiber(Fiber *f)
{
    g_cur = f;
#if SIMT_ASAN
    __sanitizer_start_switch_fiber(&g_fake, f->stack, kStack);
#endif
    simt_switch(&g_sched_sp, f->sp);
#if SIMT_ASAN
    __sanitizer_finish_switch_fiber(g_fake, nullptr, nullptr);
#endif
    g_cur = nullptr;
}

// from the current fiber back to the scheduler
void park()
{
    Fiber *f = g_cur;
#if SIMT_ASAN
    void *fake = nullptr;
    __sanitizer_start_switch_fiber(f->state == kDone ? nullptr : &fake, g_sched_bottom, g_sched_size);
#endif
    simt_switch(&f->sp, g_sched_sp);
#if SIMT_ASAN
    __sanitizer_finish_switch_fiber(fake, &g_sched_bottom, &g_sched_size);
#endif
}

[[noreturn]] void entry()
{
#if SIMT_ASAN
    __sanitizer_finish_switch_fiber(nullptr, &g_sched_bottom, &g_sched_size);
#endif
    g_body();
    g_cur->state = kDone;
    park();
    abort();   // a finished fiber is never resumed
}

// A new fiber's stack: six zero callee-saved registers, then entry as the
// return address of its first switch (16-byte aligned at entry's first
// instruction, as a call leaves it).
void *initial_sp(char *stack)
{
    uintptr_t top = ((uintptr_t)(stack + kStack)) & ~(uintptr_t)15;
    void **sp = (void **)top;
    *--sp = nullptr;                 // alignment slot: entry sees (rsp + 8) % 16 == 0
    *--sp = (void *)&entry;          // return address of the first switch
    for (int i = 0; i < 6; i++) *--sp = nullptr;
    return sp;
}

// every live lane of the wave is parked at a cross-lane operation: check it
// is the same one and hand out the results
void resolve_wave(Fiber *w, int n, unsigned b, int wi)
{
    int first = -1;
    for (int l = 0; l < n; l++)
        if (w[l].state != kDone) {
            first = l;
            break;
        }
    const Fiber &f0 = w[first];
    for (int l = 0; l < n; l++) {
        if (w[l].state == kDone) continue;
        if (w[l].kind != f0.kind || w[l].width != f0.width ||
            ((f0.kind == kShflUp || f0.kind == kShflDown || f0.kind == kShflXor ||
              f0.kind == kReadLane || f0.kind == kDpp) &&
             w[l].param != f0.param))
            fail("lanes of one wave at different cross-lane operations", b, wi);
    }
    g_ops++;
    for (int l = 0; l < n; l++) {
        if (w[l].state == kDone) continue;
        int src = l;
        const int wd = f0.width, base = l - l % wd, ll = l % wd;
        switch (f0.kind) {
        case kShflUp: src = (ll >= w[l].param) ? l - w[l].param : l; break;
        case kShflDown: src = (ll + w[l].param < wd) ? l + w[l].param : l; break;
        case kShflXor: src = base + ((ll ^ w[l].param) % wd); break;
        case kShflIdx: src = base + ((w[l].param % wd + wd) % wd); break;
        case kReadFirst: src = first; break;
        case kReadLane: src = w[l].param; break;
        case kClock: break;
        case kDpp: {
            const int c = w[l].param & 0xFFFF, rows = (w[l].param >> 16) & 0xF, r = l & 15, row = l >> 4;
            if (c > 0x100 && c < 0x110) src = (r + (c - 0x100) < 16) ? l + (c - 0x100) : -1;       // row_shl
            else if (c > 0x110 && c < 0x120) src = (r - (c - 0x110) >= 0) ? l - (c - 0x110) : -1;  // row_shr
            else if (c == 0x130) src = (l + 1 < kWave) ? l + 1 : -1;                              // wave_shl1
            else if (c == 0x138) src = (l >= 1) ? l - 1 : -1;                                       // wave_shr1
            else if (c == 0x142) src = (row >= 1) ? 16 * row - 1 : -1;                             // row_bcast15
            else fail("unsupported DPP control", b, wi);
            if (!((rows >> row) & 1)) src = -1;                                                     // row masked off
            break;
        }
        default: fail("unknown cross-lane operation", b, wi);
        }
        if (f0.kind == kClock) {
            w[l].out = g_ops * 100;   // 100 ticks per resolved operation
        } else if (f0.kind == kDpp) {
            const bool masked = !((((w[l].param >> 16) & 0xF) >> (l >> 4)) & 1);
            if (src < 0 && !masked && (w[l].param >> 20) & 1) {
                w[l].out = 0;                                                 // zero fill
            } else if (src < 0) {
                w[l].out = w[l].in >> 32;                                     // keeps old
            } else {
                if (src >= n || w[src].state == kDone) fail("DPP reads a lane that has exited", b, wi);
                w[l].out = w[src].in & 0xffffffffu;
            }
        } else {
            if (src >= n || w[src].state == kDone) fail("a lane reads a lane that has exited", b, wi);
            w[l].out = w[src].in;
        }
        w[l].state = kRun;
    }
}

}  // namespace

dim3 thread_idx() { return dim3(g_cur->tid, 0, 0); }
dim3 block_idx() { return g_bidx; }
dim3 block_dim() { return g_block; }
dim3 grid_dim() { return g_grid; }
unsigned long long ops_resolved() { return g_ops; }

uint64_t lane_op(int kind, uint64_t bits, int param, int width)
{
    Fiber *f = g_cur;
    f->kind = kind;
    f->in = bits;
    f->param = param;
    f->width = width;
    f->state = kLaneOp;
    park();
    return f->out;
}

void sync_block()
{
    g_cur->state = kBarrier;
    park();
}

void launch(dim3 grid, dim3 block, std::function<void()> body)
{
    const unsigned nt = block.x * block.y * block.z, nb = grid.x * grid.y * grid.z;
    g_block = block;
    g_grid = grid;
    g_body = std::move(body);
    for (unsigned b = 0; b < nb; b++) {
        g_bidx = dim3(b, 0, 0);
        g_fibers.assign(nt, Fiber());
        for (unsigned t = 0; t < nt; t++) {
            Fiber &f = g_fibers[t];
            f.tid = t;
            f.stack = (char *)malloc(kStack);
            f.sp = initial_sp(f.stack);
        }
        for (;;) {
            bool ran = false;
            for (unsigned t = 0; t < nt; t++)
                if (g_fibers[t].state == kRun) {
                    run_fiber(&g_fibers[t]);
                    ran = true;
                }
            bool all_done = true, progress = false;
            for (unsigned t = 0; t < nt; t++) all_done = all_done && g_fibers[t].state == kDone;
            if (all_done) break;
            // waves whose live lanes are all at a cross-lane operation
            for (unsigned w0 = 0; w0 < nt; w0 += kWave) {
                const int n = (int)std::min<unsigned>(kWave, nt - w0);
                int live = 0, at_op = 0;
                for (int l = 0; l < n; l++) {
                    const int st = g_fibers[w0 + l].state;
                    live += st != kDone;
                    at_op += st == kLaneOp;
                }
                if (at_op == 0) continue;
                if (at_op != live) {
                    bool waiting = false;   // some lanes still running: not yet
                    for (int l = 0; l < n; l++) waiting = waiting || g_fibers[w0 + l].state == kRun;
                    if (!waiting) fail("lanes of one wave split between a cross-lane operation and a barrier", b, w0 / kWave);
                    continue;
                }
                resolve_wave(&g_fibers[w0], n, b, w0 / kWave);
                progress = true;
            }
            if (!progress) {
                bool all_barrier = true;
                for (unsigned t = 0; t < nt; t++)
                    all_barrier = all_barrier && (g_fibers[t].state == kBarrier || g_fibers[t].state == kDone);
                if (all_barrier) {
                    for (unsigned t = 0; t < nt; t++)
                        if (g_fibers[t].state == kBarrier) g_fibers[t].state = kRun;
                    progress = true;
                }
            }
            if (!progress && !ran) fail("no thread can proceed (deadlock)", b, -1);
        }
        for (unsigned t = 0; t < nt; t++) free(g_fibers[t].stack);
        g_fibers.clear();
    }
    g_body = nullptr;
}

}  // namespace simt

// ---- host API: device memory is host memory, the stream runs synchronously
struct simt_event {
    unsigned long long ops = 0;
};

static hipError_t g_last = hipSuccess;
hipError_t hipSetDevice(int d) { return d == 0 ? hipSuccess : hipErrorInvalidDevice; }
hipError_t hipGetDevice(int *d)
{
    *d = 0;
    return hipSuccess;
}
hipError_t hipDeviceGetAttribute(int *v, hipDeviceAttribute_t a, int)
{
    *v = (a == hipDeviceAttributeMultiprocessorCount) ? 1 : 100000;   // 1 CU; 100 MHz clock
    return hipSuccess;
}
hipError_t hipHostMalloc(void **p, size_t n, unsigned)
{
    *p = malloc(n);
    return *p ? hipSuccess : hipErrorInvalidValue;
}
hipError_t hipHostFree(void *p)
{
    free(p);
    return hipSuccess;
}
hipError_t hipEventCreate(hipEvent_t *e)
{
    *e = new simt_event();
    return hipSuccess;
}
hipError_t hipEventCreateWithFlags(hipEvent_t *e, unsigned) { return hipEventCreate(e); }
hipError_t hipEventDestroy(hipEvent_t e)
{
    delete e;
    return hipSuccess;
}
hipError_t hipEventRecord(hipEvent_t e, hipStream_t)
{
    e->ops = simt::ops_resolved();
    return hipSuccess;
}
hipError_t hipEventSynchronize(hipEvent_t) { return hipSuccess; }
hipError_t hipEventElapsedTime(float *ms, hipEvent_t a, hipEvent_t b)
{
    *ms = (float)((double)(b->ops - a->ops) * 1e-3);   // 1 us per cross-lane operation
    return hipSuccess;
}
hipError_t hipMemcpyAsync(void *d, const void *s, size_t n, hipMemcpyKind, hipStream_t)
{
    memmove(d, s, n);
    return hipSuccess;
}
hipError_t hipMemcpy(void *d, const void *s, size_t n, hipMemcpyKind k) { return hipMemcpyAsync(d, s, n, k, nullptr); }
hipError_t hipStreamSynchronize(hipStream_t) { return hipSuccess; }
hipError_t hipStreamQuery(hipStream_t) { return hipSuccess; }
hipError_t hipEventQuery(hipEvent_t) { return hipSuccess; }
hipError_t hipGetLastError()
{
    const hipError_t e = g_last;
    g_last = hipSuccess;
    return e;
}
const char *hipGetErrorString(hipError_t e) { return e == hipSuccess ? "no error" : "emulated error"; }
