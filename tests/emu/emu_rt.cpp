// Test-side executor: runs HIP kernel source on the CPU.
//
// A block's threads are fibers, each on a stack of its own, switched by a
// small x86-64 routine that saves only the callee-saved registers (ucontext's
// swapcontext also saves the signal mask, a system call on every switch).  A
// fiber runs until it reaches a
// synchronisation point: a wave intrinsic (ballot, readlane, readfirstlane,
// shuffle, wave barrier), which completes when all 64 lanes of its wave have
// reached the same intrinsic, or __syncthreads, which completes when every
// thread of the block has arrived.  Lanes of one wave that reach different
// intrinsics, an intrinsic reached by part of a wave while the rest has
// finished, and a block where nothing can advance are reported and abort the
// process: on the GPU these are divergence bugs or hangs.
#include <hip/hip_runtime.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

// emu_switch(save, to): pushes rbp, rbx, r12-r15, stores the stack pointer
// in *save, loads `to` as the stack pointer, pops the same registers of the
// other fiber and returns into it.
extern "C" void emu_switch(void **save, void *to);
asm(R"(
  .pushsection .text
  .p2align 4
  .globl emu_switch
  .hidden emu_switch
  .type emu_switch,@function
emu_switch:
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
  .size emu_switch, .-emu_switch
  .popsection
)");

namespace {

enum State { RUNNABLE, AT_WAVE, AT_BLOCK, DONE };

struct Fiber {
  void *sp = nullptr;
  unsigned tid = 0;
  State st = RUNNABLE;
  int kind = 0;
  uint64_t val = 0, aux = 0, res = 0;
  char *stack = nullptr;
};

struct Block {
  std::vector<Fiber> f;
  unsigned nthreads = 0, bid = 0, bdim = 0, gdim = 0;
  void *sched = nullptr;
  void (*fn)(void *) = nullptr;
  void *arg = nullptr;
};

Block *g_blk = nullptr;
Fiber *g_cur = nullptr;
const size_t STACK = 256 * 1024;
uint64_t g_syncs = 0;
uint64_t g_sync_limit = 0;  // 0: none

// First code of every fiber (entered by emu_switch's return); never returns.
[[noreturn]] void fiber_entry() {
  g_blk->fn(g_blk->arg);
  g_cur->st = DONE;
  emu_switch(&g_cur->sp, g_blk->sched);
  abort();
}

// A fresh stack as emu_switch leaves one: six zero registers, then
// fiber_entry as the return address, then an empty slot so that fiber_entry
// starts with the stack aligned as after a call (rsp = 8 mod 16).
void *fresh_stack(char *stack) {
  void **sp = (void **)(((uintptr_t)stack + STACK) & ~(uintptr_t)15);
  *--sp = nullptr;
  *--sp = (void *)&fiber_entry;
  for (int i = 0; i < 6; i++) *--sp = nullptr;
  return sp;
}

[[noreturn]] void die(const char *msg, unsigned w) {
  fprintf(stderr, "emu: %s (block %u, wave %u)\n", msg, g_blk->bid, w);
  for (unsigned t = w * 64; t < std::min(g_blk->nthreads, w * 64 + 64); t++) {
    const Fiber &f = g_blk->f[t];
    fprintf(stderr, "  lane %u: state %d kind %d aux %llu\n", t & 63, (int)f.st, f.kind, (unsigned long long)f.aux);
  }
  fflush(stderr);
  abort();
}

void resolve_wave(unsigned w) {
  Block &B = *g_blk;
  const unsigned t0 = w * 64, t1 = std::min(B.nthreads, t0 + 64);
  unsigned at = 0, done = 0;
  for (unsigned t = t0; t < t1; t++) {
    at += B.f[t].st == AT_WAVE;
    done += B.f[t].st == DONE;
  }
  if (at == 0 || at + done < t1 - t0) return;  // lanes still running or waiting on the block
  if (done) die("wave intrinsic reached by part of a wave while other lanes finished", w);
  const int kind = B.f[t0].kind;
  for (unsigned t = t0; t < t1; t++)
    if (B.f[t].kind != kind) die("lanes of one wave at different intrinsics", w);
  uint64_t mask = 0;
  if (kind == EMU_BALLOT)
    for (unsigned t = t0; t < t1; t++)
      if (B.f[t].val) mask |= 1ull << (t - t0);
  for (unsigned t = t0; t < t1; t++) {
    Fiber &f = B.f[t];
    switch (kind) {
      case EMU_BALLOT: f.res = mask; break;
      case EMU_READLANE: {
        if (f.aux != B.f[t0].aux) die("readlane with a lane index that differs between lanes", w);
        unsigned src = t0 + (unsigned)(f.aux & 63);
        if (src >= t1) die("readlane of a lane outside the wave", w);
        f.res = B.f[src].val;
        break;
      }
      case EMU_FIRSTLANE: f.res = B.f[t0].val; break;
      case EMU_WRITELANE: {
        if (f.aux != B.f[t0].aux) die("writelane with a value or lane index that differs between lanes", w);
        f.res = (t - t0) == (unsigned)(f.aux & 63) ? (f.aux >> 32) : f.val;
        break;
      }
      case EMU_SHFL: {
        unsigned src = t0 + ((unsigned)f.aux & 63);
        f.res = src < t1 ? B.f[src].val : 0;
        break;
      }
      case EMU_SHFL_XOR: {
        unsigned src = t0 + (((t - t0) ^ (unsigned)f.aux) & 63);
        f.res = src < t1 ? B.f[src].val : f.val;
        break;
      }
      default: f.res = 0;
    }
    f.st = RUNNABLE;
  }
}

extern "C" char __start_emu_lds[], __stop_emu_lds[];
uint64_t g_fill = 0x9E3779B97F4A7C15ull;
std::vector<char> g_garbage;  // xorshift bytes, twice the LDS section

// LDS holds garbage when a block starts: every __shared__ variable (of all
// kernels: one section) is filled from a random pool at a random offset, so
// that a value left by an earlier block, or a fixed pattern, cannot pass for
// an initialised one.
void scramble_lds() {
  const size_t n = (size_t)(__stop_emu_lds - __start_emu_lds);
  if (g_garbage.size() < 2 * n) {
    g_garbage.resize(2 * n);
    for (auto &c : g_garbage) {
      g_fill ^= g_fill << 13;
      g_fill ^= g_fill >> 7;
      g_fill ^= g_fill << 17;
      c = (char)g_fill;
    }
  }
  g_fill ^= g_fill << 13;
  g_fill ^= g_fill >> 7;
  g_fill ^= g_fill << 17;
  memcpy(__start_emu_lds, g_garbage.data() + (size_t)(g_fill % (n + 1)), n);
}

void run_block(unsigned bid) {
  Block &B = *g_blk;
  B.bid = bid;
  scramble_lds();
  for (unsigned t = 0; t < B.nthreads; t++) {
    Fiber &f = B.f[t];
    f.tid = t;
    f.st = RUNNABLE;
    f.sp = fresh_stack(f.stack);
  }
  const unsigned nw = (B.nthreads + 63) / 64;
  for (;;) {
    bool ran = false;
    for (unsigned t = 0; t < B.nthreads; t++) {
      Fiber &f = B.f[t];
      if (f.st != RUNNABLE) continue;
      ran = true;
      g_cur = &f;
      emu_switch(&B.sched, f.sp);
      g_cur = nullptr;
    }
    for (unsigned w = 0; w < nw; w++) resolve_wave(w);
    unsigned done = 0, atb = 0;
    for (auto &f : B.f) {
      done += f.st == DONE;
      atb += f.st == AT_BLOCK;
    }
    if (done == B.nthreads) return;
    if (atb && atb + done == B.nthreads) {
      if (done) {
        fprintf(stderr, "emu: __syncthreads reached by part of the block while other threads finished (block %u)\n",
                bid);
        abort();
      }
      for (auto &f : B.f) f.st = RUNNABLE;
      continue;
    }
    bool any = false;
    for (auto &f : B.f) any |= f.st == RUNNABLE;
    if (!ran && !any) {
      fprintf(stderr, "emu: no thread can advance in block %u (a hang on the GPU)\n", bid);
      for (unsigned w = 0; w < nw; w++) {
        const Fiber &f = B.f[w * 64];
        fprintf(stderr, "  wave %u lane 0: state %d kind %d\n", w, (int)f.st, f.kind);
      }
      abort();
    }
  }
}

}  // namespace

extern "C" {

uint64_t g_kind_count[8];
uint64_t emu_kind_count(int k) { return k >= 0 && k < 8 ? g_kind_count[k] : 0; }

uint64_t emu_wave_sync(int kind, uint64_t v, uint64_t aux) {
  Fiber *f = g_cur;
  if ((f->tid & 63) == 0 && kind >= 0 && kind < 8) g_kind_count[kind]++;
  if (g_sync_limit && ++g_syncs > g_sync_limit) {
    fprintf(stderr, "emu: sync limit reached (a kernel that does not finish)\n");
    abort();
  }
  f->kind = kind;
  f->val = v;
  f->aux = aux;
  f->st = AT_WAVE;
  emu_switch(&f->sp, g_blk->sched);
  return f->res;
}

void emu_block_sync(void) {
  Fiber *f = g_cur;
  f->st = AT_BLOCK;
  emu_switch(&f->sp, g_blk->sched);
}

unsigned emu_tid(void) { return g_cur->tid; }
unsigned emu_bid(void) { return g_blk->bid; }
unsigned emu_bdim(void) { return g_blk->bdim; }
unsigned emu_gdim(void) { return g_blk->gdim; }
int emu_n_cu(void) { return 2; }

void emu_set_sync_limit(uint64_t n) {
  g_sync_limit = n;
  g_syncs = 0;
}

static uint64_t g_launch_id = 0;
void emu_run_grid(void (*fn)(void *), void *arg, unsigned grid, unsigned block) {
  uint64_t before[8];
  for (int k = 0; k < 8; k++) before[k] = g_kind_count[k];
  if (getenv("EMU_TRACE"))
    fprintf(stderr, "emu: launch %llu grid %u block %u\n", (unsigned long long)g_launch_id, grid, block);
  Block B;
  B.nthreads = block;
  B.bdim = block;
  B.gdim = grid;
  B.fn = fn;
  B.arg = arg;
  B.f.resize(block);
  for (auto &f : B.f) f.stack = (char *)malloc(STACK);
  Block *prev = g_blk;
  g_blk = &B;
  for (unsigned b = 0; b < grid; b++) run_block(b);
  g_blk = prev;
  for (auto &f : B.f) free(f.stack);
  if (getenv("EMU_TRACE"))
    fprintf(stderr, "emu: launch %llu done: ballot %llu readlane %llu firstlane %llu shfl %llu wavebar %llu\n",
            (unsigned long long)g_launch_id++, (unsigned long long)(g_kind_count[1] - before[1]),
            (unsigned long long)(g_kind_count[2] - before[2]), (unsigned long long)(g_kind_count[3] - before[3]),
            (unsigned long long)(g_kind_count[4] - before[4]), (unsigned long long)(g_kind_count[5] - before[5]));
}

}  // extern "C"
