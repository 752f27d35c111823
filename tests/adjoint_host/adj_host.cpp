// Host emulation of the adjoint's workgroup tasks, for tests only.
//
// The library runs every task of paper_1901_06101_amd/csrc/hb_adj.h on one
// GPU workgroup.  This file compiles the same task code for the host and
// runs each workgroup as `nt` operating-system threads that meet at a
// std::barrier wherever the device code calls __syncthreads(), in the
// launch order the library uses (adj_execute).  It checks the tasks'
// arithmetic, indexing and barrier placement against the oracle on the CPU;
// it is not linked into the library, which has no host path.
//
// A second mode runs the nt lanes as fibers (ucontext) on one thread, which
// makes the GPU's 256 lanes affordable: each lane runs until its next
// barrier, and a barrier that some lanes reach while others have finished
// the task (a barrier inside lane-dependent control flow, which would hang
// a GPU workgroup) is reported instead of deadlocking.
#include <ucontext.h>

#include <barrier>
#include <chrono>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <thread>
#include <vector>

#include "../../paper_1901_06101_amd/csrc/hb_adj_plan.h"

namespace {

struct Fibers;

struct WgHost {
  int tid, nt;
  double* red;
  std::barrier<>* bar;
  Fibers* fib;
  void sync();
};

// One workgroup's lanes as fibers: the scheduler resumes every lane in
// turn; a lane runs until it reaches a barrier or ends the task.
struct Fibers {
  static constexpr size_t kStack = 256 * 1024;
  ucontext_t sched;
  std::vector<ucontext_t> ctx;
  std::vector<std::vector<char>> stack;
  std::vector<int> state;  // 0 running, 1 at a barrier, 2 done
  const AdjArgs* a = nullptr;
  double* red = nullptr;
  int nt = 0, kind = 0, task = 0, cur = 0;
  int64_t barriers = 0;
  double crit_ns = 0.0;  // sum over barrier intervals of the slowest lane's segment
  bool diverged = false;

  static thread_local Fibers* self;

  static void entry() {
    Fibers* f = self;
    const int t = f->cur;
    WgHost w{t, f->nt, f->red, nullptr, f};
    adj_run_task(w, *f->a, f->kind, f->task);
    f->state[t] = 2;  // uc_link returns to the scheduler
  }

  void yield(int t) {
    state[t] = 1;
    swapcontext(&ctx[t], &sched);
  }

  // Runs one task to its end; false if its lanes did not all meet at the
  // same barriers.
  bool run(const AdjArgs& args, int k, int tk, double* r, int lanes) {
    a = &args;
    kind = k;
    task = tk;
    red = r;
    nt = lanes;
    ctx.assign(nt, ucontext_t{});
    if ((int)stack.size() < nt) stack.resize(nt);
    state.assign(nt, 0);
    self = this;
    for (int t = 0; t < nt; ++t) {
      stack[t].resize(kStack);
      getcontext(&ctx[t]);
      ctx[t].uc_stack.ss_sp = stack[t].data();
      ctx[t].uc_stack.ss_size = kStack;
      ctx[t].uc_link = &sched;
      cur = t;
      makecontext(&ctx[t], (void (*)())entry, 0);
    }
    using clk = std::chrono::steady_clock;
    for (;;) {
      double seg_max = 0.0;
      for (int t = 0; t < nt; ++t) {
        if (state[t] == 2) continue;
        state[t] = 0;
        cur = t;
        const auto t0 = clk::now();
        swapcontext(&sched, &ctx[t]);
        const double ns = std::chrono::duration<double, std::nano>(clk::now() - t0).count();
        seg_max = ns > seg_max ? ns : seg_max;
      }
      crit_ns += seg_max;
      int done = 0;
      for (int t = 0; t < nt; ++t) done += state[t] == 2;
      if (done == nt) return true;
      if (done != 0) {
        diverged = true;
        return false;  // lanes left at a barrier are abandoned with their stacks
      }
      ++barriers;
    }
  }
};

thread_local Fibers* Fibers::self = nullptr;

void WgHost::sync() {
  if (fib)
    fib->yield(tid);
  else
    bar->arrive_and_wait();
}

static bool g_fibers = false;
static int g_fiber_error = 0;
static int64_t g_fiber_barriers = 0;
// per task kind: sum over launches of the slowest task's critical path (ns)
// and of its barrier count, and the launches
static double g_crit_ns[32];
static int64_t g_crit_bar[32], g_crit_launches[32];

struct HostExec {
  AdjArgs a;
  int nt;
  void launch(int kind, int base, int count) {
    double crit = 0.0;
    int64_t crit_bar = 0;
    for (int g = 0; g < count; ++g) {
      std::vector<double> red(3 * nt + ADJ_RED_EXTRA, 0.0);
      if (g_fibers && nt > 1) {
        Fibers f;
        if (!f.run(a, kind, base + g, red.data(), nt)) {
          g_fiber_error = 1;
          std::fprintf(stderr, "adj_host: lanes diverged at a barrier (kind %d, task %d)\n",
                       kind, base + g);
          return;
        }
        g_fiber_barriers += f.barriers;
        if (f.crit_ns > crit) {
          crit = f.crit_ns;
          crit_bar = f.barriers;
        }
        if (g + 1 == count && kind >= 0 && kind < 32) {
          g_crit_ns[kind] += crit;
          g_crit_bar[kind] += crit_bar;
          ++g_crit_launches[kind];
        }
        continue;
      }
      std::barrier<> bar(nt);
      if (nt == 1) {
        WgHost w{0, 1, red.data(), &bar, nullptr};
        adj_run_task(w, a, kind, base + g);
        continue;
      }
      std::vector<std::thread> th;
      th.reserve(nt);
      for (int t = 0; t < nt; ++t)
        th.emplace_back([&, t] {
          WgHost w{t, nt, red.data(), &bar, nullptr};
          adj_run_task(w, a, kind, base + g);
        });
      for (auto& x : th) x.join();
    }
  }
};

}  // namespace

// row chunking of tall merges (the library's defaults unless a test sets them)
static int64_t g_chunk_rows = AdjPlanIn().chunk_rows;
static int g_max_chunks = AdjPlanIn().max_chunks;
static int g_split = 0, g_nchunks = 0;

static int make_plan(int64_t m, int64_t n, int L, int dim, int dmax, int fz_stride,
                     const int64_t* leaf_info, const int32_t* recs, const int32_t* ranks,
                     AdjPlan& P) {
  AdjPlanIn in;
  in.m = m;
  in.n = n;
  in.L = L;
  in.dim = dim;
  in.dmax = dmax;
  in.fz_stride = fz_stride;
  in.chunk_rows = g_chunk_rows;
  in.max_chunks = g_max_chunks;
  const int nb = 1 << L;
  for (int b = 0; b < nb * nb; ++b) {
    const int64_t* f = leaf_info + 7 * b;
    AdjLeafIn li;
    li.row0 = f[0];
    li.col0 = f[1];
    li.m0 = (int32_t)f[2];
    li.n0 = (int32_t)f[3];
    li.nrec = (int32_t)f[4];
    li.rank_leaf = (int32_t)f[5];
    li.rec = recs + f[6] * fz_stride;
    in.leaves.push_back(li);
  }
  int64_t off = 0;
  for (int l = 1; l <= L; ++l) {
    const int nbc = 1 << (L - l + 1), nbp = nbc / 2;
    in.hrank.emplace_back(ranks + off, ranks + off + nbc * nbp);
    off += nbc * nbp;
    in.vrank.emplace_back(ranks + off, ranks + off + nbp * nbp);
    off += nbp * nbp;
  }
  const int st = adj_plan(in, P);
  g_split = 0;
  for (const AdjMerge& M : P.merges) g_split += M.G > 1;
  g_nchunks = (int)P.chunks.size();
  return st;
}

static AdjArgs make_args(const AdjPlan& P, std::vector<double>& D, int64_t m, int64_t n, int dim,
                         int dmax, const double* Xsoa, const double* Ysoa, double h, double c) {
  AdjArgs a{};
  a.D = D.data();
  a.ws = D.data() + P.ws_off;
  a.fz = P.fz.data();
  a.leaves = P.leaves.data();
  a.blocks = P.blocks.data();
  a.merges = P.merges.data();
  a.chunks = P.chunks.data();
  a.tasks = P.tasks.data();
  a.X = Xsoa;
  a.Y = Ysoa;
  a.ldx = m;
  a.ldy = n;
  a.dim = dim;
  a.dmax = dmax;
  a.fz_stride = 3 + 3 * dmax;
  a.root = P.root;
  a.nb = P.nb;
  a.nleaves = (int32_t)P.leaves.size();
  a.h = h;
  a.nic = -1.0 / (c * h * h);
  return a;
}

extern "C" {

// Row chunking of tall merges for the following calls (tests force small
// chunks to run the split path at small sizes).
void adj_host_set_chunking(int64_t chunk_rows, int max_chunks) {
  g_chunk_rows = chunk_rows;
  g_max_chunks = max_chunks;
}

// Lanes as fibers on the calling thread (on != 0) or as threads.  Returns,
// and clears, whether a task's lanes diverged at a barrier since the last
// call; *barriers gets the barrier count.
int adj_host_set_fibers(int on, int64_t* barriers) {
  g_fibers = on != 0;
  const int e = g_fiber_error;
  g_fiber_error = 0;
  if (barriers) *barriers = g_fiber_barriers;
  g_fiber_barriers = 0;
  return e;
}

// Fiber mode's critical-path profile per task kind (32 entries each): the
// sum over launches of the slowest task's time summed over its barrier
// intervals (each interval costing its slowest lane), its barriers, and
// the launches; cleared after the call.
void adj_host_fiber_profile(double* crit_ns, int64_t* barriers, int64_t* launches) {
  for (int k = 0; k < 32; ++k) {
    crit_ns[k] = g_crit_ns[k];
    barriers[k] = g_crit_bar[k];
    launches[k] = g_crit_launches[k];
    g_crit_ns[k] = 0.0;
    g_crit_bar[k] = 0;
    g_crit_launches[k] = 0;
  }
}

// Number of merges the last plan split, and their chunks.
void adj_host_last_split(int* merges, int* chunks) {
  *merges = g_split;
  *chunks = g_nchunks;
}

// leaf_info: per leaf (b = t 2^L + v) row0, col0, m0, n0, records,
// rank_leaf, first record index; recs: records of fz_stride ints; ranks:
// per level l = 1..L the horizontal ranks (block (ti, v), ti-major) then
// the vertical ranks (block (t, v), t-major).  Points are structure of
// arrays.  The arena starts filled with NaN so that a read of memory no
// task wrote shows up in the outputs.  Returns the planner's status.
int adj_host_vjp(int64_t m, int64_t n, int L, int dim, int dmax, int fz_stride,
                 const int64_t* leaf_info, const int32_t* recs, const int32_t* ranks,
                 const double* Xsoa, const double* Ysoa, double h, double c, const double* w,
                 const double* ybar, double* gw, double* gh, double* gX, double* gY, int nt,
                 int64_t* arena_out) {
  AdjPlan P;
  const int st = make_plan(m, n, L, dim, dmax, fz_stride, leaf_info, recs, ranks, P);
  if (st != 0) return st;
  if (arena_out) *arena_out = P.arena;
  std::vector<double> D(P.arena, std::numeric_limits<double>::quiet_NaN());
  AdjArgs a = make_args(P, D, m, n, dim, dmax, Xsoa, Ysoa, h, c);
  a.w = w;
  a.ybar = ybar;
  a.gw = gw;
  a.gh = gh;
  a.gX = gX;
  a.gY = gY;
  HostExec ex{a, nt};
  adj_execute(ex, P, gX != nullptr, gY != nullptr, gh != nullptr);
  return 0;
}

// The plan alone: the arena size in doubles (workspace included).
int adj_host_plan_size(int64_t m, int64_t n, int L, int dim, int dmax, int fz_stride,
                       const int64_t* leaf_info, const int32_t* recs, const int32_t* ranks,
                       int64_t* arena, int64_t* ws) {
  AdjPlan P;
  const int st = make_plan(m, n, L, dim, dmax, fz_stride, leaf_info, recs, ranks, P);
  if (st != 0) return st;
  *arena = P.arena;
  *ws = P.ws_size;
  return 0;
}

// The frozen operator alone (the forward tasks): its root rank in *rank,
// and, when the buffers hold cap columns, U (m x rank), S and Vt (n x rank).
int adj_host_forward(int64_t m, int64_t n, int L, int dim, int dmax, int fz_stride,
                     const int64_t* leaf_info, const int32_t* recs, const int32_t* ranks,
                     const double* Xsoa, const double* Ysoa, double h, double c, int nt, int cap,
                     double* U, double* S, double* Vt, int32_t* rank) {
  AdjPlan P;
  const int st = make_plan(m, n, L, dim, dmax, fz_stride, leaf_info, recs, ranks, P);
  if (st != 0) return st;
  std::vector<double> D(P.arena, std::numeric_limits<double>::quiet_NaN());
  AdjArgs a = make_args(P, D, m, n, dim, dmax, Xsoa, Ysoa, h, c);
  HostExec ex{a, nt};
  adj_execute_forward(ex, P);
  const AdjBlock& B = P.blocks[P.root];
  *rank = B.r;
  if (B.r > cap) return 1;
  for (int j = 0; j < B.r; ++j) {
    for (int64_t i = 0; i < m; ++i) U[i + j * m] = D[B.U + i + j * B.ldU];
    for (int64_t i = 0; i < n; ++i) Vt[i + j * n] = D[B.Vt + i + j * B.ldVt];
    S[j] = D[B.S + j];
  }
  return 0;
}

}  // extern "C"

#ifdef ADJ_HOST_MAIN
// Stand-alone driver (for the sanitizer builds): reads the inputs of
// adj_host_vjp from argv[1], runs it with argv[3] lanes per workgroup (and,
// if given, row chunks of at least argv[4] rows, at most argv[5] per merge)
// and writes gw, gh, gX, gY to argv[2].
int main(int argc, char** argv) {
  if (argc < 4) return 2;
  if (argc >= 6) adj_host_set_chunking(std::atoll(argv[4]), std::atoi(argv[5]));
  FILE* f = std::fopen(argv[1], "rb");
  if (!f) return 2;
  int64_t hd[9];
  if (std::fread(hd, 8, 9, f) != 9) return 2;
  const int64_t m = hd[0], n = hd[1], nleaves = hd[6], nrec = hd[7], nrank = hd[8];
  const int L = (int)hd[2], dim = (int)hd[3], dmax = (int)hd[4], stride = (int)hd[5];
  std::vector<int64_t> info(7 * nleaves);
  std::vector<int32_t> recs(nrec), ranks(nrank + 1);
  std::vector<double> X(dim * m), Y(dim * n), hc(2), w(n), yb(m);
  bool ok = std::fread(info.data(), 8, info.size(), f) == info.size();
  ok = ok && std::fread(recs.data(), 4, nrec, f) == (size_t)nrec;
  ok = ok && std::fread(ranks.data(), 4, nrank, f) == (size_t)nrank;
  ok = ok && std::fread(X.data(), 8, X.size(), f) == X.size();
  ok = ok && std::fread(Y.data(), 8, Y.size(), f) == Y.size();
  ok = ok && std::fread(hc.data(), 8, 2, f) == 2;
  ok = ok && std::fread(w.data(), 8, n, f) == (size_t)n;
  ok = ok && std::fread(yb.data(), 8, m, f) == (size_t)m;
  std::fclose(f);
  if (!ok) return 2;
  std::vector<double> gw(n), gh(1), gX(m * dim), gY(n * dim);
  const int st = adj_host_vjp(m, n, L, dim, dmax, stride, info.data(), recs.data(), ranks.data(),
                              X.data(), Y.data(), hc[0], hc[1], w.data(), yb.data(), gw.data(),
                              gh.data(), gX.data(), gY.data(), std::atoi(argv[3]), nullptr);
  if (st != 0) return 3;
  FILE* o = std::fopen(argv[2], "wb");
  if (!o) return 2;
  std::fwrite(gw.data(), 8, n, o);
  std::fwrite(gh.data(), 8, 1, o);
  std::fwrite(gX.data(), 8, gX.size(), o);
  std::fwrite(gY.data(), 8, gY.size(), o);
  std::fclose(o);
  return 0;
}
#endif
