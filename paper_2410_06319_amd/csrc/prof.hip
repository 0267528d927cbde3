// Opt-in per-kernel timing: an event pair for every launch of the profiled
// kernel classes (stamped by the launch itself for single kernels, recorded
// around the launches for the two-kernel Gram-Schmidt class), summed after
// the call has synchronised.  The record is per host thread.
#include <vector>

#include "common.h"
#include "kernels.h"

namespace ls {
namespace {
struct Pair {
  hipEvent_t a, b;
  int cls;
  double work;
};
// per host thread: concurrent calls on different threads keep separate records
thread_local bool g_on = false;
thread_local std::vector<Pair> g_pool;
thread_local size_t g_used = 0;
}  // namespace

void prof_reset(bool on) {
  g_on = on;
  g_used = 0;
}

void prof_begin(int cls, hipStream_t st) {
  if (!g_on) return;
  if (g_used == g_pool.size()) {
    Pair p{};
    if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) {
      g_on = false;
      return;
    }
    g_pool.push_back(p);
  }
  g_pool[g_used].cls = cls;
  (void)hipEventRecord(g_pool[g_used].a, st);
}

void prof_end(int cls, hipStream_t st, double work) {
  if (!g_on || g_used >= g_pool.size() || g_pool[g_used].cls != cls) return;
  g_pool[g_used].work = work;
  (void)hipEventRecord(g_pool[g_used].b, st);
  ++g_used;
}

ProfEv prof_events(int cls) {
  ProfEv ev;
  if (!g_on) return ev;
  if (g_used == g_pool.size()) {
    Pair p{};
    if (hipEventCreate(&p.a) != hipSuccess || hipEventCreate(&p.b) != hipSuccess) {
      g_on = false;
      return ev;
    }
    g_pool.push_back(p);
  }
  g_pool[g_used].cls = cls;
  ev.a = g_pool[g_used].a;
  ev.b = g_pool[g_used].b;
  return ev;
}

void prof_commit(int cls, double work) {
  if (!g_on || g_used >= g_pool.size() || g_pool[g_used].cls != cls) return;
  g_pool[g_used].work = work;
  ++g_used;
}

size_t prof_mark() { return g_used; }

void prof_keep(int cls, size_t from, int keep) {
  if (!g_on) return;
  for (size_t i = from; i < g_used; ++i) {
    if (g_pool[i].cls != cls) continue;
    if (keep > 0) --keep;
    else g_pool[i].cls = -1;   // a launch queued after convergence: not filed
  }
}

void prof_collect(ls_stats_t* stats) {
  if (!stats) return;
  for (int c = 0; c < kProfClasses; ++c) {
    stats->kernel_ms[c] = 0.0;
    stats->kernel_launches[c] = 0;
    stats->kernel_work[c] = 0.0;
  }
  for (size_t i = 0; i < g_used; ++i) {
    if (g_pool[i].cls < 0) continue;
    float ms = 0.f;
    if (hipEventElapsedTime(&ms, g_pool[i].a, g_pool[i].b) == hipSuccess) {
      stats->kernel_ms[g_pool[i].cls] += ms;
      stats->kernel_launches[g_pool[i].cls] += 1;
      stats->kernel_work[g_pool[i].cls] += g_pool[i].work;
    }
  }
  g_used = 0;
}
}  // namespace ls
