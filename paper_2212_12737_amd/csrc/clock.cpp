// Kernel clocks: HIP event pairs recorded on the launching stream around the
// hot kernels (every launch, or every stride-th one to keep the markers' own
// cost out of the timed work), accumulated per kernel id.  Recording never
// synchronizes; pairs are harvested when their end event has completed
// (checked without waiting whenever many are pending) or at a read, which
// synchronizes the device.
#include <deque>
#include <vector>

#include "common.hpp"

namespace ffk {

namespace {

struct Pending {
  int id;
  hipEvent_t a, b;
};

struct ClockState {
  bool on = false;
  int stride = 1;
  int device = -1;
  int64_t seen[CLK_COUNT] = {};
  std::vector<hipEvent_t> pool;
  std::deque<Pending> pending;
  hipEvent_t open[CLK_COUNT] = {};
  double total_ms[CLK_COUNT] = {};
  int64_t launches[CLK_COUNT] = {};
};

ClockState g_clk;
thread_local int g_paused = 0;

hipEvent_t take_event() {
  if (!g_clk.pool.empty()) {
    hipEvent_t e = g_clk.pool.back();
    g_clk.pool.pop_back();
    return e;
  }
  hipEvent_t e;
  HIPCHK(hipEventCreate(&e));
  return e;
}

void settle(const Pending& p) {
  float ms = 0.f;
  HIPCHK(hipEventElapsedTime(&ms, p.a, p.b));
  g_clk.total_ms[p.id] += ms;
  g_clk.launches[p.id] += 1;
  g_clk.pool.push_back(p.a);
  g_clk.pool.push_back(p.b);
}

// settle completed pairs from the front without waiting
void harvest_ready() {
  while (!g_clk.pending.empty()) {
    const hipError_t q = hipEventQuery(g_clk.pending.front().b);
    if (q == hipErrorNotReady) return;
    HIPCHK(q);
    settle(g_clk.pending.front());
    g_clk.pending.pop_front();
  }
}

void drain_all() {
  for (const Pending& p : g_clk.pending) {
    HIPCHK(hipEventSynchronize(p.b));
    settle(p);
  }
  g_clk.pending.clear();
}

}  // namespace

ClockPause::ClockPause() { ++g_paused; }
ClockPause::~ClockPause() { --g_paused; }

void clk_begin(int id, hipStream_t st) {
  if (!g_clk.on || g_paused) return;
  if (g_clk.seen[id]++ % g_clk.stride != 0) return;   // time every stride-th launch
  if (g_clk.pending.size() > 256) harvest_ready();
  hipEvent_t a = take_event();
  HIPCHK(hipEventRecord(a, st));
  g_clk.open[id] = a;
}

void clk_end(int id, hipStream_t st) {
  if (!g_clk.on || g_paused || !g_clk.open[id]) return;
  hipEvent_t b = take_event();
  HIPCHK(hipEventRecord(b, st));
  g_clk.pending.push_back(Pending{id, g_clk.open[id], b});
  g_clk.open[id] = nullptr;
}

void clock_enable(int stride) {
  const bool on = stride > 0;
  HIPCHK(hipDeviceSynchronize());
  drain_all();
  for (int i = 0; i < CLK_COUNT; ++i) {
    g_clk.total_ms[i] = 0.0;
    g_clk.launches[i] = 0;
    g_clk.seen[i] = 0;
    if (g_clk.open[i]) g_clk.pool.push_back(g_clk.open[i]);
    g_clk.open[i] = nullptr;
  }
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (on && g_clk.device >= 0 && dev != g_clk.device) {
    // events of another device cannot time this one's streams
    for (hipEvent_t e : g_clk.pool) (void)hipEventDestroy(e);
    g_clk.pool.clear();
  }
  g_clk.device = dev;
  g_clk.on = on;
  g_clk.stride = on ? stride : 1;
}

void clock_read(int id, double* total_ms, int64_t* launches) {
  require(id >= 0 && id < CLK_COUNT, "clock_read: unknown clock id");
  HIPCHK(hipDeviceSynchronize());
  drain_all();
  *total_ms = g_clk.total_ms[id];
  *launches = g_clk.launches[id];
}

}  // namespace ffk
