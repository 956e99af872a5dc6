// RK4 stepping (step (ii)): launch plans over grouped tiled launches,
// resident and generic kernels, HIP-graph capture and replay, the split and
// integrating-factor schemes, the thresholded representation, batches.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cfloat>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <fstream>
#include <map>
#include <memory>
#include <mutex>
#include <set>
#include <sstream>
#include <stdexcept>
#include <string>
#include <unordered_map>
#include <vector>

#include "hgf.h"
#include "hgf_internal.h"
#include "hgf_host.h"
#include "hgf_kernels.h"
#include "hgf_runtime.h"

namespace hgf {

// ------------------------------------------------------------------ stepping

void reset_flag(hgf_operator_s* op, hipStream_t st) {
  hip_check(hipMemsetAsync(op->dflag, 0, sizeof(int), st), "reset flag");
}



MemberArgs member_args(const PlanItem& it) {
  Function& f = *it.f;
  MemberArgs m{};
  m.g = f.ga;
  m.in[0] = it.precision == HGF_MIXED ? f.yf : f.y;
  m.in[1] = f.s1;
  m.in[2] = f.s2;
  m.in[3] = f.s3;
  m.x1 = f.s1;
  m.y = f.y;
  m.yf = it.precision == HGF_MIXED ? f.yf : nullptr;
  m.out[0] = f.s1;
  m.out[1] = f.s2;
  m.out[2] = f.s3;
  m.out[3] = nullptr;
  m.h = it.h;
  return m;
}

StepPlan* build_plan(const std::vector<PlanItem>& items, bool allow_resident) {
  std::unique_ptr<StepPlan> plan(new StepPlan);
  std::map<std::vector<int>, std::vector<PlanItem>> by_key, res_key;
  for (const PlanItem& it : items) {
    const GridArgs& g = it.f->ga;
    if (allow_resident && it.f->resident)
      res_key[{it.f->full ? g.n / 2 : g.n, g.real, it.precision, it.f->full ? 1 : 0}].push_back(it);
    else if (g.blocks > 0)
      by_key[{g.nfast, g.n - g.nfast, g.real, it.precision}].push_back(it);
    else
      plan->generic.push_back(it);
  }
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  for (auto& kv : by_key) {
    std::vector<MemberArgs> mem;
    GroupLaunch gl{};
    gl.nfast = kv.first[0];
    gl.nslow = kv.first[1];
    gl.real = kv.first[2];
    gl.precision = kv.first[3];
    int64_t tiles = 0;
    for (const PlanItem& it : kv.second) {
      MemberArgs m = member_args(it);
      m.tile_begin = tiles;
      tiles += it.f->ga.ntiles;
      gl.threads = std::max(gl.threads, it.f->ga.threads);
      gl.lds_bytes = std::max(gl.lds_bytes, it.f->ga.lds_bytes);
      mem.push_back(m);
    }
    gl.nmem = (int)mem.size();
    gl.total_tiles = tiles;
    int occ = tiled_max_blocks_per_cu(gl.nfast, gl.nslow, gl.threads, gl.precision, gl.lds_bytes, gl.real,
                                      mem.size() == 1 ? (kv.second[0].f->ga.pipe ? 2 : 1) : 0);
    int cap_all = kv.second[0].f->ga.occ_cap;  // members' common cap on resident workgroups per CU
    for (const PlanItem& it : kv.second)
      if (it.f->ga.occ_cap != cap_all) cap_all = 0;
    if (cap_all > 0) occ = std::min(occ, cap_all);
    gl.blocks = (int)std::max<int64_t>(8, std::min<int64_t>((int64_t)cus * occ, 8 * ((tiles + 7) / 8)));
    if (mem.size() == 1) gl.blocks = kv.second[0].f->ga.blocks;  // the function's own (possibly tuned) grid
    void* d = dmalloc(mem.size() * sizeof(MemberArgs));
    plan->dmem.push_back(d);
    hip_check(hipMemcpy(d, mem.data(), mem.size() * sizeof(MemberArgs), hipMemcpyHostToDevice), "upload members");
    gl.members = (const MemberArgs*)d;
    gl.single = mem[0];
    plan->groups.push_back(gl);
  }
  for (auto& kv : res_key) {
    ResidentLaunch rl{};
    rl.nfast = kv.first[0];
    rl.real = kv.first[1];
    rl.precision = kv.first[2];
    rl.full = kv.first[3];
    std::vector<ResidentItem> host;
    for (const PlanItem& it : kv.second) {
      ResidentItem ri{};
      ri.g = it.f->full ? it.f->ga : it.f->rga;
      ri.y = it.f->y;
      ri.yf = it.precision == HGF_MIXED ? it.f->yf : nullptr;
      ri.x1 = it.f->s1;
      ri.steps = 0;
      ri.h = it.h;
      host.push_back(ri);
      rl.threads = std::max(rl.threads, it.f->res_threads);
      rl.lds_bytes = std::max(rl.lds_bytes, it.f->res_lds_bytes);
    }
    rl.count = (int)host.size();
    void* d = dmalloc(host.size() * sizeof(ResidentItem));
    plan->dmem.push_back(d);
    rl.items = (const ResidentItem*)d;
    plan->resident.push_back(rl);
    plan->res_host.push_back(std::move(host));
  }
  return plan.release();
}

// Advance the plan's resident functions by `steps` RK4 steps (launches of at
// most kResidentChunk steps each).
void run_resident(StepPlan& plan, int64_t steps, int* flag, hipStream_t st) {
  for (size_t k = 0; k < plan.resident.size(); ++k) {
    std::vector<ResidentItem>& host = plan.res_host[k];
    for (int64_t done = 0; done < steps;) {
      const int n = (int)std::min(kResidentChunk, steps - done);
      if (host[0].steps != n) {
        for (auto& ri : host) ri.steps = n;
        hip_check(hipMemcpyAsync((void*)plan.resident[k].items, host.data(), host.size() * sizeof(ResidentItem),
                                 hipMemcpyHostToDevice, st),
                  "upload resident items");
        hip_check(hipStreamSynchronize(st), "synchronize");  // the host copy may change before the next launch
      }
      launch_resident(plan.resident[k], flag, st);
      done += n;
    }
  }
}

// One Horner stage of one function with explicit buffers (stage input `in`,
// X1, state, stage output), on the tiled kernel where the function has a
// tiled configuration, else the generic one.
void stage_launch(const Function& f, int precision, int stage, const void* in, const void* x1, void* y,
                         void* yf, void* out, double h, int* flag, hipStream_t st) {
  if (f.ga.blocks == 0) {
    launch_horner(stage, precision, f.ga, in, x1, y, yf, out, h, flag, st);
    return;
  }
  GroupLaunch gl{};
  MemberArgs& m = gl.single;
  m.g = f.ga;
  m.in[stage - 1] = in;
  m.x1 = x1;
  m.y = y;
  m.yf = yf;
  m.out[stage - 1] = out;
  m.h = h;
  gl.members = nullptr;
  gl.nmem = 1;
  gl.total_tiles = f.ga.ntiles;
  gl.nfast = f.ga.nfast;
  gl.nslow = f.ga.n - f.ga.nfast;
  gl.threads = f.ga.threads;
  gl.lds_bytes = f.ga.lds_bytes;
  gl.blocks = f.ga.blocks;
  gl.real = f.ga.real;
  gl.precision = precision;
  launch_group(gl, stage, flag, st);
}

void generic_stage(const PlanItem& it, int s, int* flag, hipStream_t st) {
  Function& f = *it.f;
  const void* in[4] = {it.precision == HGF_MIXED ? f.yf : f.y, f.s1, f.s2, f.s3};
  void* out[4] = {f.s1, f.s2, f.s3, nullptr};
  (f.full ? (f.ga.fblocks > 0 ? launch_full_tiled : launch_full_horner) : launch_horner)(s, it.precision, f.ga, in[s - 1], f.s1, f.y,
                                                it.precision == HGF_MIXED ? f.yf : nullptr, out[s - 1], it.h, flag,
                                                st);
}

void run_plan_step(const StepPlan& plan, int* flag, hipStream_t st) {
  for (int s = 1; s <= 4; ++s) {
    for (const GroupLaunch& gl : plan.groups) launch_group(gl, s, flag, st);
    for (const PlanItem& it : plan.generic) generic_stage(it, s, flag, st);
  }
}

void drop_graph(hgf_operator_s* op) {
  if (op->graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)op->graph_exec);
  op->graph_exec = nullptr;
  op->graph_steps = 0;
}

void drop_plan(hgf_operator_s* op) {
  drop_graph(op);
  delete op->plan;
  op->plan = nullptr;
}

void ensure_plan(hgf_operator_s* op, double h) {
  if (op->plan && op->graph_dt == h) return;
  drop_plan(op);
  std::vector<PlanItem> items;
  for (auto& f : op->fn) items.push_back({&f, op->precision, h});
  op->plan = build_plan(items);
  op->graph_dt = h;
}


// Streams a capture forks onto (one per grouped launch beyond the first),
// per host thread and device (so that captures on several threads never
// share one), created with the default priority and kept until the process
// ends.
static hipStream_t branch_stream(int dev, size_t i) {
  static thread_local std::map<int, std::vector<hipStream_t>> pool;
  std::vector<hipStream_t>& v = pool[dev];
  while (v.size() <= i) {
    hipStream_t s;
    hip_check(hipStreamCreateWithFlags(&s, hipStreamNonBlocking), "stream");
    v.push_back(s);
  }
  return v[i];
}

// HGF_GRAPH_BRANCHES=0 captures every launch in one chain.
static bool graph_branches() {
  const char* env = std::getenv("HGF_GRAPH_BRANCHES");
  return !(env && std::string(env) == "0");
}

// `chunk` steps of the plan as one graph.  The plan's chains of launches
// (each grouped launch, each function on the untiled kernels) are
// independent of each other (different functions), so with several chains
// they are spread over up to kGraphBranches branches of the graph (forked
// from and joined back to `cap`; chain c on branch c mod branches): a chain
// too small to fill the chip then runs beside the others instead of after
// them.  Within a branch the stages keep their order; results do not depend
// on the branching.
constexpr size_t kGraphBranches = 8;
hipGraphExec_t capture_steps(const StepPlan& plan, int* flag, int chunk, hipStream_t cap) {
  hipGraph_t graph;
  const size_t ng = plan.groups.size(), nchain = ng + plan.generic.size();
  const size_t nb = graph_branches() ? std::min(nchain, kGraphBranches) : 1;
  auto launch_chain = [&](size_t c, int stage, hipStream_t s) {
    if (c < ng)
      launch_group(plan.groups[c], stage, flag, s);
    else
      generic_stage(plan.generic[c - ng], stage, flag, s);
  };
  auto branch_steps = [&](size_t b, hipStream_t s) {
    for (int k = 0; k < chunk; ++k)
      for (int stage = 1; stage <= 4; ++stage)
        for (size_t c = b; c < nchain; c += nb) launch_chain(c, stage, s);
  };
  std::vector<hipEvent_t> ev;  // ev[0]: fork; ev[b]: join of branch b
  auto drop_events = [&] {
    for (hipEvent_t e : ev) (void)hipEventDestroy(e);
    ev.clear();
  };
  int dev = 0;
  if (nb > 1) hip_check(hipGetDevice(&dev), "hipGetDevice");
  hip_check(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
  try {
    if (nb <= 1) {
      for (int k = 0; k < chunk; ++k) run_plan_step(plan, flag, cap);
    } else {
      for (size_t b = 0; b < nb; ++b) {
        hipEvent_t e;
        hip_check(hipEventCreateWithFlags(&e, hipEventDisableTiming), "event");
        ev.push_back(e);
      }
      hip_check(hipEventRecord(ev[0], cap), "fork");
      for (size_t b = 1; b < nb; ++b) {
        hipStream_t bs = branch_stream(dev, b - 1);
        hip_check(hipStreamWaitEvent(bs, ev[0], 0), "fork");
        branch_steps(b, bs);
        hip_check(hipEventRecord(ev[b], bs), "join");
      }
      branch_steps(0, cap);
      for (size_t b = 1; b < nb; ++b) hip_check(hipStreamWaitEvent(cap, ev[b], 0), "join");
    }
  } catch (...) {
    hipGraph_t partial;
    if (hipStreamEndCapture(cap, &partial) == hipSuccess) (void)hipGraphDestroy(partial);
    drop_events();
    throw;
  }
  const hipError_t ec = hipStreamEndCapture(cap, &graph);
  drop_events();
  hip_check(ec, "end capture");
  hipGraphExec_t exec;
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  hip_check(e, "graph instantiate");
  return exec;
}

// Steps per captured graph: at most 64, and at most kMaxGraphNodes kernel
// nodes (an operator whose many functions each take their own generic launch
// would otherwise capture graphs of millions of nodes).  0: launch eagerly.
int graph_chunk(const StepPlan& plan, int64_t steps) {
  const int64_t per_step = 4 * (int64_t)(plan.groups.size() + plan.generic.size());
  if (per_step == 0) return 0;
  return (int)std::min<int64_t>({steps, 64, kMaxGraphNodes / per_step});
}

// One graph holds `chunk` merged steps of every function of the operator.
void ensure_graph(hgf_operator_s* op, double h, int chunk) {
  ensure_plan(op, h);
  if (op->graph_exec && op->graph_steps == chunk) return;
  drop_graph(op);
  if (!op->cap_stream) hip_check(hipStreamCreateWithFlags(&op->cap_stream, hipStreamNonBlocking), "stream");
  op->graph_exec = capture_steps(*op->plan, op->dflag, chunk, op->cap_stream);
  op->graph_steps = chunk;
}

void split_step(hgf_operator_s* op, Function& f, double h, hipStream_t st) {
  // stage products c_x c_y of the scalar RK4 for (c_x, c_y), then the
  // classical stages of R with point sources scaled by them
  cd cx = f.cx, cy = f.cy;
  cd kx[4], ky[4], X[4], Y[4];
  X[0] = cx;
  Y[0] = cy;
  const double a[4] = {0.0, 0.5, 0.5, 1.0};
  for (int s = 0; s < 4; ++s) {
    if (s > 0) {
      X[s] = cx + a[s] * h * kx[s - 1];
      Y[s] = cy + a[s] * h * ky[s - 1];
    }
    kx[s] = f.ax * X[s];
    ky[s] = f.ay * Y[s];
  }
  PointSources ps{};
  ps.count = (int)f.sources.size();
  for (int i = 0; i < ps.count; ++i) {
    ps.index[i] = f.sources[i].first;
    ps.re[i] = f.sources[i].second.real();
    ps.im[i] = f.sources[i].second.imag();
  }
  void* in[4] = {f.y, f.s1, f.s2, f.s1};
  void* nx[4] = {f.s1, f.s2, f.s1, nullptr};
  for (int s = 0; s < 4; ++s) {
    const cd P = X[s] * Y[s];
    ps.scale_re = P.real();
    ps.scale_im = P.imag();
    launch_classical(s + 1, op->precision, f.ga, in[s], f.y, f.s4, nx[s], h, ps, op->dflag, st);
  }
  f.cx = cx + h / 6.0 * (kx[0] + 2.0 * kx[1] + 2.0 * kx[2] + kx[3]);
  f.cy = cy + h / 6.0 * (ky[0] + 2.0 * ky[1] + 2.0 * ky[2] + ky[3]);
}

// Integrating-factor scheme: per-axis factors exp(lam_j(m) h/2) of a function
// for step h (uploaded once per step size).
void ensure_lawson_tables(Function& f, double h, hipStream_t st) {
  if (f.ehtab && f.eh_h == h) return;
  std::vector<double2> t;
  for (int j = 0; j < f.tab.n; ++j)
    for (int m = 0; m < f.tab.ext[j]; ++m) {
      const cd e = std::exp(f.tab.lam[j][m] * (0.5 * h));
      t.push_back(make_double2(e.real(), e.imag()));
    }
  if (!f.ehtab) f.ehtab = dmalloc(t.size() * sizeof(double2));
  hip_check(hipMemcpyAsync(f.ehtab, t.data(), t.size() * sizeof(double2), hipMemcpyHostToDevice, st), "upload");
  hip_check(hipStreamSynchronize(st), "synchronize");  // the host table is freed on return
  f.eh0 = std::exp(f.tab.lam0 * (0.5 * h));
  f.eh_h = h;
}

// Integrating-factor RK4 steps of every function of an operator: one grouped
// launch per stage and element type (complex and real grids), items in device
// memory for the call (stage buffers: s1 and s2 take v2, v3, v4 in turn, s3 the
// increment).  Steps are captured in HIP graphs of up to 64 steps.
void lawson_steps(hgf_operator_s* op, int64_t steps, double h, hipStream_t st) {
  for (auto& f : op->fn) ensure_lawson_tables(f, h, st);
  const bool mixed = op->precision == HGF_MIXED;
  constexpr int kMaxRows = 65535;  // grid rows per launch
  struct Group {
    bool real;
    std::vector<LawsonItem> items;
    int row_blocks = 1;
    size_t offset = 0;
  };
  Group groups[2] = {{false, {}}, {true, {}}};
  for (auto& f : op->fn) groups[f.real ? 1 : 0].row_blocks = std::max(groups[f.real ? 1 : 0].row_blocks,
                                                                         lawson_row_blocks(f.ga));
  for (auto& f : op->fn) {
    Group& gr = groups[f.real ? 1 : 0];
    LawsonItem it{};
    it.g = f.ga;
    it.sd = lawson_row_digits(f.ga, gr.row_blocks);
    it.y = f.y;
    it.yf = mixed ? f.yf : nullptr;
    it.s1 = f.s1;
    it.s2 = f.s2;
    it.s3 = f.s3;
    it.eh = (const double2*)f.ehtab;
    it.e0 = make_double2(f.eh0.real(), f.eh0.imag());
    gr.items.push_back(it);
  }
  std::vector<LawsonItem> all;
  for (auto& gr : groups) {
    gr.offset = all.size();
    all.insert(all.end(), gr.items.begin(), gr.items.end());
  }
  DBuf ditems(all.size() * sizeof(LawsonItem));
  hip_check(hipMemcpyAsync(ditems.p, all.data(), all.size() * sizeof(LawsonItem), hipMemcpyHostToDevice, st),
            "upload items");
  hip_check(hipStreamSynchronize(st), "synchronize");  // the host copy is freed on return
  int launches = 0;
  for (auto& gr : groups) launches += (int)((gr.items.size() + kMaxRows - 1) / kMaxRows);
  auto step = [&](hipStream_t s) {
    for (int stage = 1; stage <= 4; ++stage)
      for (auto& gr : groups)
        for (size_t b = 0; b < gr.items.size(); b += kMaxRows) {
          const int n = (int)std::min<size_t>(kMaxRows, gr.items.size() - b);
          launch_lawson_group(stage, op->precision, gr.real, ditems.as<LawsonItem>() + gr.offset + b, n,
                              gr.row_blocks, h, op->dflag, s);
        }
  };
  const int64_t per_step = 4 * (int64_t)std::max(1, launches);
  const int chunk = (int)std::min<int64_t>({steps, 64, kMaxGraphNodes / per_step});
  int64_t done = 0;
  if (chunk > 1) {
    if (!op->cap_stream) hip_check(hipStreamCreateWithFlags(&op->cap_stream, hipStreamNonBlocking), "stream");
    hip_check(hipStreamBeginCapture(op->cap_stream, hipStreamCaptureModeThreadLocal), "begin capture");
    for (int k = 0; k < chunk; ++k) step(op->cap_stream);
    hipGraph_t graph;
    hip_check(hipStreamEndCapture(op->cap_stream, &graph), "end capture");
    hipGraphExec_t exec;
    hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    hip_check(e, "graph instantiate");
    GraphHolder g(exec);
    for (; done + chunk <= steps; done += chunk) hip_check(hipGraphLaunch(g.e, st), "graph launch");
    hip_check(hipStreamSynchronize(st), "synchronize");  // the graph must outlive its launches
  }
  for (; done < steps; ++done) step(st);
  hip_check(hipStreamSynchronize(st), "synchronize");  // the items must outlive the launches
}

int read_flag(hgf_operator_s* op, hipStream_t st) {
  int flag = 0;
  hip_check(hipMemcpyAsync(&flag, op->dflag, sizeof(int), hipMemcpyDeviceToHost, st), "read flag");
  hip_check(hipStreamSynchronize(st), "synchronize");
  return flag;
}

// Thresholded representation: drop every coefficient with |g| <= threshold
// from the operator's full-grid functions and update the peak count.
// Tile of a network operator's full grid: the (k, l) block of the last two
// positions (the stage kernel's tile), or the whole grid below three modes.
int64_t full_tile_points(const Function& f) {
  int64_t t = 1;
  for (int a = std::max(0, f.ga.n - 4); a < f.ga.n; ++a) t *= f.ga.ext[a];
  return t;
}

void apply_threshold(hgf_operator_s* op, hipStream_t st) {
  for (auto& f : op->fn)
    launch_threshold((double2*)f.y, f.ga.points, op->threshold, full_tile_points(f), op->dcount, st);
  launch_threshold_peak(op->dcount, st);
}

void evolve_impl(hgf_operator_s* op, int64_t steps, double h, hipStream_t st, int scheme) {
  if (scheme == HGF_LAWSON_RK4 && op->layout != HGF_MERGED)
    fail(HGF_EUNSUPPORTED, "the integrating-factor scheme runs on merged-layout operators only");
  if (scheme == HGF_LAWSON_RK4 && op->sys.full)
    fail(HGF_EUNSUPPORTED, "the integrating-factor scheme needs uncoupled sectors (no drive or exchange)");
  if (op->sep) {  // separated layout: classical RK4 on (Gx_i, Gy_i, R)
    separated_evolve(op, steps, h, st);
    op->steps_done += steps;
    op->time_us += steps * h;
    return;
  }
  if (steps == 0) return;
  if (op->fn.empty()) {  // the zero operator stays zero
    op->steps_done += steps;
    op->time_us += steps * h;
    return;
  }
  check_stability(op->fn, h, scheme == HGF_LAWSON_RK4);
  // keep a copy of the states for recovery after a non-finite result
  for (auto& f : op->fn) {
    const size_t bytes = state_bytes(f);
    if (!f.ybak) f.ybak = dmalloc(bytes);
    hip_check(hipMemcpyAsync(f.ybak, f.y, bytes, hipMemcpyDeviceToDevice, st), "backup");
  }
  std::vector<cd> cx0, cy0;
  for (auto& f : op->fn) {
    cx0.push_back(f.cx);
    cy0.push_back(f.cy);
  }
  reset_flag(op, st);
  if (scheme == HGF_LAWSON_RK4) {
    lawson_steps(op, steps, h, st);
  } else if (op->layout == HGF_MERGED && op->threshold > 0.0) {
    // one step at a time, the representation truncated after each
    ensure_plan(op, h);
    for (int64_t k = 0; k < steps; ++k) {
      run_resident(*op->plan, 1, op->dflag, st);
      run_plan_step(*op->plan, op->dflag, st);
      apply_threshold(op, st);
    }
  } else if (op->layout == HGF_MERGED) {
    ensure_plan(op, h);
    run_resident(*op->plan, steps, op->dflag, st);
    const int chunk = graph_chunk(*op->plan, steps);
    int64_t done = 0;
    if (chunk > 0) {
      ensure_graph(op, h, chunk);
      while (steps - done >= chunk) {
        hip_check(hipGraphLaunch((hipGraphExec_t)op->graph_exec, st), "graph launch");
        done += chunk;
      }
    }
    if (!op->plan->groups.empty() || !op->plan->generic.empty())
      for (; done < steps; ++done) run_plan_step(*op->plan, op->dflag, st);
  } else {
    for (int64_t s = 0; s < steps; ++s)
      for (auto& f : op->fn) split_step(op, f, h, st);
  }
  hip_check(hipGetLastError(), "kernel launch");
  const int flag = read_flag(op, st);
  if (flag & 2) {
    op->error_state = 1;
    fail(HGF_EDEVICE, "stage kernel launched outside its configuration contract");
  }
  if (flag) {
    for (size_t i = 0; i < op->fn.size(); ++i) {
      const size_t bytes = state_bytes(op->fn[i]);
      hip_check(hipMemcpyAsync(op->fn[i].y, op->fn[i].ybak, bytes, hipMemcpyDeviceToDevice, st), "restore");
      launch_shadow(op->precision, op->fn[i].ga, op->fn[i].y, op->fn[i].yf, st);
      op->fn[i].cx = cx0[i];
      op->fn[i].cy = cy0[i];
    }
    hip_check(hipStreamSynchronize(st), "synchronize");
    op->error_state = 1;
    fail(HGF_ENONFINITE, "non-finite value in an evolved function; state restored to the start of this call");
  }
  op->steps_done += steps;
  op->time_us += steps * h;
}

// Batched evolve: all members' functions advance together, one grouped launch
// per stage and element-type group, captured in a HIP graph.  Members with
// fewer steps drop out: the batch runs in phases between consecutive distinct
// step counts, each phase with its own launch plan and graph.
void batch_impl(hgf_operator* ops, int n, const std::vector<int64_t>& steps, const double* dt, hipStream_t st) {
  DBuf dflag(sizeof(int));
  hip_check(hipMemsetAsync(dflag.p, 0, sizeof(int), st), "reset flag");
  for (int i = 0; i < n; ++i)
    for (auto& f : ops[i]->fn) {
      const size_t bytes = state_bytes(f);
      if (!f.ybak) f.ybak = dmalloc(bytes);
      hip_check(hipMemcpyAsync(f.ybak, f.y, bytes, hipMemcpyDeviceToDevice, st), "backup");
    }
  std::vector<int64_t> levels(steps.begin(), steps.end());
  std::sort(levels.begin(), levels.end());
  levels.erase(std::unique(levels.begin(), levels.end()), levels.end());
  hipStream_t cap = nullptr;
  hip_check(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "stream");
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() {
      if (s) (void)hipStreamDestroy(s);
    }
  } sg{cap};
  int64_t prev = 0;
  for (int64_t level : levels) {
    const int64_t nst = level - prev;
    prev = level;
    if (nst <= 0) continue;
    std::vector<PlanItem> items;
    for (int i = 0; i < n; ++i)
      if (steps[i] >= level)
        for (auto& f : ops[i]->fn) items.push_back({&f, ops[i]->precision, dt[i]});
    if (items.empty()) continue;
    std::unique_ptr<StepPlan> plan(build_plan(items));
    run_resident(*plan, nst, dflag.as<int>(), st);
    const int chunk = graph_chunk(*plan, nst);
    int64_t done = 0;
    if (chunk > 0) {
      GraphHolder g(capture_steps(*plan, dflag.as<int>(), chunk, cap));
      while (nst - done >= chunk) {
        hip_check(hipGraphLaunch(g.e, st), "graph launch");
        done += chunk;
      }
      // the graph must outlive its launches
      hip_check(hipStreamSynchronize(st), "synchronize");
    }
    if (!plan->groups.empty() || !plan->generic.empty())
      for (; done < nst; ++done) run_plan_step(*plan, dflag.as<int>(), st);
    // the plan's device buffers must outlive the launches that read them
    hip_check(hipStreamSynchronize(st), "synchronize");
  }
  hip_check(hipGetLastError(), "kernel launch");
  int flag = 0;
  hip_check(hipMemcpyAsync(&flag, dflag.p, sizeof(int), hipMemcpyDeviceToHost, st), "read flag");
  hip_check(hipStreamSynchronize(st), "synchronize");
  if (flag) {
    for (int i = 0; i < n; ++i) {
      for (auto& f : ops[i]->fn) {
        hip_check(hipMemcpyAsync(f.y, f.ybak, state_bytes(f), hipMemcpyDeviceToDevice, st), "restore");
        launch_shadow(ops[i]->precision, f.ga, f.y, f.yf, st);
      }
      ops[i]->error_state = 1;
    }
    hip_check(hipStreamSynchronize(st), "synchronize");
    fail((flag & 2) ? HGF_EDEVICE : HGF_ENONFINITE,
         "non-finite value (or a launch outside its contract) in a batch member; every member restored to the start "
         "of this call");
  }
  for (int i = 0; i < n; ++i) {
    ops[i]->steps_done += steps[i];
    ops[i]->time_us += steps[i] * dt[i];
  }
}

}  // namespace hgf
