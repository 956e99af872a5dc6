// Discrete-adjoint gradient of J = <psi0|A(T)|psi0> with respect to the
// system parameters (the transposed stencil on the forward stage kernels).
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

// ------------------------------------------------------------------ gradient

// L^T of a sector's generator as tables of the same stencil form:
// (L^T mu)(m) = lam(m) mu(m) + sum_j [alpha_j(m_j + 1) mu(m + e_j) + beta_j(m_j - 1) mu(m - e_j)],
// i.e. alpha'_j(m) = beta_j(m - 1) (0 at m = 0) and beta'_j(m) = alpha_j(m + 1)
// (0 at the top of the axis): transpose only, no conjugation.
SectorTables transposed_tables(const SectorTables& t) {
  SectorTables r = t;
  for (int j = 0; j < t.n; ++j) {
    const int e = t.ext[j];
    for (int m = 0; m < e; ++m) {
      r.alpha[j][m] = m >= 1 ? t.beta[j][m - 1] : 0.0;
      r.beta[j][m] = m + 1 < e ? t.alpha[j][m + 1] : 0.0;
    }
  }
  return r;
}

// Longest reverse segment captured as one graph (about 10 nodes per step).
constexpr int64_t kGradGraphSteps = 512;
// A segment keeps every step's stage grids X1, V1, V2 next to its state when
// they fit in this many bytes (the reverse sweep then recomputes nothing, and
// keeps each step's adjoint grids, as many bytes again, for the segment's
// parameter products); otherwise, or with HGF_GRAD_STORE=0 in the
// environment, it keeps the states only and recomputes the three stages of
// each step in the sweep (the same numbers either way).
constexpr int64_t kGradStoreBytes = (int64_t)2 << 30;

// J's part from one sector: its grid contracted with the weights `dw`.
static cd sector_value(const Function& f, const double2* dw, hipStream_t st) {
  std::vector<int> start = {0, expect_blocks(f.ga)};
  cd one = 1.0;
  DBuf dpart(start[1] * sizeof(double2)), dstart(2 * sizeof(int)), dcoef(sizeof(double2)), dout(sizeof(double2));
  hip_check(hipMemcpyAsync(dstart.p, start.data(), 2 * sizeof(int), hipMemcpyHostToDevice, st), "upload");
  hip_check(hipMemcpyAsync(dcoef.p, &one, sizeof(double2), hipMemcpyHostToDevice, st), "upload");
  launch_expect_partial(f.ga, f.y, true, dw, dpart.as<double2>(), st);
  launch_expect_final(dpart.as<double2>(), dstart.as<int>(), dcoef.as<double2>(), 1, make_double2(0, 0),
                      dout.as<double2>(), st);
  double2 r;
  hip_check(hipMemcpyAsync(&r, dout.p, sizeof(double2), hipMemcpyDeviceToHost, st), "download");
  hip_check(hipStreamSynchronize(st), "synchronize");
  return cd(r.x, r.y);
}

// Parameter derivatives from one sector's accumulator planes Q: the marginals
// of Q against the derivative tables of every parameter (unit systems).
static void sector_grad(const System& sys, const Function& f, const double2* Q, std::vector<cd>& grad,
                        hipStream_t st) {
  const int nb = marginal_bins(f.ga);
  DBuf dbins(nb * sizeof(double2));
  launch_marginals(f.ga, Q, dbins.as<double2>(), st);
  hip_check(hipGetLastError(), "kernel launch");
  std::vector<cd> bins(nb);
  hip_check(hipMemcpyAsync(bins.data(), dbins.p, nb * sizeof(double2), hipMemcpyDeviceToHost, st), "download");
  hip_check(hipStreamSynchronize(st), "synchronize");
  int tot_e = 0;
  for (int j = 0; j < sys.n; ++j) tot_e += f.ga.ext[j];
  cd S0 = 0.0;
  for (int v = 0; v < f.ga.ext[0]; ++v) S0 += bins[v];
  for (size_t p = 0; p < grad.size(); ++p) {
    const System u = unit_system(sys, (int)p);
    const SectorTables tp = sector_tables(u, f.tab.d);
    cd g = tp.lam0 * S0;
    for (int j = 0; j < sys.n; ++j) {
      for (int v = 0; v < f.ga.ext[j]; ++v) {
        g += tp.lam[j][v] * bins[f.ga.off[j] + v];
        g += tp.alpha[j][v] * bins[tot_e + f.ga.off[j] + v];
        g += tp.beta[j][v] * bins[2 * tot_e + f.ga.off[j] + v];
      }
    }
    grad[p] += g;
  }
}

// Small sectors (at most four axes and 1024 points, the generator and its
// transpose both on the resident integrator's layout) run the gradient on chip
// and together, one workgroup per sector in every launch: the forward pass
// with its checkpoints on the resident integrator; per segment, from the last,
// one launch of the resident integrator that also records every step's y, X1,
// V1, V2 (the same arithmetic as the plain form) and one launch of
// k_adjoint_resident (the reverse sweep with its parameter products).  `fas`
// are the sectors' transposed functions.
static void grad_on_chip(const System& sys, const std::vector<Function*>& fs, std::vector<Function>& fas,
                         const std::vector<std::vector<cd>>& ws, int64_t M, int ce, double dt, cd& value,
                         std::vector<cd>& grad, int* dflag, hipStream_t st) {
  const size_t K = fs.size();
  if (K == 0) return;
  const int64_t nseg = (M + ce - 1) / ce;
  const int64_t seg_steps = std::min<int64_t>(ce, std::max<int64_t>(M, 1));
  const int64_t rest = M - (nseg - 1) * ce;  // steps of the last segment
  // With several segments the recompute of segment c - 1 runs beside the
  // reverse sweep of segment c (two streams, two record buffers per sector,
  // as on the stage launches); HGF_GRAD_OVERLAP=0 runs them in sequence
  // (the same results).
  const char* ov_env = std::getenv("HGF_GRAD_OVERLAP");
  const bool overlap = nseg > 1 && !(ov_env && std::string(ov_env) == "0");
  const int nbuf = overlap ? 2 : 1;
  struct Sector {
    DBuf ckpt, seg, mu, Q, wt, y0, dw;
    Sector(int64_t pts, int64_t nseg, int64_t seg_steps, int n, size_t nw, int nbuf)
        : ckpt((size_t)(nseg + 1) * pts * sizeof(double2)),
          seg((size_t)(4 * seg_steps * nbuf) * pts * sizeof(double2)),
          mu(pts * sizeof(double2)),
          Q((size_t)(1 + 2 * n) * pts * sizeof(double2)),
          wt(pts * sizeof(double2)),
          y0(pts * sizeof(double2)),
          dw(nw * sizeof(double2)) {}
  };
  std::vector<std::unique_ptr<Sector>> sec;
  int threads = 0, athreads = 0, lds = 0, alds = 0;
  for (size_t k = 0; k < K; ++k) {
    Function& f = *fs[k];
    const int64_t pts = f.ga.points;
    const size_t gb = pts * sizeof(double2);
    sec.emplace_back(new Sector(pts, nseg, seg_steps, sys.n, ws[k].size(), nbuf));
    Sector& x = *sec.back();
    hip_check(hipMemcpyAsync(x.dw.p, ws[k].data(), ws[k].size() * sizeof(double2), hipMemcpyHostToDevice, st),
              "upload");
    launch_fill_weights(f.ga, x.dw.as<double2>(), x.wt.as<double2>(), st);
    hip_check(hipMemcpyAsync(x.ckpt.p, f.y, gb, hipMemcpyDeviceToDevice, st), "checkpoint");
    hip_check(hipMemcpyAsync(x.y0.p, f.y, gb, hipMemcpyDeviceToDevice, st), "copy");
    threads = std::max(threads, f.res_threads);
    athreads = std::max(athreads, fas[k].res_threads);
    lds = std::max(lds, f.res_lds_bytes);
    alds = std::max(alds, fas[k].res_lds_bytes);
  }
  if (std::max(lds, alds) > 65536) hip_check(grad_resident_allow_lds(kResidentLdsMax), "LDS limit");
  // every sector's state and checkpoints, for the batched checkpoint copies
  std::vector<CheckpointItem> cki(K);
  int64_t max_pts = 0;
  for (size_t k = 0; k < K; ++k) {
    cki[k] = CheckpointItem{(double2*)fs[k]->y, sec[k]->ckpt.as<double2>(), fs[k]->ga.points};
    max_pts = std::max(max_pts, fs[k]->ga.points);
  }
  DBuf dcki(K * sizeof(CheckpointItem));
  hip_check(hipMemcpy(dcki.p, cki.data(), K * sizeof(CheckpointItem), hipMemcpyHostToDevice), "upload items");
  const CheckpointItem* ckp = dcki.as<CheckpointItem>();
  // forward, a checkpoint of every sector after every `ce` steps
  std::vector<PlanItem> items;
  for (Function* f : fs) items.push_back(PlanItem{f, HGF_FP64, dt});
  std::unique_ptr<StepPlan> plan(build_plan(items, true));
  const int64_t full = M / ce;
  for (int64_t c = 1; c <= full; ++c) {
    run_resident(*plan, ce, dflag, st);
    launch_checkpoint_batch(ckp, (int)K, max_pts, c, true, st);
  }
  run_resident(*plan, M - full * ce, dflag, st);
  for (size_t k = 0; k < K; ++k) value += sector_value(*fs[k], sec[k]->dw.as<double2>(), st);
  // reverse sweep: mu_M = w; items per record buffer b, for a full segment
  // (l = 0) and for the last one (l = 1), at [(2 b + l) K + k]
  std::vector<ResidentItem> ri(4 * K);
  std::vector<AdjointResidentItem> ai(4 * K);
  for (size_t k = 0; k < K; ++k) {
    Function& f = *fs[k];
    Sector& x = *sec[k];
    const int64_t pts = f.ga.points;
    hip_check(hipMemcpyAsync(x.mu.p, x.wt.p, pts * sizeof(double2), hipMemcpyDeviceToDevice, st), "seed");
    launch_fill_zero(x.Q.as<double2>(), (int64_t)(1 + 2 * sys.n) * pts, st);
    for (int b = 0; b < 2; ++b)
      for (int l = 0; l < 2; ++l) {
        double2* buf = x.seg.as<double2>() + (b < nbuf ? b : 0) * 4 * seg_steps * pts;
        ResidentItem& r = ri[(2 * b + l) * K + k];
        r = ResidentItem{};
        r.g = f.rga;
        r.y = f.y;
        r.x1 = f.s1;
        r.steps = (int)(l == 0 ? seg_steps : rest);
        r.h = dt;
        r.rec = buf;
        AdjointResidentItem& a = ai[(2 * b + l) * K + k];
        a = AdjointResidentItem{};
        a.g = fas[k].rga;
        a.mu = x.mu.p;
        a.seg = buf;
        a.Q = x.Q.p;
        a.steps = r.steps;
        a.h = dt;
      }
  }
  DBuf dri(ri.size() * sizeof(ResidentItem)), dai(ai.size() * sizeof(AdjointResidentItem));
  hip_check(hipMemcpy(dri.p, ri.data(), ri.size() * sizeof(ResidentItem), hipMemcpyHostToDevice), "upload items");
  hip_check(hipMemcpy(dai.p, ai.data(), ai.size() * sizeof(AdjointResidentItem), hipMemcpyHostToDevice),
            "upload items");
  const int n = fs[0]->ga.n;
  auto item_at = [&](int64_t c) { return (size_t)(2 * (overlap ? (c & 1) : 0) + (c == nseg - 1 ? 1 : 0)) * K; };
  // restore every sector's state to checkpoint c and record segment c
  auto record = [&](int64_t c, hipStream_t s) {
    launch_checkpoint_batch(ckp, (int)K, max_pts, c, false, s);
    launch_grad_record(dri.as<ResidentItem>() + item_at(c), (int)K, n, threads, lds, dflag, s);
  };
  auto sweep = [&](int64_t c, hipStream_t s) {
    launch_grad_reverse(dai.as<AdjointResidentItem>() + item_at(c), (int)K, n, athreads, alds, dflag, s);
  };
  if (!overlap) {
    for (int64_t c = nseg - 1; c >= 0; --c) {
      record(c, st);
      sweep(c, st);
    }
  } else {
    hipStream_t sb = nullptr;
    hip_check(hipStreamCreateWithFlags(&sb, hipStreamNonBlocking), "stream");
    // (on every exit, error paths included, both streams are drained before
    // the events recorded on them and the second stream are destroyed)
    struct Guard {
      hipStream_t s, main;
      hipEvent_t e[5] = {};
      ~Guard() {
        if (s) (void)hipStreamSynchronize(s);
        (void)hipStreamSynchronize(main);
        for (hipEvent_t x : e)
          if (x) (void)hipEventDestroy(x);
        if (s) (void)hipStreamDestroy(s);
      }
    } gd{sb, st};  // events 0, 1: record into buffer b done; 2, 3: sweep of buffer b done; 4: start
    for (hipEvent_t& x : gd.e) hip_check(hipEventCreateWithFlags(&x, hipEventDisableTiming), "event");
    hip_check(hipEventRecord(gd.e[4], st), "record");
    hip_check(hipStreamWaitEvent(sb, gd.e[4], 0), "wait");
    auto record_on_sb = [&](int64_t c) {
      const int b = (int)(c & 1);
      if (c + 2 <= nseg - 1) hip_check(hipStreamWaitEvent(sb, gd.e[2 + b], 0), "wait");  // buffer b free
      record(c, sb);
      hip_check(hipEventRecord(gd.e[b], sb), "record");
    };
    record_on_sb(nseg - 1);
    for (int64_t c = nseg - 1; c >= 0; --c) {
      const int b = (int)(c & 1);
      hip_check(hipStreamWaitEvent(st, gd.e[b], 0), "wait");
      sweep(c, st);
      hip_check(hipEventRecord(gd.e[2 + b], st), "record");
      if (c >= 1) record_on_sb(c - 1);
    }
    // both streams drained before the events (recorded on both) and the
    // second stream are destroyed
    hip_check(hipStreamSynchronize(sb), "synchronize");
    hip_check(hipStreamSynchronize(st), "synchronize");
  }
  hip_check(hipGetLastError(), "kernel launch");
  for (size_t k = 0; k < K; ++k) {
    const int64_t pts = fs[k]->ga.points;
    hip_check(hipMemcpyAsync(fs[k]->y, sec[k]->y0.p, pts * sizeof(double2), hipMemcpyDeviceToDevice, st),
              "restore");
    sector_grad(sys, *fs[k], sec[k]->Q.as<double2>(), grad, st);
  }
}

void grad_impl(const System& sys, const hgf_operator_desc* desc, const hgf_state_desc* psi, double T,
                      double dt, int ce, double* value_out, double* grad_out, hipStream_t st) {
  const int64_t M = check_steps(T, dt);
  if (ce < 1) fail(HGF_EINVAL, "checkpoint_every must be >= 1");
  if (sys.full) fail(HGF_EUNSUPPORTED, "gradients need uncoupled sectors (no drive or exchange)");
  validate_state(sys, psi);
  hgf_operator_s op;
  op.sys = sys;
  op.precision = HGF_FP64;
  op.layout = HGF_MERGED;
  hip_check(hipGetDevice(&op.device), "hipGetDevice");
  hgf_operator_desc d2 = *desc;
  d2.layout = HGF_MERGED;
  d2.precision = HGF_FP64;
  struct OpGuard {
    hgf_operator_s& o;
    ~OpGuard() {
      for (auto& f : o.fn) free_function(f);
      if (o.dflag) dfree(*(void**)&o.dflag);
    }
  } guard{op};
  op.dflag = (int*)dmalloc(sizeof(int));
  hipStream_t cap = nullptr;
  hip_check(hipStreamCreateWithFlags(&cap, hipStreamNonBlocking), "stream");
  struct StreamGuard {
    hipStream_t s;
    ~StreamGuard() {
      if (s) (void)hipStreamDestroy(s);
    }
  } sg{cap};
  build_functions(&op, &d2, false);
  check_stability(op.fn, dt);
  const auto amps = all_amps(sys, psi);
  const int P = num_params(sys.n);
  std::vector<cd> grad(P, 0.0);
  cd value = 0.0;
  reset_flag(&op, st);
  // sectors small enough for the gradient on chip (HGF_RESIDENT=0 or
  // HGF_GRAD_STORE=0 keep every sector on the stage launches)
  std::vector<Function*> chip;
  std::vector<Function> chip_t;  // their transposed functions
  std::vector<std::vector<cd>> chip_w;
  {
    const char* store_env = std::getenv("HGF_GRAD_STORE");
    const bool no_store = store_env && std::string(store_env) == "0";
    chip_t.reserve(op.fn.size());
    for (auto& f : op.fn) {
      if (no_store || !f.resident || f.ga.n > 4 || f.ga.points > 2 * 512) continue;
      chip_t.emplace_back();
      Function& fa = chip_t.back();
      fa.tab = transposed_tables(f.tab);
      fill_grid_args(fa, HGF_FP64, false);
      if (!fa.resident || fa.res_threads != f.res_threads || fa.res_lds_bytes != f.res_lds_bytes) {
        free_function(fa);
        chip_t.pop_back();
        continue;
      }
      chip.push_back(&f);
      chip_w.push_back(sector_weights(sys, f, amps));
    }
  }
  struct FreeChip {
    std::vector<Function>& v;
    ~FreeChip() {
      for (auto& f : v) free_function(f);
    }
  } chip_guard{chip_t};
  grad_on_chip(sys, chip, chip_t, chip_w, M, ce, dt, value, grad, op.dflag, st);
  for (auto& f : op.fn) {
    if (std::find(chip.begin(), chip.end(), &f) != chip.end()) continue;
    const int64_t pts = f.ga.points;
    const size_t gb = pts * sizeof(double2);
    const int64_t nseg = (M + ce - 1) / ce;
    const int64_t seg_steps = std::min<int64_t>(ce, std::max<int64_t>(M, 1));
    const char* store_env = std::getenv("HGF_GRAD_STORE");  // "0": keep states only
    const bool store = 4 * seg_steps * (int64_t)gb <= kGradStoreBytes && !(store_env && std::string(store_env) == "0");
    const int64_t per_step = store ? 4 : 1;  // grids kept per step: y (and X1, V1, V2)
    // adjoint grids: mu, and a set of Vb2, Vb1, Xb1 and a copy of mu per
    // step of a segment (with stored stages: the parameter products then run
    // once per segment) or one set
    const int64_t adj_sets = store ? seg_steps : 1;
    DBuf ckpt((size_t)(nseg + 1) * gb), segbuf((size_t)(seg_steps * per_step) * gb), mu(gb),
        adj((size_t)(4 * adj_sets) * gb), Q((size_t)(1 + 2 * sys.n) * gb), wt(gb);
    // the adjoint stencils run on the forward stage kernels of L^T
    Function fa;
    struct FreeOnExit {
      Function& f;
      ~FreeOnExit() { free_function(f); }
    } fa_guard{fa};
    fa.tab = transposed_tables(f.tab);
    fill_grid_args(fa, HGF_FP64, false);
    DBuf zero(gb);
    launch_fill_zero(zero.as<double2>(), pts, st);
    const auto w = sector_weights(sys, f, amps);
    DBuf dw(w.size() * sizeof(double2));
    hip_check(hipMemcpyAsync(dw.p, w.data(), w.size() * sizeof(double2), hipMemcpyHostToDevice, st), "upload");
    launch_fill_weights(f.ga, dw.as<double2>(), wt.as<double2>(), st);
    // forward with checkpoints (f.y is the working state)
    double2* ck = ckpt.as<double2>();
    hip_check(hipMemcpyAsync(ck, f.y, gb, hipMemcpyDeviceToDevice, st), "checkpoint");
    DBuf y0(gb);
    hip_check(hipMemcpyAsync(y0.p, f.y, gb, hipMemcpyDeviceToDevice, st), "copy");
    std::unique_ptr<StepPlan> fplan(build_plan({PlanItem{&f, HGF_FP64, dt}}, false));
    // forward: graphs of up to 64 steps, a checkpoint after every `ce` steps
    {
      const int64_t full = M / ce;
      if (full > 0) {
        const int chunk = (int)std::min<int64_t>(ce, 64);
        GraphHolder g(capture_steps(*fplan, op.dflag, chunk, cap));
        for (int64_t c = 1; c <= full; ++c) {
          int64_t done = 0;
          for (; done + chunk <= ce; done += chunk) hip_check(hipGraphLaunch(g.e, st), "graph launch");
          for (; done < ce; ++done) run_plan_step(*fplan, op.dflag, st);
          hip_check(hipMemcpyAsync(ck + c * pts, f.y, gb, hipMemcpyDeviceToDevice, st), "checkpoint");
        }
        hip_check(hipStreamSynchronize(st), "synchronize");
      }
      for (int64_t s = full * ce; s < M; ++s) run_plan_step(*fplan, op.dflag, st);
    }
    value += sector_value(f, dw.as<double2>(), st);
    // reverse sweep: mu_M = w
    hip_check(hipMemcpyAsync(mu.p, wt.p, gb, hipMemcpyDeviceToDevice, st), "seed");
    launch_fill_zero(Q.as<double2>(), (int64_t)(1 + 2 * sys.n) * pts, st);
    double2* seg = segbuf.as<double2>();
    double2* Qp = Q.as<double2>();
    // One segment of L steps: recompute y_{s0} .. y_{s0+L-1} from the state in
    // f.y into a segment buffer (with each step's X1, V1, V2 when `store`),
    // then sweep them in reverse.  The work of a segment depends only on L
    // (and the buffer), so it is captured once per length.  The stage launches
    // are those of the forward pass (same kernel, shape and operands), so the
    // recomputed states equal the checkpointed trajectory bit for bit.
    auto slot = [&](double2* seg, int64_t i, int k) { return seg + (i * per_step + k) * pts; };  // k: y, X1, V1, V2
    auto recompute = [&](double2* seg, int64_t L, hipStream_t s) {
      for (int64_t i = 0; i < L; ++i) {
        launch_copy2(slot(seg, i, 0), (const double2*)f.y, pts, s);
        if (!store) {
          if (i + 1 < L) run_plan_step(*fplan, op.dflag, s);
          continue;
        }
        double2 *y_ = slot(seg, i, 0), *x1_ = slot(seg, i, 1), *v1_ = slot(seg, i, 2), *v2_ = slot(seg, i, 3);
        stage_launch(f, HGF_FP64, 1, y_, nullptr, y_, nullptr, x1_, dt, op.dflag, s);
        stage_launch(f, HGF_FP64, 2, x1_, x1_, y_, nullptr, v1_, dt, op.dflag, s);
        stage_launch(f, HGF_FP64, 3, v1_, x1_, y_, nullptr, v2_, dt, op.dflag, s);
        if (i + 1 < L) stage_launch(f, HGF_FP64, 4, v2_, x1_, f.y, nullptr, nullptr, dt, op.dflag, s);
      }
    };
    // With stored stages the parameter products of the whole segment run after
    // its sweep in one launch per four modes (k_adjoint_q_seg: the same sums in
    // the same order as step by step, with one pass over Q); otherwise after
    // each step (k_adjoint_q).
    auto reverse = [&](double2* seg, int64_t L, hipStream_t s) {
      for (int64_t i = L - 1; i >= 0; --i) {
        double2* yn = slot(seg, i, 0);
        const double2 *x1 = (const double2*)f.s1, *v1 = (const double2*)f.s2, *v2 = (const double2*)f.s3;
        if (store) {
          x1 = slot(seg, i, 1);
          v1 = slot(seg, i, 2);
          v2 = slot(seg, i, 3);
        } else {  // forward stage grids X1, V1, V2 of this step (FP64: s1, s2, s3)
          stage_launch(f, HGF_FP64, 1, yn, nullptr, yn, nullptr, f.s1, dt, op.dflag, s);
          stage_launch(f, HGF_FP64, 2, f.s1, f.s1, yn, nullptr, f.s2, dt, op.dflag, s);
          stage_launch(f, HGF_FP64, 3, f.s2, f.s1, yn, nullptr, f.s3, dt, op.dflag, s);
        }
        double2* set = adj.as<double2>() + (store ? i : 0) * 4 * pts;
        double2 *pm = mu.as<double2>(), *pv2 = set, *pv1 = set + pts, *px = set + 2 * pts, *pmc = set + 3 * pts;
        // stage-1 form (out = h' L^T in): B1, B2 and B3's stencil part
        stage_launch(fa, HGF_FP64, 1, pm, nullptr, pm, nullptr, pv2, 0.5 * dt, op.dflag, s);
        stage_launch(fa, HGF_FP64, 1, pv2, nullptr, pv2, nullptr, pv1, dt / 3.0, op.dflag, s);
        stage_launch(fa, HGF_FP64, 1, pv1, nullptr, pv1, nullptr, px, 0.25 * dt, op.dflag, s);
        launch_adjoint_x(pts, pm, pv2, pv1, px, pmc, s);
        if (!store) launch_adjoint_q(f.ga, pmc, pv2, pv1, px, v2, v1, x1, yn, Qp, dt, s);
        // stage-4 form (y += x1 + (h'/2) L^T in) with x1 = 0, h' = 2h: B4
        stage_launch(fa, HGF_FP64, 4, px, zero.p, pm, nullptr, nullptr, 2.0 * dt, op.dflag, s);
      }
      if (store) launch_adjoint_q_segment(f.ga, adj.as<double2>(), seg, (int)L, Qp, dt, s);
    };
    // graphs by (part, length, buffer): part 0 = recompute and reverse of one
    // segment, 1 = recompute alone, 2 = reverse alone
    std::map<std::vector<int64_t>, std::unique_ptr<GraphHolder>> seg_graphs;
    auto graph_of = [&](int part, int64_t L, int b, double2* sb) -> hipGraphExec_t {
      const std::vector<int64_t> key = {part, L, b};
      auto it = seg_graphs.find(key);
      if (it == seg_graphs.end()) {
        hip_check(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
        try {
          if (part != 2) recompute(sb, L, cap);
          if (part != 1) reverse(sb, L, cap);
        } catch (...) {
          hipGraph_t partial;
          if (hipStreamEndCapture(cap, &partial) == hipSuccess) (void)hipGraphDestroy(partial);
          throw;
        }
        hipGraph_t graph;
        hip_check(hipStreamEndCapture(cap, &graph), "end capture");
        hipGraphExec_t exec;
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        hip_check(e, "graph instantiate");
        it = seg_graphs.emplace(key, std::unique_ptr<GraphHolder>(new GraphHolder(exec))).first;
      }
      return it->second->e;
    };
    // With stored stages the recompute of segment c - 1 touches only f.y and
    // its own segment buffer, and the reverse sweep of segment c only the
    // adjoint buffers and the other segment buffer: the two run side by side
    // on two streams (each launch of this small grid leaves most of the chip
    // idle), alternating between two segment buffers.  HGF_GRAD_OVERLAP=0
    // runs them one after the other.
    const char* ov_env = std::getenv("HGF_GRAD_OVERLAP");
    const bool overlap = store && nseg > 1 && ce <= kGradGraphSteps && !(ov_env && std::string(ov_env) == "0");
    if (!overlap) {
      for (int64_t c = nseg - 1; c >= 0; --c) {
        const int64_t s0 = c * ce, L = std::min<int64_t>(ce, M - s0);
        hip_check(hipMemcpyAsync(f.y, ck + c * pts, gb, hipMemcpyDeviceToDevice, st), "restore");
        if (L > kGradGraphSteps) {  // long segments run without a graph
          recompute(seg, L, st);
          reverse(seg, L, st);
          continue;
        }
        hip_check(hipGraphLaunch(graph_of(0, L, 0, seg), st), "graph launch");
      }
    } else {
      DBuf segbuf2((size_t)(seg_steps * per_step) * gb);
      double2* bufs[2] = {seg, segbuf2.as<double2>()};
      hipStream_t sb = nullptr;
      hip_check(hipStreamCreateWithFlags(&sb, hipStreamNonBlocking), "stream");
      StreamGuard sbg{sb};
      struct Events {
        hipStream_t a, b;
        hipEvent_t e[5] = {};
        ~Events() {  // both streams drained first (error paths included)
          (void)hipStreamSynchronize(a);
          (void)hipStreamSynchronize(b);
          for (hipEvent_t x : e)
            if (x) (void)hipEventDestroy(x);
        }
      } ev{sb, st};  // 0, 1: recompute into buffer b done; 2, 3: reverse of buffer b done; 4: start
      for (hipEvent_t& x : ev.e) hip_check(hipEventCreateWithFlags(&x, hipEventDisableTiming), "event");
      hip_check(hipEventRecord(ev.e[4], st), "record");
      hip_check(hipStreamWaitEvent(sb, ev.e[4], 0), "wait");
      auto len = [&](int64_t c) { return std::min<int64_t>(ce, M - c * ce); };
      auto launch_recompute = [&](int64_t c) {
        const int b = (int)(c & 1);
        if (c + 2 <= nseg - 1) hip_check(hipStreamWaitEvent(sb, ev.e[2 + b], 0), "wait");  // buffer free
        hip_check(hipMemcpyAsync(f.y, ck + c * pts, gb, hipMemcpyDeviceToDevice, sb), "restore");
        hip_check(hipGraphLaunch(graph_of(1, len(c), b, bufs[b]), sb), "graph launch");
        hip_check(hipEventRecord(ev.e[b], sb), "record");
      };
      launch_recompute(nseg - 1);
      for (int64_t c = nseg - 1; c >= 0; --c) {
        const int b = (int)(c & 1);
        hip_check(hipStreamWaitEvent(st, ev.e[b], 0), "wait");
        hip_check(hipGraphLaunch(graph_of(2, len(c), b, bufs[b]), st), "graph launch");
        hip_check(hipEventRecord(ev.e[2 + b], st), "record");
        if (c >= 1) launch_recompute(c - 1);
      }
      hip_check(hipStreamSynchronize(sb), "synchronize");
      hip_check(hipStreamSynchronize(st), "synchronize");
    }
    hip_check(hipStreamSynchronize(st), "synchronize");  // graphs are destroyed with seg_graphs
    // leave the function at its initial state
    hip_check(hipMemcpyAsync(f.y, y0.p, gb, hipMemcpyDeviceToDevice, st), "restore");
    sector_grad(sys, f, Q.as<double2>(), grad, st);
  }
  if (read_flag(&op, st)) fail(HGF_ENONFINITE, "non-finite value during the gradient sweep");
  value_out[0] = value.real();
  value_out[1] = value.imag();
  for (int p = 0; p < P; ++p) {
    grad_out[2 * p] = grad[p].real();
    grad_out[2 * p + 1] = grad[p].imag();
  }
}

}  // namespace hgf
