// Launch-shape autotuner of the tiled stage kernels and its text cache.
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

// ------------------------------------------------------------------ launch-shape autotuner
// The tiled stage kernel's launch shape (fast axes, workgroup size, XCD tile
// order, pipelined loads) is chosen per grid shape by timing candidate shapes
// on the function's own buffers.  Results are kept in a text cache, one line
// per shape: "<key> <nfast> <threads> <xblock> <pipe> <wgs_per_cu> <walk_block> <stage_us>", the key
// naming the device (architecture, CU count), precision, real or complex grid
// and the extents.

// Re-configure one function's stage kernel; the function is left unchanged
// when the shape is not feasible (HGF_EINVAL).
void retile(Function& f, int precision, const TileChoice& c) {
  if (f.full) fail(HGF_EINVAL, "a network operator's shape is set by hgf_set_tile_config's network form");
  if (f.split) {
    if (c.nfast == 0) return;
    fail(HGF_EUNSUPPORTED, "split-layout functions run the classical stage kernel only");
  }
  GridArgs g = f.ga;
  if (c.nfast == 0) {
    if (f.real) fail(HGF_EINVAL, "a real grid needs the tiled stage kernel (nfast >= 1)");
    g.blocks = 0;
    g.nfast = 0;
    g.real = 0;
    g.tile_points = 1;
    g.ntiles = g.points;
    g.xblock = 0;
    g.pipe = 0;
  } else if ((!g.phase_linear && precision == HGF_MIXED) || !configure_tiles(g, precision, f.real, c) ||
             (g.real != 0) != f.real) {
    fail(HGF_EINVAL, "tile configuration not feasible for this grid");
  }
  g.tiles = nullptr;
  g.walk = nullptr;
  void* rec = g.blocks > 0 ? upload_tile_records(g, f.tab, precision) : nullptr;
  dfree(f.ttab);
  f.ttab = rec;
  f.ga = g;
  f.tuned_us = 0.0;
}

std::string device_tag() {
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  hipDeviceProp_t prop;
  hip_check(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  return arch + ":" + std::to_string(prop.multiProcessorCount);
}

std::string tune_key(const std::string& dev, const Function& f, int precision) {
  std::string k = dev + (precision == HGF_FP64 ? ":fp64" : ":mixed") + (f.real ? ":real:" : ":complex:");
  for (int j = 0; j < f.ga.n; ++j) k += (j ? "x" : "") + std::to_string(f.ga.ext[j]);
  return k;
}


std::map<std::string, TuneEntry> read_tune_cache(const char* path) {
  std::map<std::string, TuneEntry> m;
  if (!path || !*path) return m;
  std::ifstream in(path);
  std::string line;
  while (std::getline(in, line)) {
    std::istringstream ls(line);
    std::string key;
    TuneEntry e;
    if (ls >> key >> e.c.nfast >> e.c.threads >> e.c.xblock >> e.c.pipe >> e.c.wgs_per_cu >> e.c.wblock >> e.us)
      m[key] = e;
  }
  return m;
}

void write_tune_cache(const char* path, const std::map<std::string, TuneEntry>& m) {
  if (!path || !*path) return;
  const std::string tmp = std::string(path) + ".tmp";
  {
    std::ofstream out(tmp, std::ios::trunc);
    if (!out) fail(HGF_EINVAL, std::string("cannot write tuning cache ") + path);
    out.precision(6);
    for (auto& kv : m)
      out << kv.first << ' ' << kv.second.c.nfast << ' ' << kv.second.c.threads << ' ' << kv.second.c.xblock << ' '
          << kv.second.c.pipe << ' ' << kv.second.c.wgs_per_cu << ' ' << std::max(0, kv.second.c.wblock) << ' '
          << kv.second.us << '\n';
    if (!out) fail(HGF_EINVAL, std::string("cannot write tuning cache ") + path);
  }
  if (std::rename(tmp.c_str(), path) != 0) fail(HGF_EINVAL, std::string("cannot replace tuning cache ") + path);
}

// Candidate launch shapes of a function: the default number of fast axes and
// one fewer; every workgroup size (multiple of 64, <= 512) whose last lane
// round is at least 3/4 full or that the default rule picks; contiguous and
// interleaved XCD orders; pipelined loads where the registers allow.
std::vector<TileChoice> tune_candidates(const Function& f, int precision) {
  std::vector<TileChoice> out;
  if (f.split || f.ga.blocks == 0) return out;
  const int fmax = f.ga.nfast;
  for (int F = fmax; F >= std::max(1, fmax - 1); --F) {
    int64_t T = 1;
    for (int q = 0; q < F; ++q) T *= f.ga.ext[f.ga.n - F + q];
    GridArgs probe = f.ga;
    TileChoice dflt;
    dflt.nfast = F;
    if (!configure_tiles(probe, precision, f.real, dflt)) continue;
    for (int th = 64; th <= 512; th += 64) {
      const int64_t rounds = (T + th - 1) / th;
      if (rounds > kTileRounds) continue;
      const double fill = (double)T / (double)(rounds * th);
      if (fill < 0.75 && th != probe.threads) continue;
      for (int xb : {0, 128})
        for (int pp : {0, 1}) {
          if (pp && f.ga.n - F > kPipeMaxSlow) continue;
          TileChoice c;
          c.nfast = F;
          c.threads = th;
          c.xblock = xb;
          c.pipe = pp;
          GridArgs g = f.ga;
          if (!configure_tiles(g, precision, f.real, c)) continue;
          out.push_back(c);
          // fewer resident workgroups: a narrower front of tiles per XCD
          // keeps more neighbour tiles in L2 (measured faster on the 6^10 grid)
          const int occ = g.occ_max;
          for (int w = occ - 1; w >= std::max(1, occ - 2); --w) {
            TileChoice d = c;
            d.wgs_per_cu = w;
            GridArgs g2 = f.ga;
            if (configure_tiles(g2, precision, f.real, d)) out.push_back(d);
          }
        }
    }
  }
  return out;
}

// The first candidate (in candidate order) within 1 % of the fastest: shapes
// that time alike within run-to-run noise resolve to the same choice.
TuneEntry pick_shape(const std::vector<TileChoice>& cands, const std::vector<double>& times) {
  double tmin = 1e300;
  for (double t : times) tmin = std::min(tmin, t);
  TuneEntry e;
  for (size_t k = 0; k < cands.size(); ++k)
    if (times[k] <= 1.01 * tmin) {
      e.c = cands[k];
      e.us = times[k];
      break;
    }
  return e;
}

// Mean stage time (us) of `steps` RK4 steps of one function alone.
double time_function_steps(Function& f, int precision, double h, int* flag, int steps, hipStream_t st) {
  std::unique_ptr<StepPlan> plan(build_plan({PlanItem{&f, precision, h}}, false));
  run_plan_step(*plan, flag, st);  // warm-up
  hipEvent_t a, b;
  hip_check(hipEventCreate(&a), "event");
  hipError_t e = hipEventCreate(&b);
  if (e != hipSuccess) {
    (void)hipEventDestroy(a);
    hip_check(e, "event");
  }
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } eg{a, b};
  hip_check(hipEventRecord(a, st), "event record");
  for (int i = 0; i < steps; ++i) run_plan_step(*plan, flag, st);
  hip_check(hipEventRecord(b, st), "event record");
  hip_check(hipEventSynchronize(b), "event sync");
  hip_check(hipGetLastError(), "kernel launch");
  float ms = 0.f;
  hip_check(hipEventElapsedTime(&ms, a, b), "event time");
  return 1e3 * (double)ms / (4.0 * steps);
}

TileChoice current_choice(const Function& f) {
  TileChoice c;
  c.nfast = f.ga.blocks > 0 ? f.ga.nfast : 0;
  c.threads = f.ga.threads;
  c.xblock = f.ga.xblock;
  c.pipe = f.ga.pipe;
  c.wgs_per_cu = f.ga.occ_cap;
  c.wblock = f.ga.wblock;
  return c;
}

// Mean stage time (us) of `steps` steps of a set of functions run as one plan.
double time_plan_steps(const std::vector<PlanItem>& items, int* flag, int steps, hipStream_t st) {
  std::unique_ptr<StepPlan> plan(build_plan(items, false));
  run_plan_step(*plan, flag, st);  // warm-up
  hipEvent_t a, b;
  hip_check(hipEventCreate(&a), "event");
  hipError_t e = hipEventCreate(&b);
  if (e != hipSuccess) {
    (void)hipEventDestroy(a);
    hip_check(e, "event");
  }
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } eg{a, b};
  hip_check(hipEventRecord(a, st), "event record");
  for (int i = 0; i < steps; ++i) run_plan_step(*plan, flag, st);
  hip_check(hipEventRecord(b, st), "event record");
  hip_check(hipEventSynchronize(b), "event sync");
  hip_check(hipGetLastError(), "kernel launch");
  float ms = 0.f;
  hip_check(hipEventElapsedTime(&ms, a, b), "event time");
  return 1e3 * (double)ms / (4.0 * steps);
}

// Grouped launches: the functions of all operators that share an axis split
// and element types run as one grouped launch per stage (a batch, or the
// sectors of one operator).  The grouped kernel is tuned as a whole: workgroup
// size, resident workgroups per CU and the number of fast axes (the members'
// own, or one more: a tile that would leave one grid too few tiles to fill
// the chip can pay off across many members, with fewer slow-axis neighbours),
// applied to every member.  The cache key names the group's composition.
void tune_groups(hgf_operator* ops, int n, double h, const std::string& dev,
                        std::map<std::string, TuneEntry>& cache, std::set<std::string>& fresh, int flags,
                        bool& measured, int* flag, hipStream_t st) {
  std::map<std::vector<int>, std::vector<std::pair<hgf_operator_s*, Function*>>> groups;
  for (int i = 0; i < n; ++i) {
    hgf_operator_s* op = ops[i];
    if (op->layout != HGF_MERGED) continue;
    for (auto& f : op->fn)
      if (f.ga.blocks > 0 && !f.resident)
        groups[{f.ga.nfast, f.ga.n - f.ga.nfast, f.ga.real, op->precision}].push_back({op, &f});
  }
  for (auto& kv : groups) {
    auto& mem = kv.second;
    if (mem.size() < 2) continue;
    const int nfast = kv.first[0], prec = kv.first[3];
    // key: device, element types, axis split, member count and a digest of the
    // members' extents (order-independent)
    std::vector<std::string> shapes;
    for (auto& m : mem) shapes.push_back(tune_key("", *m.second, prec));
    std::sort(shapes.begin(), shapes.end());
    uint64_t dig = 1469598103934665603ull;
    for (auto& sh : shapes)
      for (char c : sh) dig = (dig ^ (uint64_t)(unsigned char)c) * 1099511628211ull;
    char buf[64];
    std::snprintf(buf, sizeof buf, "%016llx", (unsigned long long)dig);
    const std::string key = dev + (prec == HGF_FP64 ? ":fp64" : ":mixed") + (kv.first[2] ? ":real" : ":complex") +
                            ":group:nf" + std::to_string(nfast) + ":ns" + std::to_string(kv.first[1]) + ":m" +
                            std::to_string(mem.size()) + ":" + buf;
    auto apply = [&](const TileChoice& c) {
      for (auto& m : mem) retile(*m.second, prec, c);
      for (int i = 0; i < n; ++i) drop_plan(ops[i]);
    };
    auto it = cache.find(key);
    if (it != cache.end() && (!(flags & HGF_TUNE_FORCE) || fresh.count(key))) {
      try {
        apply(it->second.c);
        for (auto& m : mem) m.second->tuned_us = it->second.us;
      } catch (const Error&) {
      }
      continue;
    }
    if (flags & HGF_TUNE_CACHED_ONLY) continue;
    // candidates: the members' fast axes or one more, workgroup sizes every
    // member can use, all resident workgroups per CU or a cap
    std::vector<TileChoice> cands;
    for (int nf = nfast; nf <= nfast + 1; ++nf)
      for (int th = 64; th <= 512; th += 64)
        for (int w : {0, 1, 2, 3, 4, 6}) {
          TileChoice c;
          c.nfast = nf;
          c.threads = th;
          c.xblock = 0;
          c.pipe = 0;
          c.wgs_per_cu = w;
          bool ok = true;
          for (auto& m : mem) {
            GridArgs g = m.second->ga;
            if (!configure_tiles(g, prec, m.second->real, c)) {
              ok = false;
              break;
            }
          }
          if (ok) cands.push_back(c);
        }
    if (cands.empty()) continue;
    std::vector<PlanItem> items;
    for (auto& m : mem) items.push_back({m.second, prec, h});
    std::vector<TileChoice> start;
    for (auto& m : mem) start.push_back(current_choice(*m.second));
    for (auto& m : mem) {
      Function& f = *m.second;
      const size_t bytes = state_bytes(f);
      if (!f.ybak) f.ybak = dmalloc(bytes);
      hip_check(hipMemcpyAsync(f.ybak, f.y, bytes, hipMemcpyDeviceToDevice, st), "backup");
    }
    TuneEntry best;
    best.us = 1e300;
    try {
      const double t0 = time_plan_steps(items, flag, 1, st);
      const int steps = (int)std::max(2.0, std::min(50.0, 2000.0 / std::max(1e-3, 4.0 * t0)));
      std::vector<double> times;
      for (const TileChoice& c : cands) {
        apply(c);
        times.push_back(time_plan_steps(items, flag, steps, st));
      }
      best = pick_shape(cands, times);
      apply(best.c);
    } catch (const Error&) {
      (void)hipStreamSynchronize(st);
      for (size_t k = 0; k < mem.size(); ++k) {
        try {
          retile(*mem[k].second, prec, start[k]);
        } catch (const Error&) {
        }
      }
      for (int i = 0; i < n; ++i) drop_plan(ops[i]);
      throw;
    }
    for (auto& m : mem) {
      Function& f = *m.second;
      f.tuned_us = best.us;
      hip_check(hipMemcpyAsync(f.y, f.ybak, state_bytes(f), hipMemcpyDeviceToDevice, st), "restore");
      launch_shadow(prec, f.ga, f.y, f.yf, st);
    }
    hip_check(hipStreamSynchronize(st), "synchronize");
    cache[key] = best;
    fresh.insert(key);
    measured = true;
  }
}

void autotune_impl(hgf_operator* ops, int n, double h, const char* cache_path, int flags, hipStream_t st) {
  const std::string dev = device_tag();
  std::map<std::string, TuneEntry> cache = read_tune_cache(cache_path);
  std::set<std::string> fresh;  // shapes measured by this call
  bool measured = false;
  DBuf dflag(sizeof(int));
  for (int i = 0; i < n; ++i) {
    hgf_operator_s* op = ops[i];
    if (op->layout != HGF_MERGED) continue;
    for (auto& f : op->fn) {
      if ((f.ga.blocks == 0 && f.real) || f.resident) continue;  // resident: one workgroup, nothing to tune
      if (f.full) continue;  // network operators keep their shape (hgf_set_tile_config sets it)
      const std::string key = tune_key(dev, f, op->precision);
      auto it = cache.find(key);
      const bool known = it != cache.end() && (!(flags & HGF_TUNE_FORCE) || fresh.count(key));
      if (known) {
        if (f.ga.blocks > 0 || it->second.c.nfast == 0) {
          try {
            retile(f, op->precision, it->second.c);
            f.tuned_us = it->second.us;
          } catch (const Error&) {
            // a cached shape that no longer fits (another build): keep the current one
          }
        }
        continue;
      }
      if (flags & HGF_TUNE_CACHED_ONLY) continue;
      std::vector<TileChoice> cands = tune_candidates(f, op->precision);
      if (cands.empty()) continue;
      // state backup: the timed steps advance y
      const size_t bytes = state_bytes(f);
      if (!f.ybak) f.ybak = dmalloc(bytes);
      hip_check(hipMemcpyAsync(f.ybak, f.y, bytes, hipMemcpyDeviceToDevice, st), "backup");
      const TileChoice start = current_choice(f);
      TuneEntry best;
      best.us = 1e300;
      try {
        // enough steps for ~3 ms of timed work per candidate (at least 4:
        // shorter runs left run-to-run noise above the 1 % tie margin)
        const double t0 = time_function_steps(f, op->precision, h, dflag.as<int>(), 1, st);
        const int steps = (int)std::max(4.0, std::min(100.0, 3000.0 / std::max(1e-3, 4.0 * t0)));
        std::vector<double> times;
        for (const TileChoice& c : cands) {
          retile(f, op->precision, c);
          times.push_back(time_function_steps(f, op->precision, h, dflag.as<int>(), steps, st));
        }
        best = pick_shape(cands, times);
        // then the walk order, on the chosen shape with the resident
        // workgroups per CU it had and with one more and one fewer (a blocked
        // walk keeps more neighbour tiles in L2 and moves the best occupancy)
        std::vector<TileChoice> wc{best.c};
        const int ns = f.ga.n - best.c.nfast;
        int occ_now = 0;
        {
          GridArgs g = f.ga;
          if (configure_tiles(g, op->precision, f.real, best.c)) occ_now = best.c.wgs_per_cu > 0 ? best.c.wgs_per_cu : g.occ_max;
        }
        for (int B : {2, 3}) {
          bool useful = false;
          for (int j = 0; j < ns; ++j) useful |= f.ga.ext[j] > B;
          if (!useful || ns < 2) continue;
          for (int w : {occ_now, occ_now + 1, occ_now - 1}) {
            if (w < 1) continue;
            TileChoice c = best.c;
            c.wblock = B;
            c.wgs_per_cu = w;
            GridArgs g = f.ga;
            if (configure_tiles(g, op->precision, f.real, c)) wc.push_back(c);
          }
        }
        if (wc.size() > 1) {
          std::vector<double> wt;
          for (const TileChoice& c : wc) {
            retile(f, op->precision, c);
            wt.push_back(time_function_steps(f, op->precision, h, dflag.as<int>(), steps, st));
          }
          best = pick_shape(wc, wt);
        }
        retile(f, op->precision, best.c);
      } catch (const Error&) {
        (void)hipStreamSynchronize(st);
        try {
          retile(f, op->precision, start);
        } catch (const Error&) {
        }
        (void)hipMemcpy(f.y, f.ybak, bytes, hipMemcpyDeviceToDevice);
        launch_shadow(op->precision, f.ga, f.y, f.yf, nullptr);
        (void)hipDeviceSynchronize();
        drop_plan(op);
        throw;
      }
      f.tuned_us = best.us;
      hip_check(hipMemcpyAsync(f.y, f.ybak, bytes, hipMemcpyDeviceToDevice, st), "restore");
      launch_shadow(op->precision, f.ga, f.y, f.yf, st);
      hip_check(hipStreamSynchronize(st), "synchronize");
      cache[key] = best;
      fresh.insert(key);
      measured = true;
    }
    drop_plan(op);
  }
  tune_groups(ops, n, h, dev, cache, fresh, flags, measured, dflag.as<int>(), st);
  if (measured) write_tune_cache(cache_path, cache);
}

}  // namespace hgf
