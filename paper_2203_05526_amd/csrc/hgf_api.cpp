// C-ABI entry points of the library: argument validation, the error state,
// device memory (hipMalloc or the caller's allocator hook) and the checks
// shared by the host modules.  The work behind the entry points lives in
// hgf_functions.cpp and hgf_network.cpp (step (i): operator -> functions),
// hgf_step.cpp (step (ii): RK4 stepping), hgf_readout.cpp (step (iii)),
// hgf_autotune.cpp, hgf_grad.cpp and hgf_separated_host.cpp.
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

// ------------------------------------------------------------------ errors

namespace {
thread_local std::string g_last_error;

struct Failure : std::exception {
  hgf_status code;
  std::string msg;
  Failure(hgf_status c, std::string m) : code(c), msg(std::move(m)) {}
};
}  // namespace

void set_error(hgf_status code, const std::string& msg) {
  (void)code;
  g_last_error = msg;
}

[[noreturn]] void fail(hgf_status code, const std::string& msg) { throw Failure(code, msg); }

void hip_check(hipError_t e, const char* what) {
  if (e != hipSuccess) {
    if (e == hipErrorOutOfMemory) fail(HGF_ENOMEM, std::string(what) + ": out of device memory");
    fail(HGF_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
  }
}

template <typename F>
static hgf_status guarded(F&& f) {
  try {
    g_last_error.clear();
    f();
    return HGF_OK;
  } catch (const Failure& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return HGF_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return HGF_EDEVICE;
  }
}

// ------------------------------------------------------------------ helpers

double sqrt_factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return std::sqrt(f);
}

double factorial(int n) {
  double f = 1.0;
  for (int i = 2; i <= n; ++i) f *= i;
  return f;
}

// ---- device memory: hipMalloc, or the caller's allocator hook
// Every block remembers where it came from: a block of a hook is returned to
// that hook, or dropped (left to the hook's owner) once the hook has been
// replaced, never passed to hipFree.
struct AllocHook {
  hgf_alloc_fn alloc = nullptr;
  hgf_free_fn free = nullptr;
  void* user = nullptr;
  uint64_t generation = 0;  // 0: hipMalloc
};
static std::mutex g_alloc_mu;
static AllocHook g_hook;
static uint64_t g_hook_generation = 0;
static std::unordered_map<void*, uint64_t> g_hooked;  // block -> generation of its hook

void* dmalloc(size_t bytes) {
  void* p = nullptr;
  if (bytes == 0) bytes = 16;
  AllocHook h;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    h = g_hook;
  }
  if (!h.alloc) {
    hip_check(hipMalloc(&p, bytes), "hipMalloc");
    return p;
  }
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  p = h.alloc(bytes, dev, h.user);
  if (!p) fail(HGF_ENOMEM, "allocator hook returned NULL");
  std::lock_guard<std::mutex> lk(g_alloc_mu);
  g_hooked[p] = h.generation;
  return p;
}

void dfree(void*& p) {
  if (!p) return;
  AllocHook h;
  bool hooked = false, current = false;
  {
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    auto it = g_hooked.find(p);
    if (it != g_hooked.end()) {
      hooked = true;
      current = g_hook.alloc && it->second == g_hook.generation;
      h = g_hook;
      g_hooked.erase(it);
    }
  }
  if (!hooked) {
    (void)hipFree(p);
  } else if (current) {
    int dev = 0;
    (void)hipGetDevice(&dev);
    h.free(p, dev, h.user);
  }
  p = nullptr;
}

int64_t check_steps(double t_total, double dt) {
  if (!(std::isfinite(t_total) && std::isfinite(dt)) || t_total < 0 || dt <= 0)
    fail(HGF_EINVAL, "t_total must be >= 0 and dt > 0, both finite");
  const double r = t_total / dt;
  const int64_t m = (int64_t)std::llround(r);
  if (std::fabs(r - (double)m) > 1e-9 * std::max(1.0, r))
    fail(HGF_EINVAL, "t_total must be an integer multiple of dt");
  return m;
}


// prod_j ext[j] with an overflow check against kMaxOperatorPoints.
int64_t checked_points(const int* ext, int n) {
  int64_t p = 1;
  for (int j = 0; j < n; ++j) {
    if (ext[j] <= 0) return 0;
    if (p > kMaxOperatorPoints / ext[j])
      fail(HGF_EINVAL, "a sector grid would exceed 2^32 points; reduce the modes or cutoffs");
    p *= ext[j];
  }
  return p;
}

// total += add, failing once the operator's points exceed the cap.
void add_points(int64_t& total, int64_t add) {
  if (add > kMaxOperatorPoints - total)
    fail(HGF_EINVAL, "the operator's sector grids would exceed 2^32 points in total");
  total += add;
}

void check_stability(const std::vector<Function>& fns, double dt, bool jumps_only) {
  // RK4's stability region holds the left half-disc of radius ~2.6; the
  // Gershgorin bound of the sector generator (of its jump terms alone for the
  // integrating-factor scheme, whose diagonal part is exact and has a
  // non-positive real part) must fit in it.
  for (const auto& f : fns) {
    double b = 0.0;
    if (f.full) {
      b = f.full_bound;
    } else if (jumps_only) {
      for (int j = 0; j < f.tab.n; ++j) {
        double mx = 0.0;
        for (int m = 0; m < f.tab.ext[j]; ++m) mx = std::max(mx, f.tab.alpha[j][m] + f.tab.beta[j][m]);
        b += mx;
      }
    } else {
      b = generator_bound(f.tab);
    }
    b *= dt;
    if (b > 2.5)
      fail(HGF_EUNSTABLE, "dt * spectral bound = " + std::to_string(b) +
                              " exceeds the RK4 stability limit 2.5; reduce dt");
  }
}

static System system_from_desc(const hgf_system_desc* d) {
  if (!d) fail(HGF_EINVAL, "system description is NULL");
  const int n = d->n_modes;
  if (n < 1 || n > kMaxModes) fail(HGF_EINVAL, "n_modes must be in 1..16");
  if (!d->cutoff || !d->detuning || !d->kerr || !d->cross_kerr || !d->gamma1 || !d->gamma_phi || !d->n_th)
    fail(HGF_EINVAL, "system description has a NULL array");
  System s;
  s.n = n;
  for (int j = 0; j < n; ++j) {
    if (d->cutoff[j] < 1 || d->cutoff[j] > kMaxCutoff) fail(HGF_EINVAL, "cutoff must be in 1..32");
    s.nc[j] = d->cutoff[j];
    s.det[j] = d->detuning[j];
    s.kerr[j] = d->kerr[j];
    s.g1[j] = d->gamma1[j];
    s.gphi[j] = d->gamma_phi[j];
    s.nth[j] = d->n_th[j];
    for (double v : {s.det[j], s.kerr[j], s.g1[j], s.gphi[j], s.nth[j]})
      if (!std::isfinite(v)) fail(HGF_EINVAL, "non-finite system parameter");
    if (s.g1[j] < 0 || s.gphi[j] < 0 || s.nth[j] < 0) fail(HGF_EINVAL, "rates and n_th must be >= 0");
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double a = d->cross_kerr[i * n + j], b = d->cross_kerr[j * n + i];
      if (!std::isfinite(a)) fail(HGF_EINVAL, "non-finite cross_kerr");
      if (i != j && a != b) fail(HGF_EINVAL, "cross_kerr must be symmetric");
      s.chi[i][j] = (i == j) ? 0.0 : a;
    }
  if (d->dissipator != HGF_DISS_LINDBLAD && d->dissipator != HGF_DISS_SECULAR) fail(HGF_EINVAL, "unknown dissipator");
  s.secular = d->dissipator == HGF_DISS_SECULAR ? 1 : 0;
  if (!s.secular && d->n_th_levels) fail(HGF_EINVAL, "n_th_levels applies to the secular dissipator only");
  size_t off = 0;
  for (int j = 0; j < n; ++j) {
    for (int t = 0; t + 1 < s.nc[j]; ++t) {
      const double v = d->n_th_levels ? d->n_th_levels[off + t] : s.nth[j];
      if (!std::isfinite(v) || v < 0) fail(HGF_EINVAL, "n_th_levels must be finite and >= 0");
      s.nlev[j][t] = v;
    }
    off += s.nc[j] - 1;
  }
  for (int j = 0; j < n; ++j) {
    s.drive_re[j] = d->drive ? d->drive[2 * j] : 0.0;
    s.drive_im[j] = d->drive ? d->drive[2 * j + 1] : 0.0;
    if (!std::isfinite(s.drive_re[j]) || !std::isfinite(s.drive_im[j])) fail(HGF_EINVAL, "non-finite drive");
    if (s.drive_re[j] != 0.0 || s.drive_im[j] != 0.0) s.full = 1;
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < n; ++j) {
      const double a = d->exchange ? d->exchange[i * n + j] : 0.0, b = d->exchange ? d->exchange[j * n + i] : 0.0;
      if (!std::isfinite(a)) fail(HGF_EINVAL, "non-finite exchange");
      if (i != j && a != b) fail(HGF_EINVAL, "exchange must be symmetric");
      s.exch[i][j] = (i == j) ? 0.0 : a;
      if (s.exch[i][j] != 0.0) s.full = 1;
    }
  if (s.full && n > kMaxFullModes) fail(HGF_EINVAL, "a driven or exchange-coupled system has at most 8 modes");
  return s;
}

}  // namespace hgf

using namespace hgf;

// ====================================================================== ABI

extern "C" {

const char* hgf_last_error(void) { return g_last_error.c_str(); }

const char* hgf_version(void) { return "hgf 0.1 (gfx950)"; }

hgf_status hgf_define_system(const hgf_system_desc* desc, hgf_system* out) {
  return guarded([&] {
    if (!out) fail(HGF_EINVAL, "out is NULL");
    System s = system_from_desc(desc);
    auto* h = new hgf_system_s;
    h->sys = s;
    *out = h;
  });
}

void hgf_destroy_system(hgf_system sys) { delete sys; }

int32_t hgf_num_params(hgf_system sys) { return sys ? num_params(sys->sys.n) : -1; }

hgf_status hgf_map_operator(hgf_system sys, const hgf_operator_desc* desc, hgf_operator* out) {
  return guarded([&] {
    if (!sys || !desc || !out) fail(HGF_EINVAL, "NULL argument");
    if (desc->precision != HGF_FP64 && desc->precision != HGF_MIXED) fail(HGF_EINVAL, "unknown precision");
    if (desc->layout != HGF_MERGED && desc->layout != HGF_SPLIT && desc->layout != HGF_SEPARATED &&
        desc->layout != HGF_SEPARATED_EXACT)
      fail(HGF_EINVAL, "unknown layout");
    if (desc->basis != HGF_BASIS_NUMBER && desc->basis != HGF_BASIS_NORMAL) fail(HGF_EINVAL, "unknown basis");
    if (!(desc->drop_tol >= 0)) fail(HGF_EINVAL, "drop_tol must be >= 0");
    hgf::precheck_operator_size(sys->sys, desc);
    auto* op = new hgf_operator_s;
    try {
      op->sys = sys->sys;
      op->precision = desc->precision;
      op->layout = desc->layout;
      hip_check(hipGetDevice(&op->device), "hipGetDevice");
      op->dflag = (int*)dmalloc(sizeof(int));
      if (op->layout == HGF_SEPARATED || op->layout == HGF_SEPARATED_EXACT)
        build_separated(op, desc);
      else
        build_functions(op, desc);
      hip_check(hipDeviceSynchronize(), "synchronize");
    } catch (...) {
      hgf_destroy_operator(op);
      throw;
    }
    *out = op;
  });
}

void hgf_destroy_operator(hgf_operator op) {
  if (!op) return;
  (void)hipSetDevice(op->device);
  drop_plan(op);
  free_separated(op);
  if (op->dcount) dfree(*(void**)&op->dcount);
  for (auto& f : op->fn) free_function(f);
  if (op->dflag) dfree(*(void**)&op->dflag);
  if (op->cap_stream) (void)hipStreamDestroy(op->cap_stream);
  delete op;
}

hgf_status hgf_set_allocator(hgf_alloc_fn alloc, hgf_free_fn free_fn, void* user) {
  return guarded([&] {
    if ((alloc == nullptr) != (free_fn == nullptr)) fail(HGF_EINVAL, "alloc and free must both be set or both NULL");
    std::lock_guard<std::mutex> lk(g_alloc_mu);
    g_hook.alloc = alloc;
    g_hook.free = free_fn;
    g_hook.user = user;
    g_hook.generation = alloc ? ++g_hook_generation : 0;
  });
}

hgf_status hgf_set_threshold(hgf_operator op, double threshold) {
  return guarded([&] {
    if (!op) fail(HGF_EINVAL, "operator is NULL");
    if (!std::isfinite(threshold) || threshold < 0.0) fail(HGF_EINVAL, "threshold must be finite and >= 0");
    bool ok = op->precision == HGF_FP64 && (op->sep != nullptr || !op->fn.empty());
    for (auto& f : op->fn) ok = ok && f.full && !f.real;  // complex128 grids
    if (!ok)
      fail(HGF_EUNSUPPORTED, "thresholded storage applies to FP64 network operators on the full grid and to the "
                             "separated layouts");
    hip_check(hipSetDevice(op->device), "hipSetDevice");
    // work still in flight on any stream may be adding to the counters
    hip_check(hipDeviceSynchronize(), "synchronize");
    if (!op->dcount) op->dcount = (unsigned long long*)dmalloc(4 * sizeof(unsigned long long));
    hip_check(hipMemset(op->dcount, 0, 4 * sizeof(unsigned long long)), "clear counters");
    op->threshold = threshold;
  });
}

hgf_status hgf_clear_error(hgf_operator op) {
  return guarded([&] {
    if (!op) fail(HGF_EINVAL, "operator is NULL");
    op->error_state = 0;
  });
}

hgf_status hgf_evolve(hgf_operator op, double t_total_us, double dt_us, int32_t scheme, void* hip_stream) {
  return guarded([&] {
    if (!op) fail(HGF_EINVAL, "operator is NULL");
    if (scheme != HGF_RK4 && scheme != HGF_LAWSON_RK4) fail(HGF_EUNSUPPORTED, "unknown time-stepping scheme");
    if (op->error_state) fail(HGF_ESTATE, "operator is in an error state after a non-finite result");
    const int64_t m = check_steps(t_total_us, dt_us);
    hip_check(hipSetDevice(op->device), "hipSetDevice");
    evolve_impl(op, m, dt_us, (hipStream_t)hip_stream, scheme);
  });
}

hgf_status hgf_evolve_batch(hgf_operator* ops, int32_t n, const double* t_total_us, const double* dt_us,
                            void* hip_stream) {
  return guarded([&] {
    if (n < 0 || (n > 0 && (!ops || !t_total_us || !dt_us))) fail(HGF_EINVAL, "bad batch arguments");
    std::vector<int64_t> steps(n);
    for (int i = 0; i < n; ++i) {
      if (!ops[i]) fail(HGF_EINVAL, "NULL operator in batch");
      if (ops[i]->error_state) fail(HGF_ESTATE, "operator in batch is in an error state");
      if (ops[i]->layout != HGF_MERGED) fail(HGF_EINVAL, "batched evolve needs the merged layout");
      if (ops[i]->threshold > 0.0)
        fail(HGF_EUNSUPPORTED, "an operator with a threshold is evolved with hgf_evolve, not in a batch");
      for (int k = 0; k < i; ++k)
        if (ops[k] == ops[i]) fail(HGF_EINVAL, "batch members must be distinct");
      steps[i] = check_steps(t_total_us[i], dt_us[i]);
      check_stability(ops[i]->fn, dt_us[i]);
    }
    for (int i = 0; i < n; ++i)
      if (ops[i]->device != ops[0]->device) fail(HGF_EINVAL, "batch members must live on one device");
    if (n > 0) {
      hip_check(hipSetDevice(ops[0]->device), "hipSetDevice");
      batch_impl(ops, n, steps, dt_us, (hipStream_t)hip_stream);
    }
  });
}

hgf_status hgf_reconstruct(hgf_operator op, int32_t levels, double* out, void* hip_stream) {
  return guarded([&] {
    if (!op || !out) fail(HGF_EINVAL, "NULL argument");
    hip_check(hipSetDevice(op->device), "hipSetDevice");
    reconstruct_impl(op, levels, out, (hipStream_t)hip_stream);
  });
}

hgf_status hgf_expectation(hgf_operator op, const hgf_state_desc* psi, double out_re_im[2], void* hip_stream) {
  return guarded([&] {
    if (!op || !out_re_im) fail(HGF_EINVAL, "NULL argument");
    hip_check(hipSetDevice(op->device), "hipSetDevice");
    const cd r = expectation_impl(op, psi, (hipStream_t)hip_stream);
    out_re_im[0] = r.real();
    out_re_im[1] = r.imag();
  });
}

hgf_status hgf_expectation_noalloc(hgf_operator op, const hgf_state_desc* psi, double out_re_im[2],
                                   void* hip_stream) {
  return guarded([&] {
    if (!op || !out_re_im) fail(HGF_EINVAL, "NULL argument");
    hip_check(hipSetDevice(op->device), "hipSetDevice");
    const cd r = expectation_impl(op, psi, (hipStream_t)hip_stream, scratch_address(), kScratchBytes);
    out_re_im[0] = r.real();
    out_re_im[1] = r.imag();
  });
}

hgf_status hgf_grad(hgf_system sys, const hgf_operator_desc* desc, const hgf_state_desc* psi, double t_total_us,
                    double dt_us, int32_t checkpoint_every, double value_out[2], double* grad_out,
                    void* hip_stream) {
  return guarded([&] {
    if (!sys || !desc || !psi || !value_out || !grad_out) fail(HGF_EINVAL, "NULL argument");
    if (desc->basis != HGF_BASIS_NUMBER && desc->basis != HGF_BASIS_NORMAL) fail(HGF_EINVAL, "unknown basis");
    hgf::precheck_operator_size(sys->sys, desc);
    grad_impl(sys->sys, desc, psi, t_total_us, dt_us, checkpoint_every, value_out, grad_out,
              (hipStream_t)hip_stream);
  });
}

hgf_status hgf_get_info(hgf_operator op, hgf_operator_info* info) {
  return guarded([&] {
    if (!op || !info) fail(HGF_EINVAL, "NULL argument");
    info->n_functions = op->sep ? separated_functions(op) : (int32_t)op->fn.size();
    info->precision = op->precision;
    info->layout = op->layout;
    info->n_modes = op->sys.n;
    int64_t pts = 0;
    for (auto& f : op->fn) pts += f.ga.points;
    info->total_points = op->sep ? separated_points(op) : pts;
    info->steps_done = op->steps_done;
    info->time_us = op->time_us;
    info->fp32_underflow = op->underflow;
    info->error_state = op->error_state;
    int nreal = 0;
    for (auto& f : op->fn) nreal += f.real ? 1 : 0;
    info->real_functions = nreal;
    int untiled = 0;
    if (op->layout == HGF_MERGED)
      for (auto& f : op->fn) untiled += ((f.full ? f.ga.fblocks == 0 : f.ga.blocks == 0) && !f.resident) ? 1 : 0;
    info->untiled_functions = untiled;
    info->reserved = 0;
    info->stored_peak = -1;
    info->stored_tiles_peak = -1;
    info->tile_points = op->sep ? separated_tile_points(op) : (op->fn.size() == 1 && op->fn[0].full)
                                                                   ? full_tile_points(op->fn[0])
                                                                   : 0;
    if (op->threshold > 0.0 && op->dcount) {
      unsigned long long c[4] = {};
      hip_check(hipSetDevice(op->device), "hipSetDevice");
      hip_check(hipMemcpy(c, op->dcount, sizeof(c), hipMemcpyDeviceToHost), "download");
      info->stored_peak = (int64_t)c[1];
      info->stored_tiles_peak = (int64_t)c[3];
    }
  });
}

hgf_status hgf_stream_ceiling(int32_t precision, int32_t real, int64_t points, int32_t reps, double us_out[4],
                              void* hip_stream) {
  return guarded([&] {
    if (!us_out) fail(HGF_EINVAL, "NULL argument");
    if (precision != HGF_FP64 && precision != HGF_MIXED) fail(HGF_EINVAL, "unknown precision");
    stream_ceiling(precision, real != 0, points, reps, us_out, (hipStream_t)hip_stream);
  });
}

hgf_status hgf_get_tile_config(hgf_operator op, int32_t idx, hgf_tile_config* out) {
  return guarded([&] {
    if (!op || !out) fail(HGF_EINVAL, "NULL argument");
    if (idx < 0 || idx >= (int32_t)op->fn.size()) fail(HGF_EINVAL, "function index out of range");
    const Function& f = op->fn[idx];
    if (f.full) {  // network operator: tiles of its last two modes, or untiled
      const bool ft = f.ga.fblocks > 0;
      *out = hgf_tile_config{};
      out->nfast = ft ? 4 : 0;
      out->threads = ft ? f.ga.fthreads : f.resident ? f.res_threads : 0;
      out->resident = f.resident ? 1 : 0;
      out->wgs_per_cu = ft ? f.ga.fwgs : 0;
      out->walk_block = ft ? f.ga.fwblock : 0;
      out->blocks = ft ? f.ga.fblocks : 0;
      out->tile_points = ft ? f.ga.ftile : 1;
      return;
    }
    const bool tiled = f.ga.blocks > 0;
    out->nfast = tiled ? f.ga.nfast : 0;
    out->threads = f.resident ? f.res_threads : tiled ? f.ga.threads : 0;
    out->xblock = tiled ? f.ga.xblock : 0;
    out->pipe = tiled ? f.ga.pipe : 0;
    out->wgs_per_cu = tiled ? f.ga.occ_cap : 0;
    out->resident = f.resident ? 1 : 0;
    out->walk_block = tiled ? f.ga.wblock : 0;
    out->blocks = tiled ? f.ga.blocks : 0;
    out->tile_points = tiled ? (int32_t)f.ga.tile_points : 1;
    out->stage_us = f.tuned_us;
  });
}

hgf_status hgf_set_tile_config(hgf_operator op, int32_t idx, const hgf_tile_config* cfg) {
  return guarded([&] {
    if (!op || !cfg) fail(HGF_EINVAL, "NULL argument");
    if (idx < 0 || idx >= (int32_t)op->fn.size()) fail(HGF_EINVAL, "function index out of range");
    if (cfg->nfast < 0 || cfg->threads < 0 || cfg->xblock < 0 || cfg->wgs_per_cu < 0 || cfg->walk_block < 0 ||
        (cfg->pipe != 0 && cfg->pipe != 1) || (cfg->resident != 0 && cfg->resident != 1))
      fail(HGF_EINVAL, "negative tile parameter, or pipe or resident not 0/1");
    TileChoice c;
    c.nfast = cfg->nfast;
    c.threads = cfg->threads;
    c.xblock = cfg->xblock;
    c.pipe = cfg->pipe;
    c.wgs_per_cu = cfg->wgs_per_cu;
    c.wblock = cfg->walk_block;
    hip_check(hipSetDevice(op->device), "hipSetDevice");
    hip_check(hipDeviceSynchronize(), "synchronize");  // no launch may still read the old records
    Function& f = op->fn[idx];
    if (f.full) {
      if (cfg->xblock != 0 || cfg->pipe != 0 || (cfg->nfast != 0 && cfg->nfast != 4) ||
          (cfg->resident && cfg->nfast != 0))
        fail(HGF_EINVAL, "a network operator takes nfast 0 (untiled, or with resident 1 the resident form) or 4 "
                         "(tiles of its last two modes), without xblock or pipe");
      if (cfg->resident) {
        Function probe;
        probe.full = true;
        probe.ga = f.ga;
        if (!full_resident_eligible(probe, op->precision))
          fail(HGF_EINVAL, "the resident form of a network operator needs its grid twice within 64 KB of LDS "
                           "and at most three modes");
      }
      if (cfg->nfast == 0)
        drop_full_tiles(f);
      else if (!configure_full_tiles(f, f.fhost.at(0), op->precision, c))
        fail(HGF_EINVAL, "tile configuration not feasible for this network grid");
      f.resident = cfg->resident && full_resident_eligible(f, op->precision);
      drop_plan(op);
      return;
    }
    if (cfg->resident) {  // check on a copy first: the function is unchanged on error
      // `threads` is the resident workgroup's size; the stage-kernel shape
      // kept beside it (for other calls) takes its default
      c.threads = 0;
      Function probe;
      probe.split = f.split;
      probe.precision_fp64 = f.precision_fp64;
      probe.ga = f.ga;
      if (c.nfast == 0 || !configure_tiles(probe.ga, op->precision, f.real, c) ||
          !resident_eligible(probe, cfg->threads))
        fail(HGF_EINVAL, "the resident form needs a grid of at most 4 axes and 4096 points (FP64: 2048 real, "
                         "2560 complex) whose two padded copies fit in 160 KB of LDS (and threads, if set, a "
                         "multiple of 64 covering it in at most 4 lane rounds, 5 on complex FP64 grids)");
    }
    retile(f, op->precision, c);
    f.resident = cfg->resident && resident_eligible(f, cfg->threads);
    drop_plan(op);
  });
}

hgf_status hgf_autotune(hgf_operator* ops, int32_t n, double dt_us, const char* cache_path, int32_t flags,
                        void* hip_stream) {
  return guarded([&] {
    if (!ops || n < 0) fail(HGF_EINVAL, "NULL ops or negative count");
    if (!(dt_us > 0.0) || !std::isfinite(dt_us)) fail(HGF_EINVAL, "dt must be positive and finite");
    if (flags & ~(HGF_TUNE_CACHED_ONLY | HGF_TUNE_FORCE)) fail(HGF_EINVAL, "unknown autotune flag");
    for (int i = 0; i < n; ++i) {
      if (!ops[i]) fail(HGF_EINVAL, "NULL operator");
      if (ops[i]->device != ops[0]->device) fail(HGF_EINVAL, "operators on different devices");
    }
    if (n == 0) return;
    hip_check(hipSetDevice(ops[0]->device), "hipSetDevice");
    hipStream_t st = (hipStream_t)hip_stream;
    hip_check(hipStreamSynchronize(st), "synchronize");
    autotune_impl(ops, n, dt_us, cache_path, flags, st);
  });
}

hgf_status hgf_get_function(hgf_operator op, int32_t idx, int32_t* sector_d, int32_t* extents, double* grid,
                            int64_t n_points, double* split_out, void* hip_stream) {
  return guarded([&] {
    if (!op) fail(HGF_EINVAL, "operator is NULL");
    if (idx < 0 || idx >= (int32_t)op->fn.size()) fail(HGF_EINVAL, "function index out of range");
    Function& f = op->fn[idx];
    if (f.full) fail(HGF_EUNSUPPORTED, "a network operator is one full (k, l) grid: read it with hgf_reconstruct");
    const int n = op->sys.n;
    if (sector_d)
      for (int j = 0; j < n; ++j) sector_d[j] = f.tab.d[j];
    if (extents)
      for (int j = 0; j < n; ++j) extents[j] = f.tab.ext[j];
    if (grid) {
      if (n_points < f.ga.points) fail(HGF_EINVAL, "grid buffer too small");
      hip_check(hipSetDevice(op->device), "hipSetDevice");
      if (f.real) {
        std::vector<double> r(f.ga.points);
        hip_check(hipMemcpyAsync(r.data(), f.y, f.ga.points * sizeof(double), hipMemcpyDeviceToHost,
                                 (hipStream_t)hip_stream),
                  "download");
        hip_check(hipStreamSynchronize((hipStream_t)hip_stream), "synchronize");
        for (int64_t i = 0; i < f.ga.points; ++i) {
          grid[2 * i] = r[i];
          grid[2 * i + 1] = 0.0;
        }
      } else {
        hip_check(hipMemcpyAsync(grid, f.y, f.ga.points * sizeof(double2), hipMemcpyDeviceToHost,
                                 (hipStream_t)hip_stream),
                  "download");
        hip_check(hipStreamSynchronize((hipStream_t)hip_stream), "synchronize");
      }
    }
    if (split_out) {
      std::vector<double> o(4 * n + 6, 0.0);
      for (int j = 0; j < n; ++j) {
        o[j] = f.split ? f.p[j] : 0;
        o[n + j] = f.split ? f.q[j] : 0;
      }
      const cd g0 = f.split ? f.g0 : cd(1.0), cx = f.split ? f.cx : cd(0.0), cy = f.split ? f.cy : cd(0.0);
      o[2 * n] = g0.real();
      o[2 * n + 1] = g0.imag();
      o[2 * n + 2] = cx.real();
      o[2 * n + 3] = cx.imag();
      o[2 * n + 4] = cy.real();
      o[2 * n + 5] = cy.imag();
      std::memcpy(split_out, o.data(), o.size() * sizeof(double));
    }
  });
}

}  // extern "C"
