// C-ABI entry points and the host runtime around the HIP kernels: system
// validation, the operator -> function map (step (i) of the method), the RK4
// step loop with HIP-graph replay (step (ii)), the expectation value
// (step (iii)) and the discrete-adjoint gradient.
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

static double factorial(int n) {
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

// Largest number of grid points in one operator (summed over its functions).
// Every kernel indexes a grid with 64-bit element counts; the cap keeps the
// point counts, their byte sizes and the sums over sectors far from int64
// overflow, and is beyond what HBM holds anyway (2^32 points of the smallest
// element set, a real mixed grid with its stage grids, take over 100 GB).
constexpr int64_t kMaxOperatorPoints = (int64_t)1 << 32;

// prod_j ext[j] with an overflow check against kMaxOperatorPoints.
static int64_t checked_points(const int* ext, int n) {
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
static void add_points(int64_t& total, int64_t add) {
  if (add > kMaxOperatorPoints - total)
    fail(HGF_EINVAL, "the operator's sector grids would exceed 2^32 points in total");
  total += add;
}

static void check_stability(const std::vector<Function>& fns, double dt, bool jumps_only = false) {
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

// ------------------------------------------------------------------ functions

// HGF_STAGE_KERNEL=generic selects the untiled stage kernel for every grid.
static bool stage_kernel_generic() {
  const char* env = std::getenv("HGF_STAGE_KERNEL");
  return env && std::string(env) == "generic";
}

// Launch shape of the tiled stage kernel.  Fields at -1 (nfast, xblock, pipe)
// or 0 (threads) take the default rule below.
struct TileChoice {
  int nfast = -1;
  int threads = 0;
  int xblock = -1;
  int pipe = -1;
  int wgs_per_cu = 0;  // resident workgroups per CU in the persistent grid (0: as many as fit)
  int wblock = -1;     // tile walk order (-1, 0: row-major; B >= 2: blocks of B per slow axis)
};

// Pipelined neighbour loads keep the register budget only up to this many
// slow axes (more spill to scratch).
constexpr int kPipeMaxSlow = 9;

// Configure the tiled stage kernel for grid g.  Default rule: the largest
// number nfast <= 4 of trailing axes whose padded tile and tables fit in 64 KB
// of LDS; 256 lanes when they cover the tile in at most kTileRounds rounds (the
// fastest shape measured on the 6^10 grid), else the smallest multiple of 64
// that does; contiguous XCD order; no pipelining.  Returns false (and sets
// g.blocks = 0, the generic kernel) when the request cannot be met.
static bool configure_tiles(GridArgs& g, int precision, bool real, const TileChoice& c) {
  g.blocks = 0;
  g.nfast = 0;
  g.real = 0;
  if (c.nfast == 0) return true;
  const int rs = precision == HGF_FP64 ? 8 : 4, ts = real ? rs : 2 * rs;
  int best = 0;
  int fmax = std::min(4, g.n);
  if (c.nfast < 0) {
    const char* env = std::getenv("HGF_MAX_NFAST");  // cap on the default rule
    if (env && std::atoi(env) >= 1) fmax = std::min(fmax, std::atoi(env));
  }
  for (int F = fmax; F >= 1; --F) {
    if (c.nfast > 0 && F != c.nfast) continue;
    if (g.n - F > tiled_max_slow_axes()) continue;
    // padded LDS tile: (e_0 + 2) x prod_{q>=1} (e_q + 1), see k_rk4_tiled
    int64_t T = 1, padded = 1, esum = 0;
    int emax = 0;
    for (int q = 0; q < F; ++q) {
      const int e = g.ext[g.n - F + q];
      T *= e;
      padded *= (q == 0) ? e + 2 : e + 1;
      esum += e;
      emax = std::max(emax, e);
    }
    const int cbits = tile_coord_bits(F);
    if (emax > (1 << cbits) || padded >= 65536) continue;
    // one point per lane; a tile takes at most kTileRounds rounds of lanes
    // (the kernel's prefetch registers)
    if (T > tiled_max_lane_groups()) continue;
    int threads = c.threads;
    if (threads == 0) {
      threads = T >= 256 ? 256 : (int)((T + 63) / 64 * 64);
      if ((T + threads - 1) / threads > kTileRounds)
        threads = (int)std::min<int64_t>(512, ((T + kTileRounds - 1) / kTileRounds + 63) / 64 * 64);
    }
    if (threads < 64 || threads > 512 || threads % 64 != 0) continue;
    if ((T + threads - 1) / threads > kTileRounds) continue;
    const int64_t bytes =
        tiled_lds((int)padded, (int)T, (int)esum, ts, rs).bytes;
    if (bytes > 65536) continue;
    best = F;
    g.nfast = F;
    g.threads = threads;
    g.cbits = cbits;
    g.tile_points = T;
    g.lds_elems = (int)padded;
    g.lds_bytes = (int)bytes;
    int64_t pst = 1;
    for (int q = F - 1; q >= 0; --q) {
      g.pstride[q] = (int)pst;
      pst *= g.ext[g.n - F + q] + 1;
    }
    break;
  }
  if (best == 0) return false;
  g.ntiles = g.points / g.tile_points;
  // 32-bit byte offsets in the tiled kernel (complex128 y is the widest operand)
  if (g.ntiles >= (int64_t)1 << 31 || g.points * 16 > (int64_t)0xffffffffLL) {
    g.blocks = 0;
    g.nfast = 0;
    return false;
  }
  g.xblock = std::max(0, c.xblock);
  g.wblock = c.wblock >= 2 ? c.wblock : 0;
  g.walk = nullptr;
  g.pipe = c.pipe > 0 ? 1 : 0;
  if (g.pipe && g.n - g.nfast > kPipeMaxSlow) {
    g.blocks = 0;
    g.nfast = 0;
    return false;
  }
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  g.real = real ? 1 : 0;
  const int occ =
      tiled_max_blocks_per_cu(g.nfast, g.n - g.nfast, g.threads, precision, g.lds_bytes, real, g.pipe ? 2 : 1);
  if (occ <= 0) {
    g.blocks = 0;
    g.nfast = 0;
    g.real = 0;
    return false;
  }
  if (c.wgs_per_cu > occ) {
    g.blocks = 0;
    g.nfast = 0;
    g.real = 0;
    return false;
  }
  g.occ_cap = c.wgs_per_cu > 0 ? c.wgs_per_cu : 0;
  g.occ_max = occ;
  const int64_t want = (int64_t)cus * (c.wgs_per_cu > 0 ? c.wgs_per_cu : occ);
  const int64_t cap = 8 * ((g.ntiles + 7) / 8);
  g.blocks = (int)std::max<int64_t>(8, std::min(want, cap));
  return true;
}

// Per-tile records of the slow-axis terms for k_rk4_tiled (layout of
// TileRec<NS, R>): lam_slow (FP64 re, im), 2*NS int32 element offsets, 2*NS R
// coefficients, with the coefficient array aligned to sizeof(R).
template <typename R>
static std::vector<char> tile_records(const GridArgs& g, const SectorTables& t) {
  const int ns = g.n - g.nfast, nd = 2 * std::max(ns, 1);
  size_t bytes = 2 * sizeof(double) + nd * sizeof(int32_t);
  bytes = (bytes + sizeof(R) - 1) / sizeof(R) * sizeof(R);
  const size_t coef_at = bytes;
  bytes += nd * sizeof(R);
  std::vector<char> out(bytes * g.ntiles, 0);
  for (int64_t tt = 0; tt < g.ntiles; ++tt) {
    char* r = out.data() + bytes * tt;
    int64_t rem = tt;
    cd lam = t.lam0;
    std::vector<int32_t> off(nd, 0);
    std::vector<R> coef(nd, 0);
    for (int j = ns - 1; j >= 0; --j) {
      const int sj = (int)(rem % t.ext[j]);
      rem /= t.ext[j];
      lam += t.lam[j][sj];
      if (sj >= 1) {
        off[2 * j] = -(int32_t)g.stride[j];
        coef[2 * j] = (R)t.alpha[j][sj];
      }
      if (sj + 1 < t.ext[j]) {
        off[2 * j + 1] = (int32_t)g.stride[j];
        coef[2 * j + 1] = (R)t.beta[j][sj];
      }
    }
    const double lr = lam.real(), li = lam.imag();
    std::memcpy(r, &lr, sizeof(double));
    std::memcpy(r + sizeof(double), &li, sizeof(double));
    std::memcpy(r + 2 * sizeof(double), off.data(), nd * sizeof(int32_t));
    std::memcpy(r + coef_at, coef.data(), nd * sizeof(R));
  }
  return out;
}

// Walk order of the tiles for g.wblock = B >= 2: the slow-axis coordinate
// space is cut into blocks of B along every slow axis (smaller at the ends);
// blocks are visited in row-major order, and the tiles of a block in row-major
// order.  A row-major walk visits the neighbours along the slowest axes
// prod(other slow extents) tiles apart, further than L2 holds; inside a block
// every neighbour is at most B^(NS-1) tiles away and only the tiles on a
// block face have neighbours outside it.
static std::vector<uint32_t> walk_order(const GridArgs& g) {
  const int ns = g.n - g.nfast, B = g.wblock;
  std::vector<uint32_t> order;
  int nb[kMaxModes], ob[kMaxModes], ib[kMaxModes], be[kMaxModes];
  int64_t nblocks = 1, nunits = 1;
  for (int j = 0; j < ns; ++j) {
    nb[j] = (g.ext[j] + B - 1) / B;
    nblocks *= nb[j];
    nunits *= g.ext[j];
  }
  order.reserve((size_t)nunits);
  for (int64_t o = 0; o < nblocks; ++o) {
    int64_t rem = o, inner = 1;
    for (int j = ns - 1; j >= 0; --j) {
      ob[j] = (int)(rem % nb[j]);
      rem /= nb[j];
      be[j] = std::min(B, g.ext[j] - ob[j] * B);
      inner *= be[j];
    }
    for (int64_t i = 0; i < inner; ++i) {
      int64_t r = i;
      for (int j = ns - 1; j >= 0; --j) {
        ib[j] = (int)(r % be[j]);
        r /= be[j];
      }
      int64_t t = 0;
      for (int j = 0; j < ns; ++j) t = t * g.ext[j] + ob[j] * B + ib[j];
      order.push_back((uint32_t)t);
    }
  }
  return order;
}

// Device copy of the tile records of grid g, followed by its walk order when
// g.wblock >= 2; sets g.tiles and g.walk (the caller owns the buffer).
static void* upload_tile_records(GridArgs& g, const SectorTables& t, int precision) {
  std::vector<char> rec = precision == HGF_FP64 ? tile_records<double>(g, t) : tile_records<float>(g, t);
  const size_t rec_bytes = (rec.size() + 255) / 256 * 256;
  std::vector<uint32_t> order;
  if (g.wblock >= 2 && g.n - g.nfast >= 1) order = walk_order(g);
  const size_t bytes = rec_bytes + order.size() * sizeof(uint32_t);
  rec.resize(bytes, 0);
  if (!order.empty()) std::memcpy(rec.data() + rec_bytes, order.data(), order.size() * sizeof(uint32_t));
  void* d = dmalloc(bytes);
  hipError_t e = hipMemcpy(d, rec.data(), bytes, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    dfree(d);
    hip_check(e, "upload tile records");
  }
  g.tiles = d;
  g.walk = order.empty() ? nullptr : (const uint32_t*)((const char*)d + rec_bytes);
  return d;
}

static void build_tile_records(Function& f, int precision) { f.ttab = upload_tile_records(f.ga, f.tab, precision); }

// A function runs on the resident kernel when its tiled configuration is a
// single tile holding every axis (then one workgroup does a stage's work in any
// case) and the tile fits the resident kernel's lane rounds.  `threads` > 0
// asks for that workgroup size (a multiple of 64 that covers the grid in the
// kernel's lane rounds), else the fewest rounds with lanes spread evenly.
static bool resident_eligible(Function& f, int threads = 0) {
  const GridArgs& g = f.ga;
  if (f.split || g.blocks == 0 || g.nfast != g.n || g.ntiles != 1) return false;
  const int max_threads = f.precision_fp64 ? 512 : 1024;  // the kernel's workgroup limit
  if (g.tile_points > (int64_t)resident_max_points() * max_threads / 1024) return false;
  // two padded copies of the grid and the down-jump tables in LDS
  const int rs = f.precision_fp64 ? 8 : 4, es = (f.ga.real ? 1 : 2) * rs;
  int esum = 0;
  for (int j = 0; j < g.n; ++j) esum += g.ext[j];
  if (g.n > 4) return false;
  for (int j = 0; j < g.n; ++j)
    if (g.ext[j] > 32) return false;  // 5-bit coordinates
  const int64_t lds = 2 * (int64_t)g.lds_elems * es + (int64_t)esum * rs;
  if (lds > 65536) return false;
  f.res_lds_bytes = (int)lds;
  if (threads > 0) {
    if (threads % 64 != 0 || threads > max_threads ||
        (g.tile_points + threads - 1) / threads * (int64_t)1024 > (int64_t)resident_max_points())
      return false;
    f.res_threads = threads;
    return true;
  }
  // lanes: enough for the fewest rounds, spread evenly over them
  const int64_t rounds = (g.tile_points + max_threads - 1) / max_threads;
  const int64_t per = (g.tile_points + rounds - 1) / rounds;
  f.res_threads = (int)std::min<int64_t>(max_threads, std::max<int64_t>(64, (per + 63) / 64 * 64));
  return true;
}

static void fill_grid_args(Function& f, int precision, bool want_real) {
  f.precision_fp64 = precision == HGF_FP64;
  GridArgs& g = f.ga;
  std::memset(&g, 0, sizeof(g));
  const SectorTables& t = f.tab;
  g.n = t.n;
  g.nfast = 0;
  checked_points(t.ext, t.n);
  int64_t s = 1;
  for (int j = t.n - 1; j >= 0; --j) {
    g.ext[j] = t.ext[j];
    g.stride[j] = s;
    s *= t.ext[j];
  }
  g.points = s;
  g.tile_points = 1;
  g.ntiles = s;
  int off = 0;
  for (int j = 0; j < t.n; ++j) {
    g.off[j] = off;
    off += t.ext[j];
  }
  g.lam0_re = t.lam0.real();
  g.lam0_im = t.lam0.imag();
  // Phase slopes: within a sector Im lam_j(m) = m * slope_j (the stage
  // kernels on complex FP32 grids form the phase from the coordinates in
  // FP64).  Every generator this library builds has this form; a table that
  // did not would run the generic kernel, which sums the tables in FP64.
  bool linear = true;
  for (int j = 0; j < t.n && !f.full; ++j) {
    const double slope = t.ext[j] > 1 ? t.lam[j][1].imag() : 0.0;
    g.phase_slope[j] = slope;
    for (int m = 0; m < t.ext[j]; ++m)
      if (std::fabs(t.lam[j][m].imag() - m * slope) > 1e-12 * std::max(1.0, std::fabs(m * slope))) linear = false;
  }
  g.phase_linear = linear ? 1 : 0;
  if (!stage_kernel_generic() && !f.full && (linear || precision == HGF_FP64))
    configure_tiles(g, precision, want_real, TileChoice{});
  f.real = g.real != 0;
  // device tables, one block: lam (double2), beta, alpha (double), beta_f,
  // alpha_f (float), each concatenated over the axes (the stencils sum the
  // diagonal rate lam in FP64 in every precision)
  const int tot = off;
  std::vector<double> lam(2 * tot), beta(tot), alpha(tot);
  std::vector<float> betaf(tot), alphaf(tot);
  for (int j = 0; j < t.n; ++j)
    for (int m = 0; m < t.ext[j]; ++m) {
      const int o = g.off[j] + m;
      lam[2 * o] = t.lam[j][m].real();
      lam[2 * o + 1] = t.lam[j][m].imag();
      beta[o] = t.beta[j][m];
      alpha[o] = t.alpha[j][m];
      betaf[o] = (float)beta[o];
      alphaf[o] = (float)alpha[o];
    }
  const size_t b_lam = sizeof(double) * 2 * tot, b_d = sizeof(double) * tot, b_f = sizeof(float) * tot;
  const size_t o_beta = b_lam, o_alpha = o_beta + b_d, o_betaf = o_alpha + b_d, o_alphaf = o_betaf + b_f,
               total = o_alphaf + b_f + 64;
  f.dtab = dmalloc(total);
  char* base = (char*)f.dtab;
  hip_check(hipMemcpy(base, lam.data(), b_lam, hipMemcpyHostToDevice), "upload tables");
  hip_check(hipMemcpy(base + o_beta, beta.data(), b_d, hipMemcpyHostToDevice), "upload tables");
  hip_check(hipMemcpy(base + o_alpha, alpha.data(), b_d, hipMemcpyHostToDevice), "upload tables");
  hip_check(hipMemcpy(base + o_betaf, betaf.data(), b_f, hipMemcpyHostToDevice), "upload tables");
  hip_check(hipMemcpy(base + o_alphaf, alphaf.data(), b_f, hipMemcpyHostToDevice), "upload tables");
  g.lam = (const double2*)base;
  g.beta = (const double*)(base + o_beta);
  g.alpha = (const double*)(base + o_alpha);
  g.beta_f = (const float*)(base + o_betaf);
  g.alpha_f = (const float*)(base + o_alphaf);
  g.tiles = nullptr;
  g.full = (const FullTables*)f.ftab;
  if (g.blocks > 0) build_tile_records(f, precision);
  f.resident = resident_eligible(f);
  const char* env = std::getenv("HGF_RESIDENT");
  if (env && std::string(env) == "0") f.resident = false;
}

static size_t state_bytes(const Function& f) { return f.ga.points * (f.real ? sizeof(double) : sizeof(double2)); }

static void alloc_function_buffers(Function& f, int precision) {
  const int64_t P = f.ga.points;
  const size_t rs = precision == HGF_FP64 ? sizeof(double) : sizeof(float);
  const size_t cs = f.real ? rs : 2 * rs;
  f.y = dmalloc(state_bytes(f));
  f.s1 = dmalloc(P * cs);
  f.s2 = dmalloc(P * cs);
  f.s3 = dmalloc(P * cs);
  if (f.split) f.s4 = dmalloc(P * sizeof(double2));
  if (precision == HGF_MIXED) f.yf = dmalloc(P * (f.real ? sizeof(float) : sizeof(float2)));
}

static void free_function(Function& f) {
  dfree(f.y);
  dfree(f.s1);
  dfree(f.s2);
  dfree(f.s3);
  dfree(f.s4);
  dfree(f.ybak);
  dfree(f.yf);
  dfree(f.dtab);
  dfree(f.ttab);
  dfree(f.ehtab);
  dfree(f.ftab);
}

static int64_t flat_index(const SectorTables& t, const int* m) {
  int64_t idx = 0;
  for (int j = 0; j < t.n; ++j) idx = idx * t.ext[j] + m[j];
  return idx;
}

// Per-mode g-matrix from the per-mode input matrix (Eqs. (6)-(8), r = 1).
static std::vector<cd> mode_g(const double* vals, int nc, int basis) {
  std::vector<cd> in(nc * nc), g(nc * nc);
  for (int i = 0; i < nc * nc; ++i) in[i] = cd(vals[2 * i], vals[2 * i + 1]);
  for (int k = 0; k < nc; ++k)
    for (int l = 0; l < nc; ++l) {
      if (basis == HGF_BASIS_NUMBER) {
        g[k * nc + l] = in[k * nc + l] / (sqrt_factorial(k) * sqrt_factorial(l));
      } else {  // Eq. (6): g_{k,l} = sum_j f_{k-j,l-j} / j!
        cd s = 0.0;
        for (int j = 0; j <= std::min(k, l); ++j) s += in[(k - j) * nc + (l - j)] / factorial(j);
        g[k * nc + l] = s;
      }
    }
  return g;
}

// Largest total dimension of an HGF_OP_DENSE operator.
constexpr int64_t kMaxDenseDim = 4096;

// All nonzero g_{k,l}(0) of the operator, as (k, l, value).
void collect_coeffs(const System& s, const hgf_operator_desc* d, std::map<std::vector<int>, std::vector<cd>>& merged,
                    std::vector<Coeff>& split, bool want_split) {
  const int n = s.n;
  if (d->kind == HGF_OP_PRODUCT) {
    if (!d->values) fail(HGF_EINVAL, "operator values is NULL");
    std::vector<std::vector<cd>> gm(n);
    std::vector<std::vector<int>> diags(n);
    size_t off = 0;
    for (int j = 0; j < n; ++j) {
      const int nc = s.nc[j];
      for (int i = 0; i < 2 * nc * nc; ++i)
        if (!std::isfinite(d->values[off + i])) fail(HGF_EINVAL, "non-finite operator entry");
      gm[j] = mode_g(d->values + off, nc, d->basis);
      off += 2 * (size_t)nc * nc;
      for (int dj = -nc + 1; dj < nc; ++dj) {
        bool nz = false;
        for (int k = 0; k < nc; ++k) {
          const int l = k + dj;
          if (l >= 0 && l < nc && gm[j][k * nc + l] != 0.0) nz = true;
        }
        if (nz) diags[j].push_back(dj);
      }
      if (diags[j].empty()) return;  // zero operator
    }
    // the sum of the sector sizes factorises over the modes: check it (and
    // so every sector) before enumerating the sectors
    {
      int tot[kMaxModes];
      for (int j = 0; j < n; ++j) {
        int64_t sj = 0;
        for (int dj : diags[j]) sj += s.nc[j] - std::abs(dj);
        tot[j] = (int)sj;
      }
      checked_points(tot, n);
    }
    // enumerate sectors as the product of per-mode diagonals
    std::vector<int> idx(n, 0);
    while (true) {
      std::vector<int> dv(n);
      for (int j = 0; j < n; ++j) dv[j] = diags[j][idx[j]];
      SectorTables t;
      t.n = n;
      int u[kMaxModes], v[kMaxModes], e[kMaxModes];
      for (int j = 0; j < n; ++j) {
        u[j] = dv[j] < 0 ? -dv[j] : 0;
        v[j] = dv[j] > 0 ? dv[j] : 0;
        e[j] = s.nc[j] - std::abs(dv[j]);
      }
      const int64_t pts = checked_points(e, n);
      if (!want_split) {
        std::vector<cd> grid(pts);
        std::vector<int> m(n, 0);
        for (int64_t f = 0; f < pts; ++f) {
          cd val = 1.0;
          for (int j = 0; j < n; ++j) val *= gm[j][(m[j] + u[j]) * s.nc[j] + (m[j] + v[j])];
          grid[f] = val;
          for (int j = n - 1; j >= 0; --j) {
            if (++m[j] < e[j]) break;
            m[j] = 0;
          }
        }
        merged[dv] = std::move(grid);
      } else {
        std::vector<int> m(n, 0);
        for (int64_t f = 0; f < pts; ++f) {
          cd val = 1.0;
          for (int j = 0; j < n; ++j) val *= gm[j][(m[j] + u[j]) * s.nc[j] + (m[j] + v[j])];
          if (val != 0.0) {
            Coeff c;
            c.k.resize(n);
            c.l.resize(n);
            for (int j = 0; j < n; ++j) {
              c.k[j] = m[j] + u[j];
              c.l[j] = m[j] + v[j];
            }
            c.v = val;
            split.push_back(std::move(c));
          }
          for (int j = n - 1; j >= 0; --j) {
            if (++m[j] < e[j]) break;
            m[j] = 0;
          }
        }
      }
      int j = n - 1;
      while (j >= 0 && ++idx[j] == (int)diags[j].size()) idx[j--] = 0;
      if (j < 0) break;
    }
    return;
  }
  if (d->kind == HGF_OP_DENSE) {
    // a dense matrix over the whole truncated space: its nonzero entries as a
    // sparse operator
    if (!d->values) fail(HGF_EINVAL, "operator values is NULL");
    int64_t dim = 1;
    for (int j = 0; j < n; ++j) {
      dim *= s.nc[j];
      if (dim > kMaxDenseDim) fail(HGF_EINVAL, "dense operator larger than 4096 x 4096; use HGF_OP_SPARSE");
    }
    std::vector<int32_t> idx;
    std::vector<double> vals;
    for (int64_t r = 0; r < dim; ++r)
      for (int64_t c = 0; c < dim; ++c) {
        const double re = d->values[2 * (r * dim + c)], im = d->values[2 * (r * dim + c) + 1];
        if (re == 0.0 && im == 0.0) continue;
        int64_t kr = r, kc = c;
        std::vector<int32_t> k(n), l(n);
        for (int j = n - 1; j >= 0; --j) {
          k[j] = (int32_t)(kr % s.nc[j]);
          kr /= s.nc[j];
          l[j] = (int32_t)(kc % s.nc[j]);
          kc /= s.nc[j];
        }
        idx.insert(idx.end(), k.begin(), k.end());
        idx.insert(idx.end(), l.begin(), l.end());
        vals.push_back(re);
        vals.push_back(im);
      }
    hgf_operator_desc sp = *d;
    sp.kind = HGF_OP_SPARSE;
    sp.values = vals.data();
    sp.indices = idx.data();
    sp.n_terms = (int64_t)(vals.size() / 2);
    collect_coeffs(s, &sp, merged, split, want_split);
    return;
  }
  if (d->kind != HGF_OP_SPARSE) fail(HGF_EINVAL, "unknown operator kind");
  if (d->n_terms < 0 || (d->n_terms > 0 && (!d->values || !d->indices)))
    fail(HGF_EINVAL, "sparse operator needs values and indices");
  // accumulate g over (k, l)
  std::map<std::pair<std::vector<int>, std::vector<int>>, cd> acc;
  for (int64_t t = 0; t < d->n_terms; ++t) {
    std::vector<int> k(n), l(n);
    for (int j = 0; j < n; ++j) {
      k[j] = d->indices[t * 2 * n + j];
      l[j] = d->indices[t * 2 * n + n + j];
      if (k[j] < 0 || k[j] >= s.nc[j] || l[j] < 0 || l[j] >= s.nc[j])
        fail(HGF_EINVAL, "sparse operator index outside the cutoff box");
    }
    const cd val(d->values[2 * t], d->values[2 * t + 1]);
    if (!std::isfinite(val.real()) || !std::isfinite(val.imag())) fail(HGF_EINVAL, "non-finite operator entry");
    if (d->basis == HGF_BASIS_NUMBER) {
      double sc = 1.0;
      for (int j = 0; j < n; ++j) sc *= sqrt_factorial(k[j]) * sqrt_factorial(l[j]);
      acc[{k, l}] += val / sc;
    } else {
      // Eq. (6) in several modes: f_{k,l} feeds g_{k+i, l+i} with weight prod_j 1/i_j!
      std::vector<int> i(n, 0);
      while (true) {
        bool inside = true;
        double w = 1.0;
        std::vector<int> kk(n), ll(n);
        for (int j = 0; j < n; ++j) {
          kk[j] = k[j] + i[j];
          ll[j] = l[j] + i[j];
          if (kk[j] >= s.nc[j] || ll[j] >= s.nc[j]) inside = false;
          w /= factorial(i[j]);
        }
        if (inside) acc[{kk, ll}] += val * w;
        int j = n - 1;
        while (j >= 0) {
          if (k[j] + i[j] + 1 < s.nc[j] && l[j] + i[j] + 1 < s.nc[j]) {
            ++i[j];
            break;
          }
          i[j] = 0;
          --j;
        }
        if (j < 0) break;
      }
    }
  }
  int64_t total_points = 0;
  for (auto& kv : acc) {
    const auto& k = kv.first.first;
    const auto& l = kv.first.second;
    if (kv.second == 0.0) continue;
    if (want_split) {
      split.push_back(Coeff{k, l, kv.second});
    } else {
      std::vector<int> dv(n);
      int e[kMaxModes], m[kMaxModes];
      for (int j = 0; j < n; ++j) {
        dv[j] = l[j] - k[j];
        e[j] = s.nc[j] - std::abs(dv[j]);
        m[j] = std::min(k[j], l[j]);
      }
      auto it = merged.find(dv);
      if (it == merged.end()) {
        const int64_t pts = checked_points(e, n);
        add_points(total_points, pts);
        it = merged.emplace(dv, std::vector<cd>(pts, 0.0)).first;
      }
      int64_t f = 0;
      for (int j = 0; j < n; ++j) f = f * e[j] + m[j];
      it->second[f] += kv.second;
    }
  }
}


// Host-side size check of an operator before any device work: the grids its
// coefficients populate must stay within kMaxOperatorPoints (per sector and in
// total), and a network operator's full (k, l) grid within kMaxFullPoints.
// Product operators: the sector sizes factorise over the modes, so the total
// is the product of the per-mode sums over their nonzero diagonals.  Sparse
// operators: each distinct sector's size once.  Dense operators are bounded
// by their own dimension limit.
static void precheck_operator_size(const System& s, const hgf_operator_desc* d) {
  const int n = s.n;
  if (s.full) {
    int64_t dim = 1;
    for (int j = 0; j < n; ++j) {
      dim *= s.nc[j];
      if (dim * dim > kMaxFullPoints) fail(HGF_EINVAL, "full (k, l) grid of the network exceeds 2^28 points");
    }
    return;
  }
  if (d->kind == HGF_OP_PRODUCT && d->values) {
    int tot[kMaxModes];
    size_t off = 0;
    for (int j = 0; j < n; ++j) {
      const int nc = s.nc[j];
      int sj = 0;
      for (int dj = -nc + 1; dj < nc; ++dj) {
        bool nz = false;
        for (int k = 0; k < nc && !nz; ++k) {
          const int l = k + dj;
          if (l >= 0 && l < nc)
            nz = d->values[off + 2 * (k * nc + l)] != 0.0 || d->values[off + 2 * (k * nc + l) + 1] != 0.0;
        }
        if (nz) sj += nc - std::abs(dj);
      }
      if (sj == 0) return;  // zero operator
      tot[j] = sj;
      off += 2 * (size_t)nc * nc;
    }
    checked_points(tot, n);
  } else if (d->kind == HGF_OP_SPARSE && d->indices && d->n_terms > 0) {
    std::set<std::vector<int>> seen;
    int64_t total = 0;
    for (int64_t t = 0; t < d->n_terms; ++t) {
      std::vector<int> dv(n);
      int e[kMaxModes];
      for (int j = 0; j < n; ++j) {
        const int k = d->indices[t * 2 * n + j], l = d->indices[t * 2 * n + n + j];
        if (k < 0 || k >= s.nc[j] || l < 0 || l >= s.nc[j])
          fail(HGF_EINVAL, "sparse operator index outside the cutoff box");
        dv[j] = l - k;
        e[j] = s.nc[j] - std::abs(dv[j]);
      }
      if (seen.insert(dv).second) add_points(total, checked_points(e, n));
    }
  }
}

static void upload_state(Function& f, const std::vector<cd>& grid, int precision) {
  static_assert(sizeof(cd) == sizeof(double2), "layout");
  if (f.real) {
    std::vector<double> r(grid.size());
    for (size_t i = 0; i < grid.size(); ++i) r[i] = grid[i].real();
    hip_check(hipMemcpy(f.y, r.data(), r.size() * sizeof(double), hipMemcpyHostToDevice), "upload state");
  } else {
    hip_check(hipMemcpy(f.y, grid.data(), grid.size() * sizeof(double2), hipMemcpyHostToDevice), "upload state");
  }
  launch_shadow(precision, f.ga, f.y, f.yf, nullptr);
  hip_check(hipGetLastError(), "shadow copy");
}

// energy of the number state |k>
static double energy(const System& s, const int* k) {
  double e = 0.0;
  for (int j = 0; j < s.n; ++j) e += s.det[j] * k[j] + 0.5 * s.kerr[j] * k[j] * (k[j] - 1);
  for (int i = 0; i < s.n; ++i)
    for (int j = i + 1; j < s.n; ++j) e += s.chi[i][j] * k[i] * k[j];
  return e;
}

// Split layout (Eqs. (9), (19)-(20)): G^{(p,q)} = c_x x^p c_y y^q + R with
//   dc_x/dt = (rho_x + C) c_x,  dc_y/dt = (rho_y - C) c_y,
//   dR/dt   = L R + c_x c_y S,  S = L[x^p y^q] - (rho_x + rho_y) x^p y^q,
// where rho_x + rho_y is the diagonal rate lambda at (p, q) minus the
// dephasing cross term, rho_x collects the p-dependent and rho_y the
// q-dependent part, and C = -(i/2)(E(p) + E(q)) minimises
// |c_x'/c_x|^2 + |c_y'/c_y|^2 of the undamped system (Eq. (20)).
static void setup_split(Function& f, const System& s, const Coeff& c) {
  const int n = s.n;
  const cd I(0.0, 1.0);
  int p[kMaxModes], q[kMaxModes], m[kMaxModes];
  for (int j = 0; j < n; ++j) {
    p[j] = c.k[j];
    q[j] = c.l[j];
    f.p[j] = p[j];
    f.q[j] = q[j];
    m[j] = std::min(p[j], q[j]);
  }
  const double Ep = energy(s, p), Eq = energy(s, q);
  cd rx = I * Ep, ry = -I * Eq;
  for (int j = 0; j < n; ++j) {
    const double down = s.g1[j] * (1 + s.nth[j]), up = s.g1[j] * s.nth[j];
    const double pt = (p[j] + 1 < s.nc[j]) ? p[j] + 1 : 0, qt = (q[j] + 1 < s.nc[j]) ? q[j] + 1 : 0;
    rx -= 0.5 * down * p[j] + 0.5 * up * pt + s.gphi[j] * double(p[j] * p[j]);
    ry -= 0.5 * down * q[j] + 0.5 * up * qt + s.gphi[j] * double(q[j] * q[j]);
  }
  const cd C = -0.5 * I * (Ep + Eq);
  f.ax = rx + C;
  f.ay = ry - C;
  f.cx = 1.0;
  f.cy = 1.0;
  f.g0 = c.v;
  f.mono_index = flat_index(f.tab, m);
  // S = L delta_{m*} - (rho_x + rho_y) delta_{m*}
  const SectorTables& t = f.tab;
  cd lam = t.lam0;
  for (int j = 0; j < n; ++j) lam += t.lam[j][m[j]];
  f.sources.clear();
  f.sources.push_back({f.mono_index, lam - (rx + ry)});
  for (int j = 0; j < n; ++j) {
    int mm[kMaxModes];
    std::memcpy(mm, m, sizeof(int) * n);
    if (m[j] + 1 < t.ext[j]) {  // (L delta)(m*+e_j) = alpha_j(m*_j + 1)
      mm[j] = m[j] + 1;
      const double a = t.alpha[j][m[j] + 1];
      if (a != 0.0) f.sources.push_back({flat_index(t, mm), cd(a, 0.0)});
    }
    if (m[j] >= 1) {  // (L delta)(m*-e_j) = beta_j(m*_j - 1)
      mm[j] = m[j] - 1;
      const double b = t.beta[j][m[j] - 1];
      if (b != 0.0) f.sources.push_back({flat_index(t, mm), cd(b, 0.0)});
    }
  }
}


// Generator tables of a network operator's full grid (see FullTables).
FullTables full_tables(const System& s) {
  FullTables ft{};
  ft.n = s.n;
  ft.secular = s.secular;
  for (int j = 0; j < s.n; ++j) {
    const int nc = s.nc[j];
    ft.nc[j] = nc;
    ft.gphi[j] = s.gphi[j];
    ft.drive_re[j] = s.drive_re[j];
    ft.drive_im[j] = s.drive_im[j];
    for (int i = 0; i < s.n; ++i) {
      ft.chi[i][j] = s.chi[i][j];
      ft.exch[i][j] = s.exch[i][j];
    }
    const double g = s.g1[j];
    for (int k = 0; k < nc; ++k) {
      ft.e[j][k] = s.det[j] * k + 0.5 * s.kerr[j] * k * (k - 1);
      if (s.secular) {
        const double* nb = s.nlev[j];
        double out = 0.0;
        if (k >= 1) out += g * k * (nb[k - 1] + 1.0);
        if (k + 1 < nc) out += g * (k + 1) * nb[k];
        ft.dk[j][k] = -0.5 * out;
        ft.adn[j][k] = k >= 1 ? g * (nb[k - 1] + 1.0) : 0.0;
        ft.aup[j][k] = k + 1 < nc ? g * nb[k] * (double)(k + 1) * (double)(k + 1) : 0.0;
      } else {
        const double kt = (k + 1 < nc) ? k + 1 : 0;
        ft.dk[j][k] = -0.5 * (g * (1.0 + s.nth[j]) * k + g * s.nth[j] * kt);
        ft.adn[j][k] = g * (1.0 + s.nth[j]);
        ft.aup[j][k] = g * s.nth[j];
      }
    }
  }
  return ft;
}

// Gershgorin-type bound on the generator of a network operator's full grid:
// the largest diagonal entry (|E(k) - E(l)| is at most the range of E over
// the grid, plus the damping and dephasing) plus every neighbour coefficient
// at its largest.
double full_generator_bound(const FullTables& ft) {
  double erange = 0.0, dmax = 0.0, b = 0.0;
  for (int j = 0; j < ft.n; ++j) {
    const int nc = ft.nc[j];
    double elo = ft.e[j][0], ehi = ft.e[j][0], dj = 0.0, a = 0.0, u = 0.0;
    for (int k = 0; k < nc; ++k) {
      elo = std::min(elo, ft.e[j][k]);
      ehi = std::max(ehi, ft.e[j][k]);
      dj = std::max(dj, std::abs(ft.dk[j][k]));
      a = std::max(a, ft.adn[j][k]);
      u = std::max(u, ft.secular ? ft.aup[j][k] : ft.aup[j][k] * nc * nc);
    }
    erange += ehi - elo;
    dmax += 2.0 * dj + ft.gphi[j] * (nc - 1) * (nc - 1);
    for (int i = 0; i < j; ++i) erange += std::abs(ft.chi[i][j]) * (ft.nc[i] - 1) * (nc - 1);
    b += a + u + std::hypot(ft.drive_re[j], ft.drive_im[j]) * 2.0 * (nc + 1);
    for (int i = 0; i < j; ++i) b += std::abs(ft.exch[i][j]) * 2.0 * (ft.nc[i] + nc);
  }
  return erange + dmax + b;
}

// Tile records of a network operator's tiled stage kernel (layout: FullTileRec
// then FullTerm entries, `rec_bytes` per tile).  Tile t is the (k, l) block of
// the last two modes at slow coordinates (k_0, l_0, ..., k_{N-3}, l_{N-3}) =
// the mixed-radix digits of t.  Terms: for every slow mode its jumps and
// drive; for every exchange pair with a slow mode its four shifts (an
// exchange with P or Q also shifts that fast axis, checked per point).
static std::vector<char> full_tile_records(const GridArgs& g, const FullTables& ft, int& rec_bytes) {
  const int n = ft.n, P = n - 2, ns = n - 2;  // P, P + 1: the fast modes
  int64_t ntiles = 1;
  for (int j = 0; j < ns; ++j) ntiles *= (int64_t)ft.nc[j] * ft.nc[j];
  auto sk = [&](int j) { return (int32_t)g.stride[2 * j]; };
  auto sl = [&](int j) { return (int32_t)g.stride[2 * j + 1]; };
  std::vector<std::vector<FullTerm>> terms((size_t)ntiles);
  std::vector<FullTileRec> heads((size_t)ntiles);
  size_t umax = 0;
  int k[kMaxFullModes], l[kMaxFullModes];
  for (int64_t t = 0; t < ntiles; ++t) {
    int64_t r = t;
    for (int j = ns - 1; j >= 0; --j) {
      l[j] = (int)(r % ft.nc[j]);
      r /= ft.nc[j];
      k[j] = (int)(r % ft.nc[j]);
      r /= ft.nc[j];
    }
    FullTileRec h{};
    std::vector<FullTerm>& tv = terms[(size_t)t];
    auto add = [&](int32_t off, double cr, double ci, int32_t meta) {
      if (cr != 0.0 || ci != 0.0) tv.push_back(FullTerm{off, meta, cr, ci});
    };
    for (int j = 0; j < ns; ++j) {
      const int kj = k[j], lj = l[j], nc = ft.nc[j];
      h.lam_re += ft.dk[j][kj] + ft.dk[j][lj] - ft.gphi[j] * (double)((kj - lj) * (kj - lj));
      h.lam_im += ft.e[j][kj] - ft.e[j][lj];
      for (int i = 0; i < j; ++i) h.lam_im += ft.chi[i][j] * (double)(k[i] * kj - l[i] * lj);
      for (int m = 0; m < 2; ++m) {
        h.ck[m] += ft.chi[j][P + m] * kj;
        h.cl[m] += ft.chi[j][P + m] * lj;
      }
      // jumps: g(k - e_j, l - e_j), g(k + e_j, l + e_j)
      if (!ft.secular || kj == lj) {
        if (kj >= 1 && lj >= 1) add(-(sk(j) + sl(j)), ft.adn[j][ft.secular ? kj : 0], 0.0, 0);
        if (kj + 1 < nc && lj + 1 < nc)
          add(sk(j) + sl(j), ft.secular ? ft.aup[j][kj] : ft.aup[j][0] * (double)((kj + 1) * (lj + 1)), 0.0, 0);
      }
      // drive: i [Om g(k-e) + conj(Om)(k+1) g(k+e) - Om (l+1) g(l+e) - conj(Om) g(l-e)]
      const double orr = ft.drive_re[j], oi = ft.drive_im[j];
      if (orr != 0.0 || oi != 0.0) {
        if (kj >= 1) add(-sk(j), -oi, orr, 0);
        if (kj + 1 < nc) add(sk(j), oi * (kj + 1), orr * (kj + 1), 0);
        if (lj + 1 < nc) add(sl(j), oi * (lj + 1), -orr * (lj + 1), 0);
        if (lj >= 1) add(-sl(j), -oi, -orr, 0);
      }
    }
    // exchange i < j with i slow: i J [(k_j+1) g(k - e_i + e_j) + (k_i+1) g(k - e_j + e_i)
    //                                  - (l_i+1) g(l - e_j + e_i) - (l_j+1) g(l - e_i + e_j)]
    for (int j = 1; j < n; ++j)
      for (int i = 0; i < std::min(j, ns); ++i) {
        const double J = ft.exch[i][j];
        if (J == 0.0) continue;
        const int nci = ft.nc[i], ncj = ft.nc[j], ki = k[i], li = l[i];
        if (j < ns) {
          const int kj = k[j], lj = l[j];
          if (ki >= 1 && kj + 1 < ncj) add(-sk(i) + sk(j), 0.0, J * (kj + 1), 0);
          if (kj >= 1 && ki + 1 < nci) add(-sk(j) + sk(i), 0.0, J * (ki + 1), 0);
          if (lj >= 1 && li + 1 < nci) add(-sl(j) + sl(i), 0.0, -J * (li + 1), 0);
          if (li >= 1 && lj + 1 < ncj) add(-sl(i) + sl(j), 0.0, -J * (lj + 1), 0);
        } else {  // j = P or Q: fast axes 2 (j - P) (k_j) and 2 (j - P) + 1 (l_j)
          const int32_t ak = 2 * (j - P), al = ak + 1;
          if (ki >= 1) add(-sk(i) + sk(j), 0.0, J, ak | kFullShift | kFullUp | kFullFactor);
          if (ki + 1 < nci) add(-sk(j) + sk(i), 0.0, J * (ki + 1), ak | kFullShift);
          if (li + 1 < nci) add(-sl(j) + sl(i), 0.0, -J * (li + 1), al | kFullShift);
          if (li >= 1) add(-sl(i) + sl(j), 0.0, -J, al | kFullShift | kFullUp | kFullFactor);
        }
      }
    h.nterms = (int32_t)tv.size();
    heads[(size_t)t] = h;
    umax = std::max(umax, tv.size());
  }
  rec_bytes = (int)(sizeof(FullTileRec) + umax * sizeof(FullTerm));
  std::vector<char> out((size_t)ntiles * rec_bytes, 0);
  for (int64_t t = 0; t < ntiles; ++t) {
    char* b = out.data() + (size_t)t * rec_bytes;
    std::memcpy(b, &heads[(size_t)t], sizeof(FullTileRec));
    if (!terms[(size_t)t].empty())
      std::memcpy(b + sizeof(FullTileRec), terms[(size_t)t].data(), terms[(size_t)t].size() * sizeof(FullTerm));
  }
  return out;
}

// Configure the tiled stage kernel of a network operator (at least three
// modes; a tile of 256 to 4096 points whose LDS fits 64 KB; records at most a
// quarter of the grid's state bytes; unless c.nfast asks for it, at least 256
// tiles).  c.threads (0: the size with the least
// idle lanes in the last round), c.wgs_per_cu and c.wblock (-1: 3 from four
// modes on) apply.  Returns false, leaving f unchanged, when the kernel does
// not fit.
static bool configure_full_tiles(Function& f, const FullTables& ft, int precision, const TileChoice& c) {
  const int n = ft.n;
  if (n < 3) return false;
  const int ncP = ft.nc[n - 2], ncQ = ft.nc[n - 1];
  const int T = ncP * ncP * ncQ * ncQ;
  if (T < 256 || T > 512 * full_tiled_max_rounds()) return false;
  // by default only grids of at least 256 tiles (fewer leave CUs idle: the
  // untiled kernel was faster on the three-mode network of 36 tiles)
  if (c.nfast < 0 && f.ga.points / T < 256) return false;
  const size_t lds = full_tiled_lds_bytes(precision, T);
  if (lds > 65536) return false;
  int threads = c.threads;
  if (threads == 0) {
    int64_t best = -1;
    for (int th = 128; th <= 512; th += 64) {
      const int64_t r = (T + th - 1) / th;
      if (r > full_tiled_max_rounds()) continue;
      if (best < 0 || r * th < best) {
        best = r * th;
        threads = th;
      }
    }
  }
  if (threads < 64 || threads > 512 || threads % 64 != 0 || (T + threads - 1) / threads > full_tiled_max_rounds())
    return false;
  int occ = full_tiled_blocks_per_cu(precision, threads, (int)lds);
  if (occ <= 0 || c.wgs_per_cu > occ) return false;
  if (c.wgs_per_cu > 0) occ = c.wgs_per_cu;
  GridArgs g = f.ga;
  int rec_bytes = 0;
  std::vector<char> rec = full_tile_records(g, ft, rec_bytes);
  const int64_t ntiles = g.points / T;
  if ((int64_t)rec.size() > std::max<int64_t>((int64_t)64 << 20, g.points * 16 / 4)) return false;
  // walk order: blocks of 3 along every slow axis unless set (fastest
  // measured on the five-mode, cutoff-6 network in both precisions)
  const int wblock = c.wblock >= 0 ? c.wblock : (n >= 4 ? 3 : 0);
  std::vector<uint32_t> order;
  if (wblock >= 2) {
    GridArgs w = g;
    w.nfast = 4;
    w.wblock = wblock;
    order = walk_order(w);
  }
  const size_t rb = (rec.size() + 255) / 256 * 256;
  rec.resize(rb + order.size() * sizeof(uint32_t), 0);
  if (!order.empty()) std::memcpy(rec.data() + rb, order.data(), order.size() * sizeof(uint32_t));
  void* d = dmalloc(rec.size());
  const hipError_t e = hipMemcpy(d, rec.data(), rec.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    dfree(d);
    hip_check(e, "upload tile records");
  }
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) == hipSuccess) (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  g.tiles = d;
  g.walk = order.empty() ? nullptr : (const uint32_t*)((const char*)d + rb);
  g.ftile = T;
  g.fntiles = ntiles;
  g.frec = rec_bytes;
  g.fthreads = threads;
  g.flds = (int)lds;
  g.fwblock = order.empty() ? 0 : wblock;
  g.fwgs = c.wgs_per_cu;
  g.fblocks = (int)std::max<int64_t>(8, std::min<int64_t>((int64_t)cus * occ, 8 * ((ntiles + 7) / 8)));
  dfree(f.ttab);
  f.ttab = d;
  f.ga = g;
  return true;
}

// Back to the untiled stage kernel.
static void drop_full_tiles(Function& f) {
  f.ga.fblocks = 0;
  f.ga.tiles = nullptr;
  f.ga.walk = nullptr;
  dfree(f.ttab);
}

// Order of the modes on a network operator's full grid: position p holds mode
// perm[p] (slowest first) and the last two positions form the tiles.  The
// pair whose own drives and mutual exchange give the most neighbour terms
// goes last (those terms then read LDS); then, from the fast end, the mode
// with the most exchange terms to the modes already placed, plus its own
// drive terms (so the remaining terms reach near tiles).  Ties keep the given
// order.
static void full_mode_order(const System& s, int* perm) {
  const int n = s.n;
  for (int p = 0; p < n; ++p) perm[p] = p;
  if (n < 3) return;
  auto drv = [&](int j) { return (s.drive_re[j] != 0.0 || s.drive_im[j] != 0.0) ? 4 : 0; };
  auto ex = [&](int i, int j) { return s.exch[i][j] != 0.0 ? 4 : 0; };
  int bp = n - 2, bq = n - 1, best = drv(n - 2) + drv(n - 1) + ex(n - 2, n - 1);
  for (int j = n - 1; j >= 1; --j)
    for (int i = j - 1; i >= 0; --i) {
      const int sc = drv(i) + drv(j) + ex(i, j);
      if (sc > best) {
        best = sc;
        bp = i;
        bq = j;
      }
    }
  bool placed[kMaxFullModes] = {};
  perm[n - 2] = bp;
  perm[n - 1] = bq;
  placed[bp] = placed[bq] = true;
  for (int p = n - 3; p >= 0; --p) {
    int bj = -1, bs = -1;
    for (int j = n - 1; j >= 0; --j) {
      if (placed[j]) continue;
      int sc = drv(j);
      for (int q = p + 1; q < n; ++q) sc += ex(j, perm[q]);
      if (sc > bs) {
        bs = sc;
        bj = j;
      }
    }
    perm[p] = bj;
    placed[bj] = true;
  }
}

// The system with its modes reordered: mode p of the result is mode perm[p].
static System permute_modes(const System& s, const int* perm) {
  System t = s;
  for (int p = 0; p < s.n; ++p) {
    const int j = perm[p];
    t.nc[p] = s.nc[j];
    t.det[p] = s.det[j];
    t.kerr[p] = s.kerr[j];
    t.g1[p] = s.g1[j];
    t.gphi[p] = s.gphi[j];
    t.nth[p] = s.nth[j];
    for (int c = 0; c < kMaxCutoff; ++c) t.nlev[p][c] = s.nlev[j][c];
    t.drive_re[p] = s.drive_re[j];
    t.drive_im[p] = s.drive_im[j];
    for (int q = 0; q < s.n; ++q) {
      t.chi[p][q] = s.chi[j][perm[q]];
      t.exch[p][q] = s.exch[j][perm[q]];
    }
  }
  return t;
}

// A network operator: every sector of the input scattered into one full
// (k, l) grid, g(k, l) = <k|A|l> / sqrt(k! l!).
static void build_full_function(hgf_operator_s* op, const hgf_operator_desc* d) {
  if (op->layout != HGF_MERGED) fail(HGF_EUNSUPPORTED, "a driven or exchange-coupled system needs the merged layout");
  const System& s = op->sys;
  const int n = s.n;
  int64_t dim = 1;
  for (int j = 0; j < n; ++j) {
    dim *= s.nc[j];
    if (dim * dim > kMaxFullPoints) fail(HGF_EINVAL, "full (k, l) grid of the network exceeds 2^28 points");
  }
  std::map<std::vector<int>, std::vector<cd>> merged;
  std::vector<Coeff> coeffs;
  collect_coeffs(s, d, merged, coeffs, false);
  int perm[kMaxFullModes];
  full_mode_order(s, perm);
  std::vector<cd> grid((size_t)(dim * dim), 0.0);
  bool any = false;
  for (auto& kv : merged) {
    const std::vector<int>& dv = kv.first;
    int u[kMaxModes], v[kMaxModes], e[kMaxModes];
    for (int j = 0; j < n; ++j) {
      u[j] = dv[j] < 0 ? -dv[j] : 0;
      v[j] = dv[j] > 0 ? dv[j] : 0;
      e[j] = s.nc[j] - std::abs(dv[j]);
    }
    std::vector<int> m(n, 0);
    for (size_t p = 0; p < kv.second.size(); ++p) {
      cd val = kv.second[p];
      if (std::abs(val) <= d->drop_tol) val = 0.0;
      if (val != 0.0) {
        any = true;
        if (std::abs(val) < FLT_MIN) op->underflow++;
        int64_t at = 0;  // axes k, l of the mode at each position
        for (int p = 0; p < n; ++p) {
          const int j = perm[p];
          at = at * s.nc[j] + m[j] + u[j];
          at = at * s.nc[j] + m[j] + v[j];
        }
        grid[(size_t)at] = val;
      }
      for (int j = n - 1; j >= 0; --j) {
        if (++m[j] < e[j]) break;
        m[j] = 0;
      }
    }
  }
  if (!any) return;  // the zero operator
  op->fn.emplace_back();
  Function& f = op->fn.back();
  f.full = true;
  SectorTables& t = f.tab;
  t.n = 2 * n;
  t.lam0 = 0.0;
  for (int a = 0; a < 2 * n; ++a) {
    t.d[a] = t.u[a] = t.v[a] = 0;
    t.ext[a] = s.nc[perm[a / 2]];
    t.lam[a].assign(t.ext[a], cd(0.0));
    t.alpha[a].assign(t.ext[a], 0.0);
    t.beta[a].assign(t.ext[a], 0.0);
  }
  const FullTables ft = full_tables(permute_modes(s, perm));
  std::copy(perm, perm + n, f.fperm);
  f.fhost.assign(1, ft);
  f.full_bound = full_generator_bound(ft);
  f.ftab = dmalloc(sizeof(FullTables));
  hip_check(hipMemcpy(f.ftab, &ft, sizeof(FullTables), hipMemcpyHostToDevice), "upload tables");
  fill_grid_args(f, op->precision, false);
  if (!stage_kernel_generic()) configure_full_tiles(f, ft, op->precision, TileChoice{});
  alloc_function_buffers(f, op->precision);
  upload_state(f, grid, op->precision);
}

static void build_functions(hgf_operator_s* op, const hgf_operator_desc* d, bool allow_real = true) {
  if (op->sys.full) {
    build_full_function(op, d);
    return;
  }
  std::map<std::vector<int>, std::vector<cd>> merged;
  std::vector<Coeff> coeffs;
  const bool split = op->layout == HGF_SPLIT;
  collect_coeffs(op->sys, d, merged, coeffs, split);
  const int n = op->sys.n;
  if (!split) {
    for (auto& kv : merged) {
      bool any = false;
      for (auto& v : kv.second) {
        if (std::abs(v) <= d->drop_tol) v = 0.0;
        if (v != 0.0) any = true;
        if (v != 0.0 && std::abs(v) < FLT_MIN) op->underflow++;
      }
      if (!any) continue;
      op->fn.emplace_back();
      Function& f = op->fn.back();
      f.tab = sector_tables(op->sys, kv.first.data());
      bool real = allow_real;
      if (real) {
        const char* env = std::getenv("HGF_REAL_GRIDS");
        if (env && std::string(env) == "0") real = false;
      }
      if (f.tab.lam0.imag() != 0.0) real = false;
      for (int j = 0; j < f.tab.n && real; ++j)
        for (const cd& l : f.tab.lam[j])
          if (l.imag() != 0.0) real = false;
      for (const cd& v : kv.second)
        if (v.imag() != 0.0) real = false;
      fill_grid_args(f, op->precision, real);
      alloc_function_buffers(f, op->precision);
      upload_state(f, kv.second, op->precision);
    }
  } else {
    for (const Coeff& c : coeffs) {
      if (std::abs(c.v) <= d->drop_tol) continue;
      if (std::abs(c.v) < FLT_MIN) op->underflow++;
      int dv[kMaxModes];
      for (int j = 0; j < n; ++j) dv[j] = c.l[j] - c.k[j];
      op->fn.emplace_back();
      Function& f = op->fn.back();
      f.split = true;
      f.tab = sector_tables(op->sys, dv);
      fill_grid_args(f, op->precision, false);
      alloc_function_buffers(f, op->precision);
      std::vector<cd> zero(f.ga.points, 0.0);
      upload_state(f, zero, op->precision);
      setup_split(f, op->sys, c);
    }
  }
}

// ------------------------------------------------------------------ stepping

void reset_flag(hgf_operator_s* op, hipStream_t st) {
  hip_check(hipMemsetAsync(op->dflag, 0, sizeof(int), st), "reset flag");
}

// ---- merged-layout stepping
// A StepPlan runs one RK4 step of a set of (function, precision, step size)
// items: functions with a tiled configuration as grouped launches (one launch
// per axis split, element type and precision, covering every member's tiles),
// the others with the generic kernel.
struct PlanItem {
  Function* f;
  int precision;
  double h;
};

struct StepPlan {
  std::vector<GroupLaunch> groups;
  std::vector<void*> dmem;
  std::vector<PlanItem> generic;
  // resident launches, with host copies of their items (the step count is set
  // per call)
  std::vector<ResidentLaunch> resident;
  std::vector<std::vector<ResidentItem>> res_host;
  ~StepPlan() {
    for (auto& p : dmem) dfree(p);
  }
};

static MemberArgs member_args(const PlanItem& it) {
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

static StepPlan* build_plan(const std::vector<PlanItem>& items, bool allow_resident = true) {
  std::unique_ptr<StepPlan> plan(new StepPlan);
  std::map<std::vector<int>, std::vector<PlanItem>> by_key, res_key;
  for (const PlanItem& it : items) {
    const GridArgs& g = it.f->ga;
    if (allow_resident && it.f->resident)
      res_key[{g.nfast, g.real, it.precision}].push_back(it);
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
    std::vector<ResidentItem> host;
    for (const PlanItem& it : kv.second) {
      ResidentItem ri{};
      ri.g = it.f->ga;
      ri.y = it.f->y;
      ri.yf = it.precision == HGF_MIXED ? it.f->yf : nullptr;
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
constexpr int64_t kResidentChunk = 8192;
static void run_resident(StepPlan& plan, int64_t steps, int* flag, hipStream_t st) {
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
static void stage_launch(const Function& f, int precision, int stage, const void* in, const void* x1, void* y,
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

static void generic_stage(const PlanItem& it, int s, int* flag, hipStream_t st) {
  Function& f = *it.f;
  const void* in[4] = {it.precision == HGF_MIXED ? f.yf : f.y, f.s1, f.s2, f.s3};
  void* out[4] = {f.s1, f.s2, f.s3, nullptr};
  (f.full ? (f.ga.fblocks > 0 ? launch_full_tiled : launch_full_horner) : launch_horner)(s, it.precision, f.ga, in[s - 1], f.s1, f.y,
                                                it.precision == HGF_MIXED ? f.yf : nullptr, out[s - 1], it.h, flag,
                                                st);
}

static void run_plan_step(const StepPlan& plan, int* flag, hipStream_t st) {
  for (int s = 1; s <= 4; ++s) {
    for (const GroupLaunch& gl : plan.groups) launch_group(gl, s, flag, st);
    for (const PlanItem& it : plan.generic) generic_stage(it, s, flag, st);
  }
}

static void drop_graph(hgf_operator_s* op) {
  if (op->graph_exec) (void)hipGraphExecDestroy((hipGraphExec_t)op->graph_exec);
  op->graph_exec = nullptr;
  op->graph_steps = 0;
}

static void drop_plan(hgf_operator_s* op) {
  drop_graph(op);
  delete op->plan;
  op->plan = nullptr;
}

static void ensure_plan(hgf_operator_s* op, double h) {
  if (op->plan && op->graph_dt == h) return;
  drop_plan(op);
  std::vector<PlanItem> items;
  for (auto& f : op->fn) items.push_back({&f, op->precision, h});
  op->plan = build_plan(items);
  op->graph_dt = h;
}

// Owns an executable graph.
struct GraphHolder {
  hipGraphExec_t e;
  explicit GraphHolder(hipGraphExec_t x) : e(x) {}
  ~GraphHolder() { (void)hipGraphExecDestroy(e); }
  GraphHolder(const GraphHolder&) = delete;
  GraphHolder& operator=(const GraphHolder&) = delete;
};

static hipGraphExec_t capture_steps(const StepPlan& plan, int* flag, int chunk, hipStream_t cap) {
  hipGraph_t graph;
  hip_check(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
  for (int s = 0; s < chunk; ++s) run_plan_step(plan, flag, cap);
  hip_check(hipStreamEndCapture(cap, &graph), "end capture");
  hipGraphExec_t exec;
  hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
  (void)hipGraphDestroy(graph);
  hip_check(e, "graph instantiate");
  return exec;
}

// Steps per captured graph: at most 64, and at most kMaxGraphNodes kernel
// nodes (an operator whose many functions each take their own generic launch
// would otherwise capture graphs of millions of nodes).  0: launch eagerly.
constexpr int64_t kMaxGraphNodes = 16384;
static int graph_chunk(const StepPlan& plan, int64_t steps) {
  const int64_t per_step = 4 * (int64_t)(plan.groups.size() + plan.generic.size());
  if (per_step == 0) return 0;
  return (int)std::min<int64_t>({steps, 64, kMaxGraphNodes / per_step});
}

// One graph holds `chunk` merged steps of every function of the operator.
static void ensure_graph(hgf_operator_s* op, double h, int chunk) {
  ensure_plan(op, h);
  if (op->graph_exec && op->graph_steps == chunk) return;
  drop_graph(op);
  if (!op->cap_stream) hip_check(hipStreamCreateWithFlags(&op->cap_stream, hipStreamNonBlocking), "stream");
  op->graph_exec = capture_steps(*op->plan, op->dflag, chunk, op->cap_stream);
  op->graph_steps = chunk;
}

static void split_step(hgf_operator_s* op, Function& f, double h, hipStream_t st) {
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
static void ensure_lawson_tables(Function& f, double h, hipStream_t st) {
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
static void lawson_steps(hgf_operator_s* op, int64_t steps, double h, hipStream_t st) {
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
static void apply_threshold(hgf_operator_s* op, hipStream_t st) {
  for (auto& f : op->fn) launch_threshold((double2*)f.y, f.ga.points, op->threshold, op->dcount, st);
  launch_threshold_peak(op->dcount, op->dcount + 1, st);
}

static void evolve_impl(hgf_operator_s* op, int64_t steps, double h, hipStream_t st, int scheme = HGF_RK4) {
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
static void batch_impl(hgf_operator* ops, int n, const std::vector<int64_t>& steps, const double* dt, hipStream_t st) {
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

// ------------------------------------------------------------------ launch-shape autotuner
// The tiled stage kernel's launch shape (fast axes, workgroup size, XCD tile
// order, pipelined loads) is chosen per grid shape by timing candidate shapes
// on the function's own buffers.  Results are kept in a text cache, one line
// per shape: "<key> <nfast> <threads> <xblock> <pipe> <wgs_per_cu> <walk_block> <stage_us>", the key
// naming the device (architecture, CU count), precision, real or complex grid
// and the extents.

// Re-configure one function's stage kernel; the function is left unchanged
// when the shape is not feasible (HGF_EINVAL).
static void retile(Function& f, int precision, const TileChoice& c) {
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

static std::string device_tag() {
  int dev = 0;
  hip_check(hipGetDevice(&dev), "hipGetDevice");
  hipDeviceProp_t prop;
  hip_check(hipGetDeviceProperties(&prop, dev), "hipGetDeviceProperties");
  std::string arch = prop.gcnArchName;
  const size_t colon = arch.find(':');
  if (colon != std::string::npos) arch = arch.substr(0, colon);
  return arch + ":" + std::to_string(prop.multiProcessorCount);
}

static std::string tune_key(const std::string& dev, const Function& f, int precision) {
  std::string k = dev + (precision == HGF_FP64 ? ":fp64" : ":mixed") + (f.real ? ":real:" : ":complex:");
  for (int j = 0; j < f.ga.n; ++j) k += (j ? "x" : "") + std::to_string(f.ga.ext[j]);
  return k;
}

struct TuneEntry {
  TileChoice c;
  double us = 0.0;
};

static std::map<std::string, TuneEntry> read_tune_cache(const char* path) {
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

static void write_tune_cache(const char* path, const std::map<std::string, TuneEntry>& m) {
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
static std::vector<TileChoice> tune_candidates(const Function& f, int precision) {
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
static TuneEntry pick_shape(const std::vector<TileChoice>& cands, const std::vector<double>& times) {
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
static double time_function_steps(Function& f, int precision, double h, int* flag, int steps, hipStream_t st) {
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

static TileChoice current_choice(const Function& f) {
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
static double time_plan_steps(const std::vector<PlanItem>& items, int* flag, int steps, hipStream_t st) {
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
// size and resident workgroups per CU, applied to every member (their numbers
// of fast axes are kept).  The cache key names the group's composition.
static void tune_groups(hgf_operator* ops, int n, double h, const std::string& dev,
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
    // candidates: workgroup sizes every member can use, full occupancy or one
    // to three workgroups per CU fewer
    std::vector<TileChoice> cands;
    for (int th = 64; th <= 512; th += 64)
      for (int w : {0, 1, 2, 3, 4, 6}) {
        TileChoice c;
        c.nfast = nfast;
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

static void autotune_impl(hgf_operator* ops, int n, double h, const char* cache_path, int flags, hipStream_t st) {
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

// ------------------------------------------------------------------ expectation

static std::vector<cd> mode_amps(const hgf_state_desc* psi, int j, int nc, size_t amp_off) {
  std::vector<cd> c(nc, 0.0);
  if (psi->kind == HGF_PSI_FOCK) {
    c[psi->fock[j]] = 1.0;
  } else if (psi->kind == HGF_PSI_COHERENT) {
    const cd a(psi->alpha[2 * j], psi->alpha[2 * j + 1]);
    double norm = 0.0;
    cd p = 1.0;
    for (int k = 0; k < nc; ++k) {
      c[k] = p / sqrt_factorial(k);
      norm += std::norm(c[k]);
      p *= a;
    }
    norm = std::sqrt(norm);
    for (auto& v : c) v /= norm;
  } else {
    for (int k = 0; k < nc; ++k) c[k] = cd(psi->amps[amp_off + 2 * k], psi->amps[amp_off + 2 * k + 1]);
  }
  return c;
}

void validate_state(const System& s, const hgf_state_desc* psi) {
  if (!psi) fail(HGF_EINVAL, "state is NULL");
  if (psi->kind == HGF_PSI_FOCK) {
    if (!psi->fock) fail(HGF_EINVAL, "fock occupations are NULL");
    for (int j = 0; j < s.n; ++j)
      if (psi->fock[j] < 0 || psi->fock[j] >= s.nc[j]) fail(HGF_EINVAL, "fock occupation outside the cutoff");
  } else if (psi->kind == HGF_PSI_COHERENT) {
    if (!psi->alpha) fail(HGF_EINVAL, "alpha is NULL");
    for (int j = 0; j < 2 * s.n; ++j)
      if (!std::isfinite(psi->alpha[j])) fail(HGF_EINVAL, "non-finite alpha");
  } else if (psi->kind == HGF_PSI_PRODUCT) {
    if (!psi->amps) fail(HGF_EINVAL, "amplitudes are NULL");
  } else {
    fail(HGF_EINVAL, "unknown state kind");
  }
}

// per-axis weights w_j(m) = sqrt(k! l!) conj(c_k) c_l of one sector, concatenated;
// on a network operator's full grid the k axes (even) take sqrt(k!) conj(c_k)
// and the l axes (odd) sqrt(l!) c_l (the weight of <k|A|l> factorises over them)
static std::vector<cd> sector_weights(const System& s, const Function& f, const std::vector<std::vector<cd>>& amps) {
  const SectorTables& t = f.tab;
  std::vector<cd> w;
  if (f.full) {
    for (int a = 0; a < t.n; ++a) {
      const int j = f.fperm[a / 2];
      for (int m = 0; m < t.ext[a]; ++m)
        w.push_back(a % 2 == 0 ? sqrt_factorial(m) * std::conj(amps[j][m]) : sqrt_factorial(m) * amps[j][m]);
    }
    return w;
  }
  for (int j = 0; j < t.n; ++j)
    for (int m = 0; m < t.ext[j]; ++m) {
      const int k = m + t.u[j], l = m + t.v[j];
      w.push_back(sqrt_factorial(k) * sqrt_factorial(l) * std::conj(amps[j][k]) * amps[j][l]);
    }
  return w;
}

std::vector<std::vector<cd>> all_amps(const System& s, const hgf_state_desc* psi) {
  std::vector<std::vector<cd>> amps(s.n);
  size_t off = 0;
  for (int j = 0; j < s.n; ++j) {
    amps[j] = mode_amps(psi, j, s.nc[j], off);
    off += 2 * (size_t)s.nc[j];
  }
  return amps;
}

// <psi0| A |psi0> over every function.  The device buffers of the call
// (weight tables, per-block partial sums, their offsets and coefficients, the
// result) are carved from `ws` (ws_bytes available; nothing is allocated) when
// it is given, else allocated for the call.  Every buffer is written before it
// is read, so `ws` need not be cleared.
static cd expectation_impl(hgf_operator_s* op, const hgf_state_desc* psi, hipStream_t st, void* ws = nullptr,
                           size_t ws_bytes = 0) {
  if (op->sep) {
    if (ws) fail(HGF_EUNSUPPORTED, "separated-layout operators are read through hgf_expectation");
    return separated_expectation(op, psi, st);
  }
  validate_state(op->sys, psi);
  const auto amps = all_amps(op->sys, psi);
  const int nf = (int)op->fn.size();
  if (nf == 0) return 0.0;
  std::vector<int> start(nf + 1, 0);
  std::vector<cd> coef(nf), wall;
  std::vector<int> woff(nf);
  cd analytic = 0.0;
  for (int i = 0; i < nf; ++i) {
    Function& f = op->fn[i];
    const auto w = sector_weights(op->sys, f, amps);
    woff[i] = (int)wall.size();
    wall.insert(wall.end(), w.begin(), w.end());
    start[i + 1] = start[i] + expect_blocks(f.ga);
    coef[i] = f.split ? f.g0 : cd(1.0);
    if (f.split) {  // separable part c_x c_y x^p y^q contracted with psi0
      cd wm = 1.0;
      for (int j = 0; j < op->sys.n; ++j) wm *= w[f.ga.off[j] + std::min(f.p[j], f.q[j])];
      analytic += f.g0 * f.cx * f.cy * wm;
    }
  }
  const size_t b_w = wall.size() * sizeof(double2), b_part = start[nf] * sizeof(double2),
               b_start = (nf + 1) * sizeof(int), b_coef = nf * sizeof(double2), b_out = sizeof(double2);
  double2 *dw, *dpart, *dcoef, *dout;
  int* dstart;
  std::vector<std::unique_ptr<DBuf>> owned;
  if (ws) {
    auto al = [](size_t x) { return (x + 255) & ~(size_t)255; };
    const size_t need = al(b_w) + al(b_part) + al(b_start) + al(b_coef) + al(b_out);
    if (need > ws_bytes)
      fail(HGF_EINVAL, "this expectation needs " + std::to_string(need) + " bytes of device scratch; the static "
                       "scratch holds " + std::to_string(ws_bytes) + " (use hgf_expectation)");
    char* p = (char*)ws;
    dw = (double2*)p;
    p += al(b_w);
    dpart = (double2*)p;
    p += al(b_part);
    dstart = (int*)p;
    p += al(b_start);
    dcoef = (double2*)p;
    p += al(b_coef);
    dout = (double2*)p;
  } else {
    for (size_t b : {b_w, b_part, b_start, b_coef, b_out}) owned.emplace_back(new DBuf(b));
    dw = owned[0]->as<double2>();
    dpart = owned[1]->as<double2>();
    dstart = owned[2]->as<int>();
    dcoef = owned[3]->as<double2>();
    dout = owned[4]->as<double2>();
  }
  hip_check(hipMemcpyAsync(dw, wall.data(), b_w, hipMemcpyHostToDevice, st), "upload");
  hip_check(hipMemcpyAsync(dstart, start.data(), b_start, hipMemcpyHostToDevice, st), "upload");
  hip_check(hipMemcpyAsync(dcoef, coef.data(), b_coef, hipMemcpyHostToDevice, st), "upload");
  for (int i = 0; i < nf; ++i)
    launch_expect_partial(op->fn[i].ga, op->fn[i].y, true, dw + woff[i], dpart + start[i], st, op->fn[i].real);
  launch_expect_final(dpart, dstart, dcoef, nf, make_double2(analytic.real(), analytic.imag()), dout, st);
  hip_check(hipGetLastError(), "kernel launch");
  double2 r;
  hip_check(hipMemcpyAsync(&r, dout, sizeof(double2), hipMemcpyDeviceToHost, st), "download");
  hip_check(hipStreamSynchronize(st), "synchronize");
  return cd(r.x, r.y);
}

// ------------------------------------------------------------------ reconstruction

// Largest output of hgf_reconstruct, in matrix elements.
constexpr int64_t kMaxReconstructElems = (int64_t)1 << 24;

// <k|A|l> for every k, l below `levels` in every mode (Eq. (11)): each
// function's grid points in that box, times sqrt(k! l!), scattered into a
// dense matrix on the device, then copied to `out`.
static void reconstruct_impl(hgf_operator_s* op, int levels, double* out, hipStream_t st) {
  if (op->sep) {
    separated_reconstruct(op, levels, out, st);
    return;
  }
  const int n = op->sys.n;
  int64_t ln = 1;
  for (int j = 0; j < n; ++j) {
    if (levels < 1 || levels > op->sys.nc[j]) fail(HGF_EINVAL, "levels must be in [1, every cutoff]");
    ln *= levels;
    if (ln * ln > kMaxReconstructElems) fail(HGF_EINVAL, "levels^(2N) exceeds 2^24 matrix elements");
  }
  const int64_t elems = ln * ln;
  std::vector<GatherBox> boxes;
  std::vector<int> fidx;
  std::vector<double> fac;
  for (size_t i = 0; i < op->fn.size(); ++i) {
    const Function& f = op->fn[i];
    GatherBox b{};
    b.ln = ln;
    b.total = 1;
    b.pq = -1;
    b.coef = make_double2(1.0, 0.0);
    std::vector<int64_t> place(n);
    {
      int64_t p = ln;
      for (int j = 0; j < n; ++j) place[j] = p /= levels;
    }
    if (f.full) {  // axes k, l of the mode at each position
      for (int a = 0; a < 2 * n; ++a) {
        const int j = f.fperm[a / 2];
        b.rp[a] = a % 2 == 0 ? place[j] : 0;
        b.cp[a] = a % 2 == 0 ? 0 : place[j];
        b.ur[a] = b.uc[a] = 0;
        b.b[a] = levels;
        b.foff[a] = (int)fac.size();
        for (int m = 0; m < levels; ++m) fac.push_back(sqrt_factorial(m));
        b.total *= levels;
      }
    } else {
      for (int j = 0; j < n; ++j) {
        b.rp[j] = b.cp[j] = place[j];
        b.ur[j] = f.tab.u[j];
        b.uc[j] = f.tab.v[j];
        b.b[j] = std::max(0, levels - std::max(b.ur[j], b.uc[j]));
        b.foff[j] = (int)fac.size();
        for (int m = 0; m < b.b[j]; ++m) fac.push_back(sqrt_factorial(m + b.ur[j]) * sqrt_factorial(m + b.uc[j]));
        b.total *= b.b[j];
      }
    }
    if (b.total == 0) continue;
    if (f.split) {  // G = g0 (c_x c_y x^p y^q + R): the separable part sits at m = min(p, q)
      b.coef = make_double2(f.g0.real(), f.g0.imag());
      int64_t gi = 0;
      bool inside = true;
      for (int j = 0; j < n; ++j) {
        const int m = std::min(f.p[j], f.q[j]);
        inside &= m < b.b[j];
        gi += m * f.ga.stride[j];
      }
      if (inside) {
        const cd a = f.cx * f.cy;
        b.pq = gi;
        b.add = make_double2(a.real(), a.imag());
      }
    }
    boxes.push_back(b);
    fidx.push_back((int)i);
  }
  DBuf dout((size_t)elems * sizeof(double2));
  launch_fill_zero(dout.as<double2>(), elems, st);
  if (!boxes.empty()) {
    DBuf dfac(fac.size() * sizeof(double));
    hip_check(hipMemcpyAsync(dfac.p, fac.data(), fac.size() * sizeof(double), hipMemcpyHostToDevice, st), "upload");
    for (size_t k = 0; k < boxes.size(); ++k) {
      const Function& f = op->fn[fidx[k]];
      launch_gather_levels(f.ga, f.y, f.real, boxes[k], dfac.as<double>(), dout.as<double2>(), st);
    }
    hip_check(hipGetLastError(), "kernel launch");
    hip_check(hipMemcpyAsync(out, dout.p, (size_t)elems * sizeof(double2), hipMemcpyDeviceToHost, st), "download");
    hip_check(hipStreamSynchronize(st), "synchronize");  // dfac and dout outlive the launches
  } else {
    hip_check(hipMemcpyAsync(out, dout.p, (size_t)elems * sizeof(double2), hipMemcpyDeviceToHost, st), "download");
    hip_check(hipStreamSynchronize(st), "synchronize");
  }
}

// ------------------------------------------------------------------ gradient

// L^T of a sector's generator as tables of the same stencil form:
// (L^T mu)(m) = lam(m) mu(m) + sum_j [alpha_j(m_j + 1) mu(m + e_j) + beta_j(m_j - 1) mu(m - e_j)],
// i.e. alpha'_j(m) = beta_j(m - 1) (0 at m = 0) and beta'_j(m) = alpha_j(m + 1)
// (0 at the top of the axis): transpose only, no conjugation.
static SectorTables transposed_tables(const SectorTables& t) {
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
// they fit in this many bytes (the reverse sweep then recomputes nothing);
// otherwise, or with HGF_GRAD_STORE=0 in the environment, it keeps the states
// only and recomputes the three stages of each step in the sweep (the same
// numbers either way).
constexpr int64_t kGradStoreBytes = (int64_t)2 << 30;

static void grad_impl(const System& sys, const hgf_operator_desc* desc, const hgf_state_desc* psi, double T,
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
  for (auto& f : op.fn) {
    const int64_t pts = f.ga.points;
    const size_t gb = pts * sizeof(double2);
    const int64_t nseg = (M + ce - 1) / ce;
    const int64_t seg_steps = std::min<int64_t>(ce, std::max<int64_t>(M, 1));
    const char* store_env = std::getenv("HGF_GRAD_STORE");  // "0": keep states only
    const bool store = 4 * seg_steps * (int64_t)gb <= kGradStoreBytes && !(store_env && std::string(store_env) == "0");
    const int64_t per_step = store ? 4 : 1;  // grids kept per step: y (and X1, V1, V2)
    DBuf ckpt((size_t)(nseg + 1) * gb), segbuf((size_t)(seg_steps * per_step) * gb), mu(gb), vb2(gb), vb1(gb),
        xb1(gb), Q((size_t)(1 + 2 * sys.n) * gb), wt(gb);
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
    // value
    {
      std::vector<int> start = {0, expect_blocks(f.ga)};
      cd one = 1.0;
      DBuf dpart(start[1] * sizeof(double2)), dstart(2 * sizeof(int)), dcoef(sizeof(double2)), dout(sizeof(double2));
      hip_check(hipMemcpyAsync(dstart.p, start.data(), 2 * sizeof(int), hipMemcpyHostToDevice, st), "upload");
      hip_check(hipMemcpyAsync(dcoef.p, &one, sizeof(double2), hipMemcpyHostToDevice, st), "upload");
      launch_expect_partial(f.ga, f.y, true, dw.as<double2>(), dpart.as<double2>(), st);
      launch_expect_final(dpart.as<double2>(), dstart.as<int>(), dcoef.as<double2>(), 1, make_double2(0, 0),
                          dout.as<double2>(), st);
      double2 r;
      hip_check(hipMemcpyAsync(&r, dout.p, sizeof(double2), hipMemcpyDeviceToHost, st), "download");
      hip_check(hipStreamSynchronize(st), "synchronize");
      value += cd(r.x, r.y);
    }
    // reverse sweep: mu_M = w
    hip_check(hipMemcpyAsync(mu.p, wt.p, gb, hipMemcpyDeviceToDevice, st), "seed");
    launch_fill_zero(Q.as<double2>(), (int64_t)(1 + 2 * sys.n) * pts, st);
    double2* seg = segbuf.as<double2>();
    double2* Qp = Q.as<double2>();
    // One segment of L steps: recompute y_{s0} .. y_{s0+L-1} from the state in
    // f.y into the segment buffer (with each step's X1, V1, V2 when `store`),
    // then sweep them in reverse.  The work of a segment depends only on L, so
    // it is captured once per length.  The stage launches are those of the
    // forward pass (same kernel, shape and operands), so the recomputed states
    // equal the checkpointed trajectory bit for bit.
    auto slot = [&](int64_t i, int k) { return seg + (i * per_step + k) * pts; };  // k: y, X1, V1, V2
    auto segment = [&](int64_t L, hipStream_t s) {
      for (int64_t i = 0; i < L; ++i) {
        launch_copy2(slot(i, 0), (const double2*)f.y, pts, s);
        if (!store) {
          if (i + 1 < L) run_plan_step(*fplan, op.dflag, s);
          continue;
        }
        stage_launch(f, HGF_FP64, 1, slot(i, 0), nullptr, slot(i, 0), nullptr, slot(i, 1), dt, op.dflag, s);
        stage_launch(f, HGF_FP64, 2, slot(i, 1), slot(i, 1), slot(i, 0), nullptr, slot(i, 2), dt, op.dflag, s);
        stage_launch(f, HGF_FP64, 3, slot(i, 2), slot(i, 1), slot(i, 0), nullptr, slot(i, 3), dt, op.dflag, s);
        if (i + 1 < L)
          stage_launch(f, HGF_FP64, 4, slot(i, 3), slot(i, 1), f.y, nullptr, nullptr, dt, op.dflag, s);
      }
      for (int64_t i = L - 1; i >= 0; --i) {
        double2* yn = slot(i, 0);
        const double2 *x1 = (const double2*)f.s1, *v1 = (const double2*)f.s2, *v2 = (const double2*)f.s3;
        if (store) {
          x1 = slot(i, 1);
          v1 = slot(i, 2);
          v2 = slot(i, 3);
        } else {  // forward stage grids X1, V1, V2 of this step (FP64: s1, s2, s3)
          stage_launch(f, HGF_FP64, 1, yn, nullptr, yn, nullptr, f.s1, dt, op.dflag, s);
          stage_launch(f, HGF_FP64, 2, f.s1, f.s1, yn, nullptr, f.s2, dt, op.dflag, s);
          stage_launch(f, HGF_FP64, 3, f.s2, f.s1, yn, nullptr, f.s3, dt, op.dflag, s);
        }
        double2 *pm = mu.as<double2>(), *pv2 = vb2.as<double2>(), *pv1 = vb1.as<double2>(), *px = xb1.as<double2>();
        // stage-1 form (out = h' L^T in): B1, B2 and B3's stencil part
        stage_launch(fa, HGF_FP64, 1, pm, nullptr, pm, nullptr, pv2, 0.5 * dt, op.dflag, s);
        stage_launch(fa, HGF_FP64, 1, pv2, nullptr, pv2, nullptr, pv1, dt / 3.0, op.dflag, s);
        stage_launch(fa, HGF_FP64, 1, pv1, nullptr, pv1, nullptr, px, 0.25 * dt, op.dflag, s);
        launch_adjoint_q(f.ga, pm, pv2, pv1, px, v2, v1, x1, yn, Qp, dt, s);
        // stage-4 form (y += x1 + (h'/2) L^T in) with x1 = 0, h' = 2h: B4
        stage_launch(fa, HGF_FP64, 4, px, zero.p, pm, nullptr, nullptr, 2.0 * dt, op.dflag, s);
      }
    };
    std::map<int64_t, std::unique_ptr<GraphHolder>> seg_graphs;
    for (int64_t c = nseg - 1; c >= 0; --c) {
      const int64_t s0 = c * ce, L = std::min<int64_t>(ce, M - s0);
      hip_check(hipMemcpyAsync(f.y, ck + c * pts, gb, hipMemcpyDeviceToDevice, st), "restore");
      if (L > kGradGraphSteps) {  // long segments run without a graph
        segment(L, st);
        continue;
      }
      auto it = seg_graphs.find(L);
      if (it == seg_graphs.end()) {
        hip_check(hipStreamSynchronize(st), "synchronize");
        hip_check(hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal), "begin capture");
        segment(L, cap);
        hipGraph_t graph;
        hip_check(hipStreamEndCapture(cap, &graph), "end capture");
        hipGraphExec_t exec;
        hipError_t e = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
        (void)hipGraphDestroy(graph);
        hip_check(e, "graph instantiate");
        it = seg_graphs.emplace(L, std::unique_ptr<GraphHolder>(new GraphHolder(exec))).first;
      }
      hip_check(hipGraphLaunch(it->second->e, st), "graph launch");
    }
    hip_check(hipStreamSynchronize(st), "synchronize");  // graphs are destroyed with seg_graphs
    // leave the function at its initial state
    hip_check(hipMemcpyAsync(f.y, y0.p, gb, hipMemcpyDeviceToDevice, st), "restore");
    // marginals of Q -> parameter derivatives
    const int nb = marginal_bins(f.ga);
    DBuf dbins(nb * sizeof(double2));
    launch_marginals(f.ga, Q.as<double2>(), dbins.as<double2>(), st);
    hip_check(hipGetLastError(), "kernel launch");
    std::vector<cd> bins(nb);
    hip_check(hipMemcpyAsync(bins.data(), dbins.p, nb * sizeof(double2), hipMemcpyDeviceToHost, st), "download");
    hip_check(hipStreamSynchronize(st), "synchronize");
    int tot_e = 0;
    for (int j = 0; j < sys.n; ++j) tot_e += f.ga.ext[j];
    cd S0 = 0.0;
    for (int v = 0; v < f.ga.ext[0]; ++v) S0 += bins[v];
    for (int p = 0; p < P; ++p) {
      const System u = unit_system(sys, p);
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
  if (read_flag(&op, st)) fail(HGF_ENONFINITE, "non-finite value during the gradient sweep");
  value_out[0] = value.real();
  value_out[1] = value.imag();
  for (int p = 0; p < P; ++p) {
    grad_out[2 * p] = grad[p].real();
    grad_out[2 * p + 1] = grad[p].imag();
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
    for (auto& f : op->fn) ok = ok && f.full;
    if (!ok)
      fail(HGF_EUNSUPPORTED, "thresholded storage applies to FP64 network operators on the full grid and to the "
                             "separated layouts");
    hip_check(hipSetDevice(op->device), "hipSetDevice");
    if (!op->dcount) op->dcount = (unsigned long long*)dmalloc(2 * sizeof(unsigned long long));
    hip_check(hipMemset(op->dcount, 0, 2 * sizeof(unsigned long long)), "clear counters");
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
    info->stored_peak = -1;
    if (op->threshold > 0.0 && op->dcount) {
      unsigned long long peak = 0;
      hip_check(hipSetDevice(op->device), "hipSetDevice");
      hip_check(hipMemcpy(&peak, op->dcount + 1, sizeof(peak), hipMemcpyDeviceToHost), "download");
      info->stored_peak = (int64_t)peak;
    }
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
      out->threads = ft ? f.ga.fthreads : 0;
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
      if (cfg->xblock != 0 || cfg->pipe != 0 || cfg->resident != 0 || (cfg->nfast != 0 && cfg->nfast != 4))
        fail(HGF_EINVAL, "a network operator takes nfast 0 (untiled) or 4 (tiles of its last two modes), "
                         "without xblock, pipe or the resident form");
      if (cfg->nfast == 0)
        drop_full_tiles(f);
      else if (!configure_full_tiles(f, f.fhost.at(0), op->precision, c))
        fail(HGF_EINVAL, "tile configuration not feasible for this network grid");
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
        fail(HGF_EINVAL, "the resident form needs the whole grid in one tile of at most 4096 points "
                         "(and threads, if set, a multiple of 64 covering it in at most 4 lane rounds)");
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
