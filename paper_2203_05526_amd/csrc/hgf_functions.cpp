// Operator -> functions (step (i) of the method): the tiled stage kernel's launch
// configuration and tile records, the grid arguments, the coefficient map of
// Eqs. (2), (6)-(8) into sector grids or split monomials (network operators:
// hgf_network.cpp).
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

// ------------------------------------------------------------------ functions

// HGF_STAGE_KERNEL=generic selects the untiled stage kernel for every grid.
bool stage_kernel_generic() {
  const char* env = std::getenv("HGF_STAGE_KERNEL");
  return env && std::string(env) == "generic";
}

// HGF_MAX_NFAST below the axis count asks small grids to run the tiled kernel
// with slow axes, so it also keeps them off the resident form by default.
static bool nfast_capped_below(int n) {
  const char* env = std::getenv("HGF_MAX_NFAST");
  return env && std::atoi(env) >= 1 && std::atoi(env) < n;
}


// Configure the tiled stage kernel for grid g.  Default rule: the largest
// number nfast <= 4 of trailing axes whose padded tile and tables fit in 64 KB
// of LDS; 256 lanes when they cover the tile in at most kTileRounds rounds (the
// fastest shape measured on the 6^10 grid), else the smallest multiple of 64
// that does; contiguous XCD order; no pipelining.  Returns false (and sets
// g.blocks = 0, the generic kernel) when the request cannot be met.
bool configure_tiles(GridArgs& g, int precision, bool real, const TileChoice& c) {
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
std::vector<uint32_t> walk_order(const GridArgs& g) {
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
void* upload_tile_records(GridArgs& g, const SectorTables& t, int precision) {
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

void build_tile_records(Function& f, int precision) { f.ttab = upload_tile_records(f.ga, f.tab, precision); }

// A function runs on the resident kernel when it has at most four axes, its
// points fit the kernel's lane rounds (4096 in mixed precision, 2048 on real
// and 2560 on complex FP64 grids)
// and two padded copies of the whole grid (the tiled kernel's layout with
// every axis in the tile) fit in the CU's LDS; its layout is kept in f.rga,
// beside the stage kernels' (f.ga), which other calls use.  `threads` > 0 asks
// for that workgroup size (a multiple of 64 that covers the grid in the
// kernel's lane rounds), else the fewest rounds with lanes spread evenly.
bool resident_eligible(Function& f, int threads) {
  const GridArgs& g = f.ga;
  if (f.split || f.full || g.n > 4) return false;
  const int max_threads = f.precision_fp64 ? 512 : 1024;  // the kernel's workgroup limit
  const int max_rounds = resident_max_rounds(f.precision_fp64, g.real != 0);
  if (g.points > (int64_t)max_rounds * max_threads) return false;
  GridArgs r = g;
  int64_t padded = 1, pst = 1;
  for (int q = 0; q < g.n; ++q) padded *= q == 0 ? g.ext[q] + 2 : g.ext[q] + 1;
  for (int q = g.n - 1; q >= 0; --q) {
    r.pstride[q] = (int)pst;
    pst *= g.ext[q] + 1;
  }
  r.nfast = g.n;
  r.tile_points = g.points;
  r.ntiles = 1;
  r.lds_elems = (int)padded;
  r.tiles = nullptr;  // the stage kernels' records (replaced by a later retile) are not its
  r.walk = nullptr;
  const int rs = f.precision_fp64 ? 8 : 4, es = (g.real ? 1 : 2) * rs;
  const int64_t lds = 2 * padded * es;
  if (lds > kResidentLdsMax) return false;
  // (the kernels' limit goes to the maximum at once, so that it never drops
  // below what another resident function of the same types needs)
  if (lds > 65536 &&
      resident_allow_lds(g.real != 0, f.precision_fp64 ? HGF_FP64 : HGF_MIXED, kResidentLdsMax) != hipSuccess) {
    (void)hipGetLastError();
    return false;
  }
  if (threads > 0 &&
      (threads % 64 != 0 || threads > max_threads ||
       (g.points + threads - 1) / threads > max_rounds))
    return false;
  f.rga = r;
  f.res_lds_bytes = (int)lds;
  if (threads > 0) {
    f.res_threads = threads;
    return true;
  }
  // lanes: enough for the fewest rounds, spread evenly over them
  const int64_t rounds = (g.points + max_threads - 1) / max_threads;
  const int64_t per = (g.points + rounds - 1) / rounds;
  f.res_threads = (int)std::min<int64_t>(max_threads, std::max<int64_t>(64, (per + 63) / 64 * 64));
  return true;
}

void fill_grid_args(Function& f, int precision, bool want_real) {
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
  f.resident = !stage_kernel_generic() && !nfast_capped_below(g.n) && resident_eligible(f);
  const char* env = std::getenv("HGF_RESIDENT");
  if (env && std::string(env) == "0") f.resident = false;
}

size_t state_bytes(const Function& f) { return f.ga.points * (f.real ? sizeof(double) : sizeof(double2)); }

void alloc_function_buffers(Function& f, int precision) {
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

void free_function(Function& f) {
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

int64_t flat_index(const SectorTables& t, const int* m) {
  int64_t idx = 0;
  for (int j = 0; j < t.n; ++j) idx = idx * t.ext[j] + m[j];
  return idx;
}

// Per-mode g-matrix from the per-mode input matrix (Eqs. (6)-(8), r = 1).
std::vector<cd> mode_g(const double* vals, int nc, int basis) {
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
void precheck_operator_size(const System& s, const hgf_operator_desc* d) {
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

void upload_state(Function& f, const std::vector<cd>& grid, int precision) {
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
double energy(const System& s, const int* k) {
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
void setup_split(Function& f, const System& s, const Coeff& c) {
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


void build_functions(hgf_operator_s* op, const hgf_operator_desc* d, bool allow_real) {
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

}  // namespace hgf
