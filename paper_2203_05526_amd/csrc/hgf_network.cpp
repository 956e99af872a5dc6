// Network operators (drive and exchange, Eq. (16)): the generator tables of
// the full (k, l) grid, the order of the modes on it, the per-tile records and
// launch configuration of its tiled stage kernel, and the map of the operator
// onto the grid.
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
std::vector<char> full_tile_records(const GridArgs& g, const FullTables& ft, int& rec_bytes) {
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
bool configure_full_tiles(Function& f, const FullTables& ft, int precision, const TileChoice& c) {
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
void drop_full_tiles(Function& f) {
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
void full_mode_order(const System& s, int* perm) {
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
System permute_modes(const System& s, const int* perm) {
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
void build_full_function(hgf_operator_s* op, const hgf_operator_desc* d) {
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
  // small untiled grids: the resident integrator (HGF_RESIDENT=0 turns it off)
  const char* env = std::getenv("HGF_RESIDENT");
  if (!stage_kernel_generic() && f.ga.fblocks == 0 && !(env && std::string(env) == "0"))
    f.resident = full_resident_eligible(f, op->precision);
  alloc_function_buffers(f, op->precision);
  upload_state(f, grid, op->precision);
}

// A network operator runs on the resident integrator when its whole grid fits
// twice in 64 KB of LDS (in the stage precision) and it has at most three
// modes (the kernel's instantiations).
bool full_resident_eligible(Function& f, int precision) {
  const int64_t T = f.ga.points, ts = precision == HGF_FP64 ? 16 : 8;
  if (!f.full || f.ga.n / 2 > 3 || 2 * T * ts > 65536) return false;
  f.res_lds_bytes = (int)(2 * T * ts);
  f.res_threads = (int)std::min<int64_t>(1024, (T + 63) / 64 * 64);
  return true;
}

}  // namespace hgf
