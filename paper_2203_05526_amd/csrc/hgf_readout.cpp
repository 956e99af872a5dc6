// Readout (step (iii)): expectation values in a product state (Eq. (11)
// contracted with the state) and the operator on the lowest levels.
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

// ------------------------------------------------------------------ expectation

std::vector<cd> mode_amps(const hgf_state_desc* psi, int j, int nc, size_t amp_off) {
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
std::vector<cd> sector_weights(const System& s, const Function& f, const std::vector<std::vector<cd>>& amps) {
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
cd expectation_impl(hgf_operator_s* op, const hgf_state_desc* psi, hipStream_t st, void* ws,
                           size_t ws_bytes) {
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
void reconstruct_impl(hgf_operator_s* op, int levels, double* out, hipStream_t st) {
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

}  // namespace hgf
