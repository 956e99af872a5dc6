// Host side of the separated layout (Eqs. (9a)-(9c)): one pair of grids
// Gx(x), Gy(y) over the N occupations per non-negligible initial
// coefficient g_{p,q}(0) (Eq. (10): Gx(0) = x^p, Gy(0) = y^q), with the
// separation constant C = -(i/2)(E(p) + E(q)) of Eq. (20) (for the
// Hamiltonian of the system: E is its energy of a number state), and one R
// holding the sum over the monomials of g_{p,q}(0) R_{p,q}, on the diagonal
// k = l (HGF_SEPARATED) or on the whole box (HGF_SEPARATED_EXACT).  The
// operator at time t is G = sum_i g_i Gx_i Gy_i + R (Eq. (11) summed over the
// monomials).  Classical RK4 on the joint state, FP64; kernels in
// hgf_separated.hip.
#include <hip/hip_runtime.h>

#include <cmath>
#include <string>
#include <vector>

#include "hgf_host.h"
#include "hgf_kernels.h"

namespace hgf {

struct SepState {
  int rmode = 1;  // 1: R on the diagonal; 0: R on the whole (k, l) box
  SepLaunch L{};
  std::vector<Coeff> monos;
  void* dft = nullptr;    // FullTables
  void* dcst = nullptr;   // +C_i (x side), then -C_i (y side): 2M complex
  void* dcoef = nullptr;  // g_i: M complex
  void* dpt = nullptr;    // per-point table of the N-mode box (SepPoint)
  void* x[4] = {};        // u, acc, ya, yb of the 2M grids (each 2M D complex)
  void* r[4] = {};        // u, acc, ya, yb of R (D or D^2 complex)
  void* src = nullptr;    // the source P-operand sum_i g_i Gx_i Gy_i (diagonal or whole box)
  void* xbak = nullptr;   // state copies for recovery after a non-finite result
  void* rbak = nullptr;
  double bound = 0.0;
  int64_t rlen = 0;
};

static int64_t flat_of(const std::vector<int>& k, const SepDims& d) {
  int64_t f = 0;
  for (int j = 0; j < d.n; ++j) f += k[j] * d.stride[j];
  return f;
}

void build_separated(hgf_operator_s* op, const hgf_operator_desc* desc) {
  const System& s = op->sys;
  if (op->precision != HGF_FP64) fail(HGF_EUNSUPPORTED, "the separated layouts run in FP64");
  if (s.n > kMaxFullModes) fail(HGF_EINVAL, "the separated layouts take at most 8 modes");
  auto* st = new SepState;
  op->sep = st;
  st->rmode = op->layout == HGF_SEPARATED ? 1 : 0;
  SepDims& d = st->L.d;
  d.n = s.n;
  d.dim = 1;
  for (int j = s.n - 1; j >= 0; --j) {
    d.stride[j] = d.dim;
    d.dim *= s.nc[j];
  }
  if (st->rmode == 0 && d.dim * d.dim > kMaxFullPoints)
    fail(HGF_EINVAL, "R on the whole (k, l) box exceeds 2^28 points; use HGF_SEPARATED");
  std::map<std::vector<int>, std::vector<cd>> unused;
  std::vector<Coeff> all;
  collect_coeffs(s, desc, unused, all, true);
  for (auto& c : all)
    if (std::abs(c.v) > desc->drop_tol) st->monos.push_back(c);
  const int64_t M = (int64_t)st->monos.size();
  if (2 * M * d.dim > ((int64_t)1 << 31)) fail(HGF_EINVAL, "the monomials' grids exceed 2^31 points");
  d.nmono = (int)M;
  FullTables ft = full_tables(s);
  st->bound = full_generator_bound(ft);
  st->dft = dmalloc(sizeof(FullTables));
  hip_check(hipMemcpy(st->dft, &ft, sizeof(FullTables), hipMemcpyHostToDevice), "upload tables");
  st->L.ft = (const FullTables*)st->dft;
  // per-point table of the N-mode box: occupations, damping and dephasing
  // sums, energy (in the order the stencils would form them)
  {
    std::vector<SepPoint> pts((size_t)d.dim);
    std::vector<int> k(s.n, 0);
    for (int64_t f = 0; f < d.dim; ++f) {
      int64_t r = f;
      for (int j = s.n - 1; j >= 0; --j) {
        k[j] = (int)(r % s.nc[j]);
        r /= s.nc[j];
      }
      SepPoint q{};
      for (int j = 0; j < s.n; ++j) {
        q.coords |= (uint64_t)k[j] << (5 * j);
        q.dks += ft.dk[j][k[j]];
        q.g2 += ft.gphi[j] * (double)(k[j] * k[j]);
        q.energy += ft.e[j][k[j]];
        for (int i = 0; i < j; ++i) q.energy += ft.chi[i][j] * (double)(k[i] * k[j]);
      }
      pts[(size_t)f] = q;
    }
    st->dpt = dmalloc(pts.size() * sizeof(SepPoint));
    hip_check(hipMemcpy(st->dpt, pts.data(), pts.size() * sizeof(SepPoint), hipMemcpyHostToDevice), "upload");
    st->L.pt = (const SepPoint*)st->dpt;
  }
  // separation constants and coefficients
  auto energy = [&](const std::vector<int>& k) {
    double e = 0.0;
    for (int j = 0; j < s.n; ++j) {
      e += ft.e[j][k[j]];
      for (int i = 0; i < j; ++i) e += ft.chi[i][j] * (double)(k[i] * k[j]);
    }
    return e;
  };
  std::vector<cd> cst(2 * M + 1), coef(M + 1);
  std::vector<int64_t> ones;
  for (int64_t i = 0; i < M; ++i) {
    const Coeff& c = st->monos[i];
    const cd C = cd(0.0, -0.5) * (energy(c.k) + energy(c.l));
    cst[i] = C;
    cst[M + i] = -C;
    coef[i] = c.v;
    ones.push_back(i * d.dim + flat_of(c.k, d));
    ones.push_back((M + i) * d.dim + flat_of(c.l, d));
  }
  st->dcst = dmalloc(cst.size() * sizeof(double2));
  st->dcoef = dmalloc(coef.size() * sizeof(double2));
  hip_check(hipMemcpy(st->dcst, cst.data(), cst.size() * sizeof(double2), hipMemcpyHostToDevice), "upload");
  hip_check(hipMemcpy(st->dcoef, coef.data(), coef.size() * sizeof(double2), hipMemcpyHostToDevice), "upload");
  const size_t xb = (size_t)std::max<int64_t>(2 * M * d.dim, 1) * sizeof(double2);
  st->rlen = st->rmode == 1 ? d.dim : d.dim * d.dim;
  const size_t rb = (size_t)st->rlen * sizeof(double2);
  for (int b = 0; b < 4; ++b) {
    st->x[b] = dmalloc(xb);
    st->r[b] = dmalloc(rb);
  }
  st->src = dmalloc(rb);
  hip_check(hipMemset(st->x[0], 0, xb), "clear");
  hip_check(hipMemset(st->r[0], 0, rb), "clear");
  if (!ones.empty()) {
    DBuf didx(ones.size() * sizeof(int64_t));
    hip_check(hipMemcpy(didx.p, ones.data(), ones.size() * sizeof(int64_t), hipMemcpyHostToDevice), "upload");
    launch_sep_ones((int64_t)ones.size(), didx.as<int64_t>(), (double2*)st->x[0], nullptr);
    hip_check(hipGetLastError(), "kernel launch");
    hip_check(hipDeviceSynchronize(), "synchronize");
  }
}

void free_separated(hgf_operator_s* op) {
  SepState* st = op->sep;
  if (!st) return;
  for (int b = 0; b < 4; ++b) {
    dfree(st->x[b]);
    dfree(st->r[b]);
  }
  dfree(st->src);
  dfree(st->xbak);
  dfree(st->rbak);
  dfree(st->dft);
  dfree(st->dcst);
  dfree(st->dcoef);
  dfree(st->dpt);
  delete st;
  op->sep = nullptr;
}

int64_t separated_points(const hgf_operator_s* op) {
  const SepState* st = op->sep;
  return 2 * (int64_t)st->L.d.nmono * st->L.d.dim + st->rlen;
}

int separated_functions(const hgf_operator_s* op) { return 2 * op->sep->L.d.nmono + 1; }

int64_t separated_tile_points(const hgf_operator_s* op) { return op->sep->L.d.dim; }

void separated_evolve(hgf_operator_s* op, int64_t steps, double h, hipStream_t strm) {
  SepState* st = op->sep;
  const SepDims& d = st->L.d;
  if (h * st->bound > 2.5)
    fail(HGF_EUNSTABLE, "dt * spectral bound = " + std::to_string(h * st->bound) +
                            " exceeds the RK4 stability limit 2.5; reduce dt");
  if (steps == 0) return;
  const size_t xb = (size_t)std::max<int64_t>(2 * (int64_t)d.nmono * d.dim, 1) * sizeof(double2);
  const size_t rb = (size_t)st->rlen * sizeof(double2);
  if (!st->xbak) st->xbak = dmalloc(xb);
  if (!st->rbak) st->rbak = dmalloc(rb);
  hip_check(hipMemcpyAsync(st->xbak, st->x[0], xb, hipMemcpyDeviceToDevice, strm), "backup");
  hip_check(hipMemcpyAsync(st->rbak, st->r[0], rb, hipMemcpyDeviceToDevice, strm), "backup");
  reset_flag(op, strm);
  double2* X[4];
  double2* R[4];
  for (int b = 0; b < 4; ++b) {
    X[b] = (double2*)st->x[b];
    R[b] = (double2*)st->r[b];
  }
  // stage inputs and outputs (u, acc, ya, yb = 0, 1, 2, 3): stage 1 reads u
  // and writes ya, 2 reads ya and writes yb, 3 reads yb and writes ya, 4
  // reads ya and writes u
  static const int in_of[5] = {0, 0, 2, 3, 2}, out_of[5] = {0, 2, 3, 2, 2};
  for (int64_t k = 0; k < steps; ++k)
    for (int s = 1; s <= 4; ++s) {
      if (d.nmono > 0) launch_sep_source(st->L, st->rmode, (const double2*)st->dcoef, X[in_of[s]], (double2*)st->src,
                                          strm);
      else hip_check(hipMemsetAsync(st->src, 0, rb, strm), "clear");
      launch_sep_r(st->L, st->rmode, s, h, (const double2*)st->src, R[0], R[1], R[in_of[s]], R[out_of[s]], op->dflag,
                   strm);
      if (d.nmono > 0)
        launch_sep_sides(st->L, s, h, (const double2*)st->dcst, X[0], X[1], X[in_of[s]], X[out_of[s]], op->dflag,
                         strm);
      if (s == 4 && op->threshold > 0.0) {  // thresholded representation of every grid
        // tiles: one grid of D points (each Gx_i, Gy_i; R per row of D)
        launch_threshold(X[0], 2 * (int64_t)d.nmono * d.dim, op->threshold, d.dim, op->dcount, strm);
        launch_threshold(R[0], st->rlen, op->threshold, d.dim, op->dcount, strm);
        launch_threshold_peak(op->dcount, strm);
      }
    }
  hip_check(hipGetLastError(), "kernel launch");
  if (read_flag(op, strm)) {
    hip_check(hipMemcpyAsync(st->x[0], st->xbak, xb, hipMemcpyDeviceToDevice, strm), "restore");
    hip_check(hipMemcpyAsync(st->r[0], st->rbak, rb, hipMemcpyDeviceToDevice, strm), "restore");
    hip_check(hipStreamSynchronize(strm), "synchronize");
    op->error_state = 1;
    fail(HGF_ENONFINITE, "non-finite value in an evolved function; state restored to the start of this call");
  }
}

cd separated_expectation(hgf_operator_s* op, const hgf_state_desc* psi, hipStream_t strm) {
  SepState* st = op->sep;
  const System& s = op->sys;
  validate_state(s, psi);
  const auto amps = all_amps(s, psi);
  // per-mode weights: sqrt(k!) conj(c_j(k)) (x side), sqrt(l!) c_j(l) (y side)
  std::vector<cd> wt((size_t)2 * kMaxFullModes * kMaxCutoff, 0.0);
  for (int j = 0; j < s.n; ++j)
    for (int k = 0; k < s.nc[j]; ++k) {
      wt[(size_t)(2 * j) * kMaxCutoff + k] = sqrt_factorial(k) * std::conj(amps[j][k]);
      wt[(size_t)(2 * j + 1) * kMaxCutoff + k] = sqrt_factorial(k) * amps[j][k];
    }
  const int np = sep_expect_parts(st->L.d);
  DBuf dwt(wt.size() * sizeof(double2)), dpart((size_t)np * sizeof(double2)), dout(sizeof(double2));
  hip_check(hipMemcpyAsync(dwt.p, wt.data(), wt.size() * sizeof(double2), hipMemcpyHostToDevice, strm), "upload");
  launch_sep_expect(st->L, st->rmode, dwt.as<double2>(), (const double2*)st->dcoef, (const double2*)st->x[0],
                    (const double2*)st->r[0], dpart.as<double2>(), dout.as<double2>(), strm);
  hip_check(hipGetLastError(), "kernel launch");
  double2 v;
  hip_check(hipMemcpyAsync(&v, dout.p, sizeof(double2), hipMemcpyDeviceToHost, strm), "download");
  hip_check(hipStreamSynchronize(strm), "synchronize");
  return cd(v.x, v.y);
}

void separated_reconstruct(hgf_operator_s* op, int levels, double* out, hipStream_t strm) {
  SepState* st = op->sep;
  const System& s = op->sys;
  int64_t ln = 1;
  for (int j = 0; j < s.n; ++j) {
    if (levels < 1 || levels > s.nc[j]) fail(HGF_EINVAL, "levels must be in [1, every cutoff]");
    ln *= levels;
    if (ln * ln > ((int64_t)1 << 24)) fail(HGF_EINVAL, "levels^(2N) exceeds 2^24 matrix elements");
  }
  std::vector<double> fac((size_t)kMaxFullModes * kMaxCutoff, 0.0);
  for (int j = 0; j < s.n; ++j)
    for (int k = 0; k < s.nc[j]; ++k) fac[(size_t)j * kMaxCutoff + k] = sqrt_factorial(k);
  DBuf dfac(fac.size() * sizeof(double)), dout((size_t)(ln * ln) * sizeof(double2));
  hip_check(hipMemcpyAsync(dfac.p, fac.data(), fac.size() * sizeof(double), hipMemcpyHostToDevice, strm), "upload");
  launch_sep_gather(st->L, st->rmode, levels, ln, dfac.as<double>(), (const double2*)st->dcoef,
                    (const double2*)st->x[0], (const double2*)st->r[0], dout.as<double2>(), strm);
  hip_check(hipGetLastError(), "kernel launch");
  hip_check(hipMemcpyAsync(out, dout.p, (size_t)(ln * ln) * sizeof(double2), hipMemcpyDeviceToHost, strm),
            "download");
  hip_check(hipStreamSynchronize(strm), "synchronize");
}

}  // namespace hgf
