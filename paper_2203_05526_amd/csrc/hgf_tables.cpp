// Host-side coefficient tables of the transformed generating-function
// equations, restricted to one occupation-difference sector.
//
// With o1 = a^+, o2 = a (r = 1), G = e^{sum x_j y_j} F (Eq. (5)) and
// coefficients g_{k,l} = <k|A|l>/sqrt(k! l!) (Eqs. (6)-(8)), the adjoint
// master equation (Eq. (3)) for the Kerr network with emission, absorption
// and dephasing becomes, coefficient by coefficient (the multimode Eq. (17)
// generalised to cross-Kerr, a thermal bath and dephasing; at n_th = 0 and no
// dephasing the jump part is the (kappa/2)(2P - x d_x - y d_y) form of the
// supplement's dissipator equation):
//   dg_{k,l}/dt = lambda(k,l) g_{k,l}
//               + sum_j gamma1_j (1 + n_th_j)               g_{k-e_j, l-e_j}
//               + sum_j gamma1_j n_th_j (k_j + 1)(l_j + 1)   g_{k+e_j, l+e_j}
//   lambda(k,l) = i (E(k) - E(l))
//               - sum_j [ gamma1_j (1+n_th_j)(k_j+l_j)/2 + gamma1_j n_th_j (kt_j+lt_j)/2
//                         + gamma_phi_j (k_j - l_j)^2 ]
// with kt = (k+1) below the top level and 0 at it (truncated a a^+).
// Inside the sector l = k + d, write k = m + u, l = m + v with u = max(0,-d),
// v = max(0,d).  The Kerr and cross-Kerr energy differences are then affine
// in m, so lambda = lam0 + sum_j lam_j(m_j):
//   lam_j(m) = -i m (K_j d_j + sum_{i!=j} chi_ij d_i)
//              - gamma1_j (1+n_th_j)(k+l)/2 - gamma1_j n_th_j (kt+lt)/2
//   lam0     = -i sum_j [Delta_j d_j + (K_j/2) d_j (|d_j| - 1)]
//              + i sum_{i<j} chi_ij (u_i u_j - v_i v_j) - sum_j gamma_phi_j d_j^2
// Secular form (Eq. (15) with the transition occupations of the supplement's
// derivation, per mode): with out(n) = gamma1 [n (nbar_{n-1} + 1) + (n+1) nbar_n]
// the total rate out of level n (terms beyond the cutoff dropped),
//   lam_j(m) = -i m (...) - (out(k) + out(l)) / 2
//   alpha_j(m) = gamma1 (nbar_{m-1} + 1),  beta_j(m) = gamma1 nbar_m (m+1)^2   if d_j = 0
//   alpha_j = beta_j = 0                                                        if d_j != 0
// (jumps of mode j only act on its populations; in coefficients g the
// population jump A[m-1,m-1] -> A[m,m] at rate gamma1 m (nbar_{m-1}+1) becomes
// gamma1 (nbar_{m-1}+1) g(m-1), since g(m) = A[m,m] / m!).  With one nbar for
// every transition these reduce to the Lindblad values on d_j = 0.
#include <cmath>
#include <cstring>

#include "hgf_internal.h"

namespace hgf {

int num_params(int n) { return n + n * (n - 1) / 2 + 3 * n; }

SectorTables sector_tables(const System& s, const int* d) {
  SectorTables t;
  t.n = s.n;
  const cd I(0.0, 1.0);
  cd lam0 = 0.0;
  for (int j = 0; j < s.n; ++j) {
    t.d[j] = d[j];
    t.u[j] = d[j] < 0 ? -d[j] : 0;
    t.v[j] = d[j] > 0 ? d[j] : 0;
    t.ext[j] = s.nc[j] - std::abs(d[j]);
    const int dj = d[j];
    lam0 += -I * (s.det[j] * dj + 0.5 * s.kerr[j] * dj * (std::abs(dj) - 1)) - s.gphi[j] * double(dj * dj);
  }
  for (int i = 0; i < s.n; ++i)
    for (int j = i + 1; j < s.n; ++j) lam0 += I * s.chi[i][j] * double(t.u[i] * t.u[j] - t.v[i] * t.v[j]);
  t.lam0 = lam0;
  for (int j = 0; j < s.n; ++j) {
    double phase = s.kerr[j] * d[j];
    for (int i = 0; i < s.n; ++i)
      if (i != j) phase += s.chi[i][j] * d[i];
    const int nc = s.nc[j];
    t.lam[j].resize(t.ext[j]);
    t.beta[j].resize(t.ext[j]);
    t.alpha[j].resize(t.ext[j]);
    if (!s.secular) {
      const double down = s.g1[j] * (1.0 + s.nth[j]);
      const double up = s.g1[j] * s.nth[j];
      for (int m = 0; m < t.ext[j]; ++m) {
        const int k = m + t.u[j], l = m + t.v[j];
        const double kt = (k + 1 < nc) ? k + 1 : 0, lt = (l + 1 < nc) ? l + 1 : 0;
        t.lam[j][m] = -I * (double(m) * phase) - 0.5 * down * (k + l) - 0.5 * up * (kt + lt);
        t.beta[j][m] = (m + 1 < t.ext[j]) ? up * double(k + 1) * double(l + 1) : 0.0;
        t.alpha[j][m] = (m >= 1) ? down : 0.0;
      }
    } else {
      const double* nb = s.nlev[j];
      const double g = s.g1[j];
      auto out = [&](int n) {
        double r = 0.0;
        if (n >= 1) r += g * n * (nb[n - 1] + 1.0);
        if (n + 1 < nc) r += g * (n + 1) * nb[n];
        return r;
      };
      for (int m = 0; m < t.ext[j]; ++m) {
        const int k = m + t.u[j], l = m + t.v[j];
        t.lam[j][m] = -I * (double(m) * phase) - 0.5 * (out(k) + out(l));
        const bool pop = d[j] == 0;
        t.beta[j][m] = (pop && m + 1 < t.ext[j]) ? g * nb[m] * double(m + 1) * double(m + 1) : 0.0;
        t.alpha[j][m] = (pop && m >= 1) ? g * (nb[m - 1] + 1.0) : 0.0;
      }
    }
  }
  return t;
}

System unit_system(const System& s, int p) {
  System u = s;
  std::memset(u.det, 0, sizeof(u.det));
  std::memset(u.kerr, 0, sizeof(u.kerr));
  std::memset(u.chi, 0, sizeof(u.chi));
  std::memset(u.g1, 0, sizeof(u.g1));
  std::memset(u.gphi, 0, sizeof(u.gphi));
  const int n = s.n;
  if (p < n) {
    u.kerr[p] = 1.0;
    return u;
  }
  p -= n;
  const int npair = n * (n - 1) / 2;
  if (p < npair) {
    int q = 0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j, ++q)
        if (q == p) u.chi[i][j] = u.chi[j][i] = 1.0;
    return u;
  }
  p -= npair;
  if (p < n) {
    u.det[p] = 1.0;
    return u;
  }
  p -= n;
  if (p < n) {
    u.g1[p] = 1.0;
    return u;
  }
  p -= n;
  u.gphi[p] = 1.0;
  return u;
}

double generator_bound(const SectorTables& t) {
  double b = std::abs(t.lam0);
  for (int j = 0; j < t.n; ++j) {
    double mx = 0.0;
    for (int m = 0; m < t.ext[j]; ++m) {
      double v = std::abs(t.lam[j][m]) + t.beta[j][m] + t.alpha[j][m];
      if (v > mx) mx = v;
    }
    b += mx;
  }
  return b;
}

}  // namespace hgf
