/*
 * Plain FP64 CPU oracle: the adjoint (Heisenberg-picture) Lindblad master
 * equation of damped, Kerr-coupled bosonic modes, written directly in the
 * truncated number basis and integrated with classical fourth-order
 * Runge-Kutta.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing in the product library links, loads or
 * calls this file; only the tests, the smoke check and the benchmark's CPU
 * baseline do.  It shares no code with the HIP path.
 *
 * What it computes (paper: adjoint master equation, Eq. (3)):
 *   dA/dt = i[H, A] + sum_n (kappa_n/2) (2 L_n^+ A L_n - {L_n^+ L_n, A})
 * with
 *   H = sum_j [Delta_j n_j + (K_j/2) a_j^+ a_j^+ a_j a_j] + sum_{i<j} chi_ij n_i n_j
 * and, for every mode j, three channels
 *   L = a_j    with kappa = gamma1_j (1 + nth_j)      (emission into the bath)
 *   L = a_j^+  with kappa = gamma1_j nth_j            (absorption from the bath)
 *   L = n_j    with kappa = 2 gamma_phi_j             (pure dephasing)
 * The ladder operators are the truncated matrices on span{|0>,...,|Nc_j-1>}
 * (a|0> = 0 and a^+|Nc-1> = 0).
 *
 * Storage.  An operator is held by "difference sectors": for a fixed integer
 * vector d, the sector holds the elements A[k, l] with l = k + d, stored as a
 * row-major array over the whole box k in prod_j [0, Nc_j) with the last mode
 * varying fastest; entries whose l falls outside the box are kept at zero.
 * The equation above maps each sector onto itself (every term moves k and l
 * together), which is why a sector can be evolved on its own; the full
 * operator is the set of all sectors.
 *
 * Secular variant (the first-principles dissipator of Eq. (15), in the form
 * of the supplement's derivation): the emission and absorption channels of
 * mode j are replaced by one channel per transition n <-> n+1 of that mode,
 *   down: |n><n+1|  at rate gamma1_j (n+1) (nbar_{j,n} + 1)
 *   up:   |n+1><n|  at rate gamma1_j (n+1) nbar_{j,n}
 * with nbar_{j,n} the bath occupation at the transition's frequency (given per
 * transition, or n_th_j for every transition).  In the Heisenberg picture a
 * jump maps A to L^+ A L, which is non-zero only where k_j = l_j (populations
 * of mode j), and the anticommutator damps A[k,l] by half the total rate out of
 * level k_j plus that out of level l_j.  Pure dephasing keeps its Lindblad form.
 *
 * Full-matrix form (the driven, exchange-coupled network of Eq. (16)): a drive
 * Omega_j a_j^+ + conj(Omega_j) a_j per mode (static in the frame rotating at
 * the drive frequency) and exchange J_ij (a_i^+ a_j + a_j^+ a_i) couple the
 * difference sectors, so these systems are held as one dense matrix A[k, l]
 * (row and column indices row-major over the modes, last mode fastest) and
 * the commutator with the added terms is written out element by element.
 *
 * Parameter order for sensitivities: K[N], chi[i<j lexicographic], Delta[N],
 * gamma1[N], gamma_phi[N].
 */
#include <complex.h>
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

#define OMAXN 16
#define OMAXC 64

typedef double complex cplx;

typedef struct {
  int n;
  int nc[OMAXN];
  double det[OMAXN], kerr[OMAXN], chi[OMAXN * OMAXN];
  double g1[OMAXN], gphi[OMAXN], nth[OMAXN];
  int secular;               /* 0: Lindblad channels a, a^+; 1: secular transitions */
  double nlev[OMAXN][OMAXC]; /* secular: bath occupation of transition n <-> n+1 of mode j */
  cplx drive[OMAXN];         /* full-matrix form only: H += Omega_j a_j^+ + conj(Omega_j) a_j */
  double exch[OMAXN * OMAXN];/* full-matrix form only: H += sum_{i<j} J_ij (a_i^+ a_j + a_j^+ a_i) */
} osys;

/* diss: 0 Lindblad, 1 secular; nlev (secular, may be NULL): per mode j the
 * nc[j] - 1 transition occupations, modes one after another. */
static int load_sys(osys *s, int n, const int *nc, const double *det, const double *kerr,
                    const double *chi, const double *g1, const double *gphi, const double *nth,
                    int diss, const double *nlev) {
  if (n < 1 || n > OMAXN || (diss != 0 && diss != 1)) return -1;
  s->n = n;
  s->secular = diss;
  long off = 0;
  for (int j = 0; j < n; ++j) {
    if (nc[j] < 1 || nc[j] > OMAXC) return -1;
    for (int t = 0; t + 1 < nc[j]; ++t) s->nlev[j][t] = nlev ? nlev[off + t] : nth[j];
    off += nc[j] - 1;
  }
  for (int j = 0; j < n; ++j) {
    if (nc[j] < 1) return -1;
    s->nc[j] = nc[j];
    s->det[j] = det[j];
    s->kerr[j] = kerr[j];
    s->g1[j] = g1[j];
    s->gphi[j] = gphi[j];
    s->nth[j] = nth[j];
    for (int i = 0; i < n; ++i) s->chi[j * n + i] = chi[j * n + i];
  }
  return 0;
}

static long box_size(const osys *s) {
  long t = 1;
  for (int j = 0; j < s->n; ++j) t *= s->nc[j];
  return t;
}

/* Energy of the number state |k> (eigenvalue of H above). */
static double energy(const osys *s, const int *k) {
  double e = 0.0;
  for (int j = 0; j < s->n; ++j)
    e += s->det[j] * k[j] + 0.5 * s->kerr[j] * k[j] * (k[j] - 1);
  for (int i = 0; i < s->n; ++i)
    for (int j = i + 1; j < s->n; ++j) e += s->chi[i * s->n + j] * k[i] * k[j];
  return e;
}

/* Matrix elements of the truncated single-mode operators. */
static double elem_a(int row, int col, int nc) { /* <row| a |col> */
  return (col >= 1 && row == col - 1 && col < nc) ? sqrt((double)col) : 0.0;
}
static double elem_adag(int row, int col, int nc) { /* <row| a^+ |col> */
  return (row >= 1 && col == row - 1 && row < nc) ? sqrt((double)row) : 0.0;
}

/*
 * One right-hand-side evaluation on one sector.  For element (k, l):
 *   i (E_k - E_l) A[k,l]
 *   + sum over channels of (kappa/2) (2 (L^+ A L)[k,l] - (L^+L)[k,k] A[k,l] - A[k,l] (L^+L)[l,l])
 * All three jump operators map a number state to (a multiple of) a single
 * number state, so L^+ A L touches exactly one element of A and L^+ L is
 * diagonal.
 */
static void rhs_sector(const osys *s, const int *d, const cplx *A, cplx *out, int part) {
  const int n = s->n;
  const long total = box_size(s);
  long stride[OMAXN];
  stride[n - 1] = 1;
  for (int j = n - 2; j >= 0; --j) stride[j] = stride[j + 1] * s->nc[j + 1];

#pragma omp parallel for schedule(static)
  for (long f = 0; f < total; ++f) {
    int k[OMAXN], l[OMAXN];
    long rem = f;
    int inside = 1;
    for (int j = 0; j < n; ++j) {
      k[j] = (int)(rem / stride[j]);
      rem %= stride[j];
      l[j] = k[j] + d[j];
      if (l[j] < 0 || l[j] >= s->nc[j]) inside = 0;
    }
    if (!inside) {
      out[f] = 0.0;
      continue;
    }
    /* part 1 (jump terms only): every term proportional to A[k,l] itself is
     * left out, i.e. the whole right-hand side is evaluated with a = 0 */
    const cplx a = part == 1 ? 0.0 : A[f];
    cplx r = I * (energy(s, k) - energy(s, l)) * a;
    for (int j = 0; j < n; ++j) {
      const int nc = s->nc[j];
      const int kj = k[j], lj = l[j];
      if (s->secular) {
        /* transitions t <-> t+1 of mode j: down |t><t+1|, up |t+1><t| */
        const double *nb = s->nlev[j];
        const double g = s->g1[j];
        /* jumps: L^+ A L is non-zero only for k_j = l_j */
        if (kj == lj) {
          if (kj >= 1) /* down from kj: (|kj><kj-1|) A (|kj-1><kj|) picks A[k-e_j, l-e_j] */
            r += g * kj * (nb[kj - 1] + 1.0) * A[f - stride[j]];
          if (kj + 1 < nc) /* up from kj: picks A[k+e_j, l+e_j] */
            r += g * (kj + 1) * nb[kj] * A[f + stride[j]];
        }
        /* anticommutators: total rate out of a level m of mode j */
        double out_k = 0.0, out_l = 0.0;
        if (kj >= 1) out_k += g * kj * (nb[kj - 1] + 1.0);
        if (kj + 1 < nc) out_k += g * (kj + 1) * nb[kj];
        if (lj >= 1) out_l += g * lj * (nb[lj - 1] + 1.0);
        if (lj + 1 < nc) out_l += g * (lj + 1) * nb[lj];
        r -= 0.5 * (out_k + out_l) * a;
        /* pure dephasing as in the Lindblad form: L = n_j at rate 2 gamma_phi */
        const double kap = 2.0 * s->gphi[j];
        r += 0.5 * kap * (2.0 * (double)kj * (double)lj - (double)(kj * kj) - (double)(lj * lj)) * a;
        continue;
      }
      /* channel L = a_j: L^+ A L = a^+ A a; (a^+ a)[m,m] = m */
      {
        const double kap = s->g1[j] * (1.0 + s->nth[j]);
        cplx sandwich = 0.0;
        if (kj >= 1 && lj >= 1) /* (a^+ A a)[k,l] = <k|a^+|k-1> A[k-1,l-1] <l-1|a|l> */
          sandwich = elem_adag(kj, kj - 1, nc) * A[f - stride[j]] * elem_a(lj - 1, lj, nc);
        r += 0.5 * kap * (2.0 * sandwich - (double)kj * a - (double)lj * a);
      }
      /* channel L = a_j^+: L^+ A L = a A a^+; (a a^+)[m,m] = m+1 below the top level, 0 at it */
      {
        const double kap = s->g1[j] * s->nth[j];
        cplx sandwich = 0.0;
        if (kj + 1 < nc && lj + 1 < nc)
          sandwich = elem_a(kj, kj + 1, nc) * A[f + stride[j]] * elem_adag(lj + 1, lj, nc);
        const double aadag_k = (kj + 1 < nc) ? (double)(kj + 1) : 0.0;
        const double aadag_l = (lj + 1 < nc) ? (double)(lj + 1) : 0.0;
        r += 0.5 * kap * (2.0 * sandwich - aadag_k * a - aadag_l * a);
      }
      /* channel L = n_j: L^+ A L = n A n; (n n)[m,m] = m^2 */
      {
        const double kap = 2.0 * s->gphi[j];
        const cplx sandwich = (double)kj * a * (double)lj;
        r += 0.5 * kap * (2.0 * sandwich - (double)(kj * kj) * a - (double)(lj * lj) * a);
      }
    }
    out[f] = r;
  }
}

static void rhs_all(const osys *s, int nsec, const int *d, const cplx *A, cplx *out) {
  const long box = box_size(s);
  for (int q = 0; q < nsec; ++q) rhs_sector(s, d + q * s->n, A + q * box, out + q * box, 0);
}

static void jumps_all(const osys *s, int nsec, const int *d, const cplx *A, cplx *out) {
  const long box = box_size(s);
  for (int q = 0; q < nsec; ++q) rhs_sector(s, d + q * s->n, A + q * box, out + q * box, 1);
}

/*
 * Diagonal coefficient of the right-hand side: the factor D[k,l] with which
 * A[k,l] enters its own derivative (Hamiltonian phase, damping from the
 * anticommutators, dephasing).  Both right-hand sides are linear, and on the
 * all-ones state the full one is D + J(ones) element by element while the
 * jump-only one is J(ones); their difference is D, term by term as written
 * above.
 */
static int diagonal_all(const osys *s, int nsec, const int *d, cplx *D) {
  const long len = box_size(s) * nsec;
  cplx *one = malloc(sizeof(cplx) * len), *full = malloc(sizeof(cplx) * len), *jmp = malloc(sizeof(cplx) * len);
  if (!one || !full || !jmp) {
    free(one); free(full); free(jmp);
    return -2;
  }
  for (long i = 0; i < len; ++i) one[i] = 1.0;
  rhs_all(s, nsec, d, one, full);
  jumps_all(s, nsec, d, one, jmp);
  for (long i = 0; i < len; ++i) D[i] = full[i] - jmp[i];
  free(one); free(full); free(jmp);
  return 0;
}

/* y <- x + c * z, elementwise */
static void axpy_into(long len, cplx *y, const cplx *x, double c, const cplx *z) {
#pragma omp parallel for schedule(static)
  for (long i = 0; i < len; ++i) y[i] = x[i] + c * z[i];
}

static void set_threads(int nthreads) {
#ifdef _OPENMP
  if (nthreads > 0) omp_set_num_threads(nthreads);
#else
  (void)nthreads;
#endif
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

int oracle_rhs(int n, const int *nc, const double *det, const double *kerr, const double *chi,
               const double *g1, const double *gphi, const double *nth, int diss, const double *nlev,
               int nsec, const int *d, const cplx *A, cplx *out, int nthreads) {
  osys s;
  if (load_sys(&s, n, nc, det, kerr, chi, g1, gphi, nth, diss, nlev)) return -1;
  set_threads(nthreads);
  rhs_all(&s, nsec, d, A, out);
  return 0;
}

/*
 * Classical RK4 with fixed step h:
 *   k1 = f(A), k2 = f(A + h/2 k1), k3 = f(A + h/2 k2), k4 = f(A + h k3),
 *   A <- A + h/6 (k1 + 2 k2 + 2 k3 + k4).
 */
int oracle_evolve(int n, const int *nc, const double *det, const double *kerr, const double *chi,
                  const double *g1, const double *gphi, const double *nth, int diss, const double *nlev,
                  int nsec, const int *d, cplx *A, long nsteps, double h, int nthreads) {
  osys s;
  if (load_sys(&s, n, nc, det, kerr, chi, g1, gphi, nth, diss, nlev)) return -1;
  set_threads(nthreads);
  const long len = box_size(&s) * nsec;
  cplx *kk = malloc(sizeof(cplx) * len);
  cplx *Y = malloc(sizeof(cplx) * len);
  cplx *acc = malloc(sizeof(cplx) * len);
  if (!kk || !Y || !acc) {
    free(kk); free(Y); free(acc);
    return -2;
  }
  for (long step = 0; step < nsteps; ++step) {
    rhs_all(&s, nsec, d, A, kk);            /* k1 */
    axpy_into(len, acc, A, h / 6.0, kk);
    axpy_into(len, Y, A, h / 2.0, kk);
    rhs_all(&s, nsec, d, Y, kk);            /* k2 */
    axpy_into(len, acc, acc, h / 3.0, kk);
    axpy_into(len, Y, A, h / 2.0, kk);
    rhs_all(&s, nsec, d, Y, kk);            /* k3 */
    axpy_into(len, acc, acc, h / 3.0, kk);
    axpy_into(len, Y, A, h, kk);
    rhs_all(&s, nsec, d, Y, kk);            /* k4 */
    axpy_into(len, A, acc, h / 6.0, kk);
  }
  free(kk); free(Y); free(acc);
  return 0;
}

/*
 * Integrating-factor ("Lawson") fourth-order Runge-Kutta with fixed step h.
 * Write the right-hand side as D A + J(A), D the diagonal coefficients above
 * and J the jump terms.  With u(tau) = exp(-D tau) A(t_n + tau) the equation
 * becomes u' = f(tau, u) = exp(-D tau) J(exp(D tau) u), integrated by the
 * classical RK4 stages from u(0) = A(t_n); then A(t_n + h) = exp(D h) u(h).
 * Elements outside the box (l out of range) stay zero.
 */
static void lawson_f(const osys *s, int nsec, const int *d, const cplx *D, double tau, const cplx *u, cplx *tmp,
                     cplx *out, long len) {
#pragma omp parallel for schedule(static)
  for (long i = 0; i < len; ++i) tmp[i] = cexp(D[i] * tau) * u[i];
  jumps_all(s, nsec, d, tmp, out);
#pragma omp parallel for schedule(static)
  for (long i = 0; i < len; ++i) out[i] *= cexp(-D[i] * tau);
}

int oracle_evolve_lawson(int n, const int *nc, const double *det, const double *kerr, const double *chi,
                         const double *g1, const double *gphi, const double *nth, int diss, const double *nlev,
                         int nsec, const int *d, cplx *A, long nsteps, double h, int nthreads) {
  osys s;
  if (load_sys(&s, n, nc, det, kerr, chi, g1, gphi, nth, diss, nlev)) return -1;
  set_threads(nthreads);
  const long len = box_size(&s) * nsec;
  cplx *D = malloc(sizeof(cplx) * len), *kk = malloc(sizeof(cplx) * len), *Y = malloc(sizeof(cplx) * len),
       *acc = malloc(sizeof(cplx) * len), *tmp = malloc(sizeof(cplx) * len);
  if (!D || !kk || !Y || !acc || !tmp) {
    free(D); free(kk); free(Y); free(acc); free(tmp);
    return -2;
  }
  if (diagonal_all(&s, nsec, d, D)) {
    free(D); free(kk); free(Y); free(acc); free(tmp);
    return -2;
  }
  for (long step = 0; step < nsteps; ++step) {
    lawson_f(&s, nsec, d, D, 0.0, A, tmp, kk, len);       /* k1 */
    axpy_into(len, acc, A, h / 6.0, kk);
    axpy_into(len, Y, A, h / 2.0, kk);
    lawson_f(&s, nsec, d, D, 0.5 * h, Y, tmp, kk, len);   /* k2 */
    axpy_into(len, acc, acc, h / 3.0, kk);
    axpy_into(len, Y, A, h / 2.0, kk);
    lawson_f(&s, nsec, d, D, 0.5 * h, Y, tmp, kk, len);   /* k3 */
    axpy_into(len, acc, acc, h / 3.0, kk);
    axpy_into(len, Y, A, h, kk);
    lawson_f(&s, nsec, d, D, h, Y, tmp, kk, len);         /* k4 */
    axpy_into(len, acc, acc, h / 6.0, kk);
#pragma omp parallel for schedule(static)
    for (long i = 0; i < len; ++i) A[i] = cexp(D[i] * h) * acc[i];
  }
  free(D); free(kk); free(Y); free(acc); free(tmp);
  return 0;
}

/*
 * Right-hand side on the full matrix.  Element (k, l), with K and L the row
 * and column indices and s_j the index stride of mode j:
 *   i (E_k - E_l) A[k,l] + dissipator terms (as in rhs_sector, with the
 *   neighbours A[k -+ e_j, l -+ e_j] taken from the full matrix)
 *   + i (Omega_j (a^+A) + conj(Omega_j) (aA) - Omega_j (Aa^+) - conj(Omega_j) (Aa))[k,l]
 *   + i J_ij ((a_i^+ a_j A) + (a_j^+ a_i A) - (A a_i^+ a_j) - (A a_j^+ a_i))[k,l]
 * with the truncated matrix elements
 *   (a_j^+ A)[k,l] = sqrt(k_j) A[k-e_j, l]        (a_j A)[k,l] = sqrt(k_j+1) A[k+e_j, l]
 *   (A a_j^+)[k,l] = sqrt(l_j+1) A[k, l+e_j]      (A a_j)[k,l] = sqrt(l_j) A[k, l-e_j]
 *   (a_i^+ a_j A)[k,l] = sqrt(k_i (k_j+1)) A[k-e_i+e_j, l]
 *   (A a_i^+ a_j)[k,l] = sqrt(l_j (l_i+1)) A[k, l-e_j+e_i]
 * (zero where an index leaves [0, Nc)).
 */
static void rhs_full(const osys *s, const cplx *A, cplx *out) {
  const int n = s->n;
  const long dim = box_size(s);
  long stride[OMAXN];
  stride[n - 1] = 1;
  for (int j = n - 2; j >= 0; --j) stride[j] = stride[j + 1] * s->nc[j + 1];

#pragma omp parallel for schedule(static)
  for (long f = 0; f < dim * dim; ++f) {
    const long K = f / dim, L = f % dim;
    int k[OMAXN], l[OMAXN];
    long rk = K, rl = L;
    for (int j = 0; j < n; ++j) {
      k[j] = (int)(rk / stride[j]);
      rk %= stride[j];
      l[j] = (int)(rl / stride[j]);
      rl %= stride[j];
    }
#define AT(KK, LL) A[(KK) * dim + (LL)]
    const cplx a = A[f];
    cplx r = I * (energy(s, k) - energy(s, l)) * a;
    for (int j = 0; j < n; ++j) {
      const int nc = s->nc[j];
      const int kj = k[j], lj = l[j];
      const long sj = stride[j];
      if (s->secular) {
        const double *nb = s->nlev[j];
        const double g = s->g1[j];
        if (kj == lj) {
          if (kj >= 1) r += g * kj * (nb[kj - 1] + 1.0) * AT(K - sj, L - sj);
          if (kj + 1 < nc) r += g * (kj + 1) * nb[kj] * AT(K + sj, L + sj);
        }
        double out_k = 0.0, out_l = 0.0;
        if (kj >= 1) out_k += g * kj * (nb[kj - 1] + 1.0);
        if (kj + 1 < nc) out_k += g * (kj + 1) * nb[kj];
        if (lj >= 1) out_l += g * lj * (nb[lj - 1] + 1.0);
        if (lj + 1 < nc) out_l += g * (lj + 1) * nb[lj];
        r -= 0.5 * (out_k + out_l) * a;
      } else {
        const double kd = s->g1[j] * (1.0 + s->nth[j]), ku = s->g1[j] * s->nth[j];
        if (kj >= 1 && lj >= 1) r += kd * sqrt((double)kj * lj) * AT(K - sj, L - sj);
        r -= 0.5 * kd * (kj + lj) * a;
        if (kj + 1 < nc && lj + 1 < nc) r += ku * sqrt((double)(kj + 1) * (lj + 1)) * AT(K + sj, L + sj);
        const double tk = (kj + 1 < nc) ? kj + 1 : 0, tl = (lj + 1 < nc) ? lj + 1 : 0;
        r -= 0.5 * ku * (tk + tl) * a;
      }
      /* dephasing, L = n_j at rate 2 gamma_phi: gamma_phi (2 k l - k^2 - l^2) */
      r += s->gphi[j] * (2.0 * kj * lj - (double)kj * kj - (double)lj * lj) * a;
      /* drive */
      const cplx om = s->drive[j];
      if (om != 0.0) {
        cplx c = 0.0;
        if (kj >= 1) c += om * sqrt((double)kj) * AT(K - sj, L);
        if (kj + 1 < nc) c += conj(om) * sqrt((double)(kj + 1)) * AT(K + sj, L);
        if (lj + 1 < nc) c -= om * sqrt((double)(lj + 1)) * AT(K, L + sj);
        if (lj >= 1) c -= conj(om) * sqrt((double)lj) * AT(K, L - sj);
        r += I * c;
      }
    }
    /* exchange */
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) {
        const double J = s->exch[i * n + j];
        if (J == 0.0) continue;
        const long si = stride[i], sj = stride[j];
        const int nci = s->nc[i], ncj = s->nc[j];
        cplx c = 0.0;
        if (k[i] >= 1 && k[j] + 1 < ncj) c += sqrt((double)k[i] * (k[j] + 1)) * AT(K - si + sj, L);
        if (k[j] >= 1 && k[i] + 1 < nci) c += sqrt((double)k[j] * (k[i] + 1)) * AT(K - sj + si, L);
        if (l[j] >= 1 && l[i] + 1 < nci) c -= sqrt((double)l[j] * (l[i] + 1)) * AT(K, L - sj + si);
        if (l[i] >= 1 && l[j] + 1 < ncj) c -= sqrt((double)l[i] * (l[j] + 1)) * AT(K, L - si + sj);
        r += I * J * c;
      }
#undef AT
    out[f] = r;
  }
}

static int load_full(osys *s, const double *drive, const double *exch) {
  for (int j = 0; j < s->n; ++j) s->drive[j] = drive ? drive[2 * j] + I * drive[2 * j + 1] : 0.0;
  for (int i = 0; i < s->n * s->n; ++i) s->exch[i] = exch ? exch[i] : 0.0;
  return 0;
}

int oracle_rhs_full(int n, const int *nc, const double *det, const double *kerr, const double *chi,
                    const double *g1, const double *gphi, const double *nth, int diss, const double *nlev,
                    const double *drive, const double *exch, const cplx *A, cplx *out, int nthreads) {
  osys s;
  if (load_sys(&s, n, nc, det, kerr, chi, g1, gphi, nth, diss, nlev) || load_full(&s, drive, exch)) return -1;
  set_threads(nthreads);
  rhs_full(&s, A, out);
  return 0;
}

/* Classical RK4 on the full matrix (stages as in oracle_evolve). */
int oracle_evolve_full(int n, const int *nc, const double *det, const double *kerr, const double *chi,
                       const double *g1, const double *gphi, const double *nth, int diss, const double *nlev,
                       const double *drive, const double *exch, cplx *A, long nsteps, double h, int nthreads) {
  osys s;
  if (load_sys(&s, n, nc, det, kerr, chi, g1, gphi, nth, diss, nlev) || load_full(&s, drive, exch)) return -1;
  set_threads(nthreads);
  const long dim = box_size(&s), len = dim * dim;
  cplx *kk = malloc(sizeof(cplx) * len), *Y = malloc(sizeof(cplx) * len), *acc = malloc(sizeof(cplx) * len);
  if (!kk || !Y || !acc) {
    free(kk); free(Y); free(acc);
    return -2;
  }
  for (long step = 0; step < nsteps; ++step) {
    rhs_full(&s, A, kk);
    axpy_into(len, acc, A, h / 6.0, kk);
    axpy_into(len, Y, A, h / 2.0, kk);
    rhs_full(&s, Y, kk);
    axpy_into(len, acc, acc, h / 3.0, kk);
    axpy_into(len, Y, A, h / 2.0, kk);
    rhs_full(&s, Y, kk);
    axpy_into(len, acc, acc, h / 3.0, kk);
    axpy_into(len, Y, A, h, kk);
    rhs_full(&s, Y, kk);
    axpy_into(len, A, acc, h / 6.0, kk);
  }
  free(kk); free(Y); free(acc);
  return 0;
}

int oracle_num_params(int n) { return n + n * (n - 1) / 2 + 3 * n; }

/*
 * The right-hand side is linear in the parameter vector
 * theta = (K, chi[i<j], Delta, gamma1, gamma_phi) for fixed nth, so its
 * derivative along theta_p is the right-hand side of a system whose only
 * non-zero parameter is theta_p = 1.
 */
static void unit_system(const osys *s, int p, osys *u) {
  const int n = s->n;
  *u = *s;
  memset(u->det, 0, sizeof(u->det));
  memset(u->kerr, 0, sizeof(u->kerr));
  memset(u->chi, 0, sizeof(u->chi));
  memset(u->g1, 0, sizeof(u->g1));
  memset(u->gphi, 0, sizeof(u->gphi));
  if (p < n) { u->kerr[p] = 1.0; return; }
  p -= n;
  const int npair = n * (n - 1) / 2;
  if (p < npair) {
    int q = 0;
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j, ++q)
        if (q == p) { u->chi[i * n + j] = 1.0; u->chi[j * n + i] = 1.0; }
    return;
  }
  p -= npair;
  if (p < n) { u->det[p] = 1.0; return; }
  p -= n;
  if (p < n) { u->g1[p] = 1.0; return; }
  p -= n;
  u->gphi[p] = 1.0;
}

/*
 * Forward sensitivities: the augmented state (A, S_1..S_P) with
 *   dS_p/dt = f(S_p) + (df/dtheta_p)(A)
 * integrated with the same RK4 steps.  S_p(T) is then the exact derivative
 * of the discrete map A(0) -> A(T) with respect to theta_p.  S must hold
 * P * nsec * box elements and is overwritten (S_p(0) = 0).
 */
int oracle_evolve_sens(int n, const int *nc, const double *det, const double *kerr,
                       const double *chi, const double *g1, const double *gphi, const double *nth,
                       int diss, const double *nlev, int nsec, const int *d, cplx *A, cplx *S,
                       long nsteps, double h, int nthreads) {
  osys s;
  if (load_sys(&s, n, nc, det, kerr, chi, g1, gphi, nth, diss, nlev)) return -1;
  set_threads(nthreads);
  const int P = oracle_num_params(n);
  const long len = box_size(&s) * nsec;
  const long tot = len * (P + 1);
  osys *units = malloc(sizeof(osys) * P);
  cplx *X = malloc(sizeof(cplx) * tot);   /* [A | S_1 | ... | S_P] */
  cplx *kk = malloc(sizeof(cplx) * tot);
  cplx *Y = malloc(sizeof(cplx) * tot);
  cplx *acc = malloc(sizeof(cplx) * tot);
  cplx *tmp = malloc(sizeof(cplx) * len);
  if (!units || !X || !kk || !Y || !acc || !tmp) {
    free(units); free(X); free(kk); free(Y); free(acc); free(tmp);
    return -2;
  }
  for (int p = 0; p < P; ++p) unit_system(&s, p, &units[p]);
  memcpy(X, A, sizeof(cplx) * len);
  memset(X + len, 0, sizeof(cplx) * len * P);

  for (long step = 0; step < nsteps; ++step) {
    for (int st = 0; st < 4; ++st) {
      const cplx *src = (st == 0) ? X : Y;
      /* kk = F(src): the augmented right-hand side */
      rhs_all(&s, nsec, d, src, kk);
      for (int p = 0; p < P; ++p) {
        rhs_all(&s, nsec, d, src + len * (p + 1), kk + len * (p + 1));
        rhs_all(&units[p], nsec, d, src, tmp);
        axpy_into(len, kk + len * (p + 1), kk + len * (p + 1), 1.0, tmp);
      }
      static const double wacc[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
      static const double wnext[3] = {0.5, 0.5, 1.0};
      if (st == 0) axpy_into(tot, acc, X, h * wacc[0], kk);
      else if (st < 3) axpy_into(tot, acc, acc, h * wacc[st], kk);
      if (st < 3) axpy_into(tot, Y, X, h * wnext[st], kk);
      else axpy_into(tot, X, acc, h * wacc[3], kk);
    }
  }
  memcpy(A, X, sizeof(cplx) * len);
  memcpy(S, X + len, sizeof(cplx) * len * P);
  free(units); free(X); free(kk); free(Y); free(acc); free(tmp);
  return 0;
}

/*
 * ------------------------------------------------------------------------
 * Separated form of the paper's method (Eqs. (9a)-(9c), with the network
 * generator of Eqs. (16)-(19)): the transformed generating function of each
 * initial monomial x^p y^q is held as G = Gx(x) Gy(y) + R(x, y) with
 *   dGx/dt = (Kx + C) Gx,   dGy/dt = (Ky - C) Gy,
 *   dR/dt  = (Kx + Ky + P) R + P (Gx Gy),
 * Gx(0) = x^p, Gy(0) = y^q, R(0) = 0, and C = -(i/2)(E(p) + E(q)) (the
 * separation constant of Eq. (20) for this Hamiltonian).  Everything is in
 * the coefficients of the generating functions (g = <k|A|l> / sqrt(k! l!)),
 * on the truncated box:
 *   Kx (left multiplication by i H plus the k-half of the dissipator):
 *     x^k  ->  [i E(k) - sum_j (out_j(k_j) / 2 + gamma_phi_j k_j^2)] x^k
 *     drive:    i Omega_j x_j + i conj(Omega_j) d/dx_j
 *     exchange: i J_ij (x_i d/dx_j + x_j d/dx_i)
 *   Ky (right multiplication by -i H plus the l-half):
 *     y^l  ->  [-i E(l) - sum_j (out_j(l_j) / 2 + gamma_phi_j l_j^2)] y^l
 *     drive:    -i Omega_j d/dy_j - i conj(Omega_j) y_j
 *     exchange: -i J_ij (y_j d/dy_i + y_i d/dy_j)
 *   P (the parts that couple x and y: jumps and the dephasing cross term):
 *     Lindblad:  gamma1_j (1 + nth_j) x_j y_j  +  gamma1_j nth_j d/dx_j d/dy_j
 *     secular:   the same two shifts restricted to the terms with k_j = l_j,
 *                with the per-transition rates (down gamma1 (nbar_{k-1} + 1),
 *                up gamma1 nbar_k (k + 1)^2 on the coefficients)
 *     dephasing: 2 gamma_phi_j k_j l_j
 * with out_j(n) the total jump rate out of level n (truncated ladders:
 * Lindblad gamma1 (1 + nth) n + gamma1 nth (n + 1)[n + 1 < Nc]; secular the
 * sum of the two transition rates).  Kx + Ky + P is the full generator of
 * the coefficients, so G follows the adjoint master equation exactly in
 * continuous time.
 *
 * Classical RK4 on the joint state (Gx_i, Gy_i of every monomial i, R).
 * R is linear with the source sum_i c_i P(Gx_i Gy_i) (c_i = g_{p_i q_i}(0)),
 * so one R holds the sum over the monomials of c_i R_i.
 *
 * rmode 0: R on the whole (k, l) box.  rmode 1: R restricted to the diagonal
 * k = l (a function of the products z_j = x_j y_j alone, the approximation
 * the paper reports for the network); each stage's derivative is taken on
 * the diagonal, where Kx + Ky reduces to -sum_j out_j(m_j) and P keeps its
 * diagonal shifts, and the off-diagonal part of every term is dropped.
 *
 * gx, gy: [nmono * dim] in/out (row-major boxes, last mode fastest), r:
 * [dim * dim] (rmode 0) or [dim] (rmode 1) in/out, coef: [nmono].
 */
static void sep_tables(const osys *s, double *outr /* [OMAXN][OMAXC] */, double *down, double *up) {
  for (int j = 0; j < s->n; ++j) {
    const int nc = s->nc[j];
    for (int m = 0; m < nc; ++m) {
      double o = 0.0, dn = 0.0, u = 0.0;
      if (s->secular) {
        const double *nb = s->nlev[j];
        if (m >= 1) o += s->g1[j] * m * (nb[m - 1] + 1.0);
        if (m + 1 < nc) o += s->g1[j] * (m + 1) * nb[m];
        if (m >= 1) dn = s->g1[j] * (nb[m - 1] + 1.0);
        if (m + 1 < nc) u = s->g1[j] * nb[m] * (m + 1.0) * (m + 1.0);
      } else {
        const double kd = s->g1[j] * (1.0 + s->nth[j]), ku = s->g1[j] * s->nth[j];
        o = kd * m + ((m + 1 < nc) ? ku * (m + 1) : 0.0);
        if (m >= 1) dn = kd;
        if (m + 1 < nc) u = ku; /* times (k_j + 1)(l_j + 1) at the point */
      }
      outr[j * OMAXC + m] = o;
      down[j * OMAXC + m] = dn;
      up[j * OMAXC + m] = u;
    }
  }
}

static void unflat(const osys *s, long f, int *k) {
  for (int j = s->n - 1; j >= 0; --j) {
    k[j] = (int)(f % s->nc[j]);
    f /= s->nc[j];
  }
}

/* out = (Kx + c) gx (side 0) or (Ky + c) gy (side 1) on one N-mode box */
static void sep_side(const osys *s, const double *outr, int side, cplx c, const cplx *g, cplx *out) {
  const int n = s->n;
  const long dim = box_size(s);
  long stride[OMAXN];
  stride[n - 1] = 1;
  for (int j = n - 2; j >= 0; --j) stride[j] = stride[j + 1] * s->nc[j + 1];
  const double sg = side == 0 ? 1.0 : -1.0;
  for (long f = 0; f < dim; ++f) {
    int k[OMAXN];
    unflat(s, f, k);
    double damp = 0.0;
    for (int j = 0; j < n; ++j) damp += 0.5 * outr[j * OMAXC + k[j]] + s->gphi[j] * k[j] * k[j];
    cplx r = (sg * I * energy(s, k) - damp + c) * g[f];
    for (int j = 0; j < n; ++j) {
      const cplx om = s->drive[j];
      if (om == 0.0) continue;
      const int nc = s->nc[j];
      /* x side: i Omega x + i conj(Omega) d/dx;  y side: -i Omega d/dy - i conj(Omega) y */
      const cplx cmul = side == 0 ? I * om : -I * conj(om);   /* multiplication by the variable */
      const cplx cder = side == 0 ? I * conj(om) : -I * om;   /* derivative */
      if (k[j] >= 1) r += cmul * g[f - stride[j]];
      if (k[j] + 1 < nc) r += cder * (k[j] + 1.0) * g[f + stride[j]];
    }
    for (int i = 0; i < n; ++i)
      for (int j = i + 1; j < n; ++j) {
        const double J = s->exch[i * n + j];
        if (J == 0.0) continue;
        /* x_i d/dx_j + x_j d/dx_i (and the same in y): v_i d/dv_j moves one
           unit from j to i with the factor (k_j + 1) of the source */
        cplx t = 0.0;
        if (k[i] >= 1 && k[j] + 1 < s->nc[j]) t += (k[j] + 1.0) * g[f - stride[i] + stride[j]];
        if (k[j] >= 1 && k[i] + 1 < s->nc[i]) t += (k[i] + 1.0) * g[f - stride[j] + stride[i]];
        r += sg * I * J * t;
      }
    out[f] = r;
  }
}

/* P applied to a full-box function S (rmode 0: every (k, l); rmode 1: only
 * the diagonal points (m, m), written to out[m]).  S(k, l) is given by a
 * callback-free representation: S = R (full) or the outer products of the
 * monomials (gx_i (x) gy_i weighted by c_i), evaluated at the points needed. */
typedef struct {
  const cplx *R;       /* full R (may be NULL) */
  int nmono;
  const cplx *gx, *gy, *coef;
  long dim;
} sep_src;

static cplx src_at(const sep_src *q, long K, long L) {
  cplx v = q->R ? q->R[K * q->dim + L] : 0.0;
  for (int i = 0; i < q->nmono; ++i) v += q->coef[i] * q->gx[i * q->dim + K] * q->gy[i * q->dim + L];
  return v;
}

static cplx apply_P(const osys *s, const double *down, const double *up, const sep_src *q, long K, long L,
                    const int *k, const int *l, const long *stride) {
  cplx r = 0.0;
  for (int j = 0; j < s->n; ++j) {
    if (s->secular && k[j] != l[j]) {
      continue;
    }
    if (k[j] >= 1 && l[j] >= 1) {
      const double dn = s->secular ? down[j * OMAXC + k[j]] : down[j * OMAXC + 1];
      r += dn * src_at(q, K - stride[j], L - stride[j]);
    }
    if (k[j] + 1 < s->nc[j] && l[j] + 1 < s->nc[j]) {
      const double u = s->secular ? up[j * OMAXC + k[j]] : up[j * OMAXC + k[j]] * (k[j] + 1.0) * (l[j] + 1.0);
      r += u * src_at(q, K + stride[j], L + stride[j]);
    }
  }
  for (int j = 0; j < s->n; ++j)
    if (s->gphi[j] != 0.0 && k[j] * l[j] != 0) r += 2.0 * s->gphi[j] * k[j] * l[j] * src_at(q, K, L);
  return r;
}

/* derivative of R: rmode 0 on the full box, rmode 1 on the diagonal */
static void sep_R(const osys *s, const double *outr, const double *down, const double *up, int rmode,
                  const cplx *R, int nmono, const cplx *gx, const cplx *gy, const cplx *coef, cplx *out) {
  const int n = s->n;
  const long dim = box_size(s);
  long stride[OMAXN];
  stride[n - 1] = 1;
  for (int j = n - 2; j >= 0; --j) stride[j] = stride[j + 1] * s->nc[j + 1];
  if (rmode == 0) {
    /* (Kx + Ky) R through the two one-sided maps on rows and columns, P on R + sum_i c_i gx_i gy_i */
    cplx *col = malloc(sizeof(cplx) * dim), *tmp = malloc(sizeof(cplx) * dim);
    for (long K = 0; K < dim; ++K) { /* Ky on each row K (a function of l) */
      sep_side(s, outr, 1, 0.0, R + K * dim, tmp);
      for (long L = 0; L < dim; ++L) out[K * dim + L] = tmp[L];
    }
    for (long L = 0; L < dim; ++L) { /* Kx on each column L (a function of k) */
      for (long K = 0; K < dim; ++K) col[K] = R[K * dim + L];
      sep_side(s, outr, 0, 0.0, col, tmp);
      for (long K = 0; K < dim; ++K) out[K * dim + L] += tmp[K];
    }
    sep_src q = {R, nmono, gx, gy, coef, dim};
#pragma omp parallel for schedule(static)
    for (long f = 0; f < dim * dim; ++f) {
      const long K = f / dim, L = f % dim;
      int k[OMAXN], l[OMAXN];
      unflat(s, K, k);
      unflat(s, L, l);
      out[f] += apply_P(s, down, up, &q, K, L, k, l, stride);
    }
    free(col); free(tmp);
  } else {
    /* diagonal: -sum_j out_j(m_j) R(m) + P (R + sum_i c_i gx_i gy_i) on (m, m); the
       dephasing terms of Kx + Ky (-gamma_phi (k^2 + l^2)) and of P (2 gamma_phi k l)
       cancel on the diagonal and are left out of both */
#pragma omp parallel for schedule(static)
    for (long m = 0; m < dim; ++m) {
      int k[OMAXN];
      unflat(s, m, k);
      double o = 0.0;
      for (int j = 0; j < n; ++j) o += outr[j * OMAXC + k[j]];
      cplx r = -o * R[m];
      /* P on the diagonal: its shifts stay on the diagonal (k - e_j, k - e_j) */
      for (int j = 0; j < n; ++j) {
        if (k[j] >= 1) {
          const double dn = s->secular ? down[j * OMAXC + k[j]] : down[j * OMAXC + 1];
          cplx v = R[m - stride[j]];
          for (int i = 0; i < nmono; ++i)
            v += coef[i] * gx[i * dim + m - stride[j]] * gy[i * dim + m - stride[j]];
          r += dn * v;
        }
        if (k[j] + 1 < s->nc[j]) {
          const double u = s->secular ? up[j * OMAXC + k[j]] : up[j * OMAXC + k[j]] * (k[j] + 1.0) * (k[j] + 1.0);
          cplx v = R[m + stride[j]];
          for (int i = 0; i < nmono; ++i)
            v += coef[i] * gx[i * dim + m + stride[j]] * gy[i * dim + m + stride[j]];
          r += u * v;
        }
        if (s->gphi[j] != 0.0 && k[j] != 0) {
          cplx v = 0.0; /* the cross term acts on the source only (its R part cancelled above) */
          for (int i = 0; i < nmono; ++i) v += coef[i] * gx[i * dim + m] * gy[i * dim + m];
          r += 2.0 * s->gphi[j] * k[j] * k[j] * v;
        }
      }
      out[m] = r;
    }
  }
}

int oracle_evolve_separated(int n, const int *nc, const double *det, const double *kerr, const double *chi,
                            const double *g1, const double *gphi, const double *nth, int diss, const double *nlev,
                            const double *drive, const double *exch, int nmono, const int *p, const int *q,
                            const cplx *coef, int rmode, cplx *gx, cplx *gy, cplx *r, long nsteps, double h,
                            int nthreads) {
  osys s;
  if (load_sys(&s, n, nc, det, kerr, chi, g1, gphi, nth, diss, nlev) || load_full(&s, drive, exch)) return -1;
  if (rmode != 0 && rmode != 1) return -1;
  set_threads(nthreads);
  const long dim = box_size(&s), rlen = rmode == 0 ? dim * dim : dim;
  const long xlen = (long)nmono * dim;
  static double outr[OMAXN * OMAXC], down[OMAXN * OMAXC], up[OMAXN * OMAXC];
  sep_tables(&s, outr, down, up);
  cplx *Cs = malloc(sizeof(cplx) * (nmono > 0 ? nmono : 1));
  for (int i = 0; i < nmono; ++i) Cs[i] = -0.5 * I * (energy(&s, p + (long)i * n) + energy(&s, q + (long)i * n));
  /* joint state u = (gx, gy, r); RK4 with stage inputs Y, derivative kk, accumulator acc */
  const long tot = 2 * xlen + rlen;
  cplx *U = malloc(sizeof(cplx) * tot), *Y = malloc(sizeof(cplx) * tot), *kk = malloc(sizeof(cplx) * tot),
       *acc = malloc(sizeof(cplx) * tot);
  if (!U || !Y || !kk || !acc || !Cs) {
    free(U); free(Y); free(kk); free(acc); free(Cs);
    return -2;
  }
  memcpy(U, gx, sizeof(cplx) * xlen);
  memcpy(U + xlen, gy, sizeof(cplx) * xlen);
  memcpy(U + 2 * xlen, r, sizeof(cplx) * rlen);
  static const double wacc[4] = {1.0 / 6.0, 1.0 / 3.0, 1.0 / 3.0, 1.0 / 6.0};
  static const double wnext[3] = {0.5, 0.5, 1.0};
  for (long step = 0; step < nsteps; ++step) {
    for (int st = 0; st < 4; ++st) {
      const cplx *src = st == 0 ? U : Y;
#pragma omp parallel for schedule(static)
      for (int i = 0; i < nmono; ++i) {
        sep_side(&s, outr, 0, Cs[i], src + (long)i * dim, kk + (long)i * dim);
        sep_side(&s, outr, 1, -Cs[i], src + xlen + (long)i * dim, kk + xlen + (long)i * dim);
      }
      sep_R(&s, outr, down, up, rmode, src + 2 * xlen, nmono, src, src + xlen, coef, kk + 2 * xlen);
      if (st == 0) axpy_into(tot, acc, U, h * wacc[0], kk);
      else axpy_into(tot, acc, acc, h * wacc[st], kk);
      if (st < 3) axpy_into(tot, Y, U, h * wnext[st], kk);
      else memcpy(U, acc, sizeof(cplx) * tot);
    }
  }
  memcpy(gx, U, sizeof(cplx) * xlen);
  memcpy(gy, U + xlen, sizeof(cplx) * xlen);
  memcpy(r, U + 2 * xlen, sizeof(cplx) * rlen);
  free(U); free(Y); free(kk); free(acc); free(Cs);
  return 0;
}
