// Separated form of the transformed generating function (Eqs. (9a)-(9c)),
// for the network generator of Eqs. (16)-(19): each initial monomial
// x^p y^q (Eq. (10)) is held as G = Gx(x) Gy(y) + R(x, y) with
//   dGx/dt = (Kx + C) Gx,   dGy/dt = (Ky - C) Gy,
//   dR/dt  = (Kx + Ky + P) R + P (Gx Gy),
// Gx and Gy are grids over the N occupations k (resp. l); R is the sum over
// the monomials of c_i R_i (R is linear in its source), either on the whole
// (k, l) box or restricted to its diagonal k = l (the paper's approximation
// of R by a function of the products x_j y_j).  In coefficients:
//   Kx:  [i E(k) + sum_j (dk_j(k_j) - gamma_phi_j k_j^2)] g(k)
//        + i Omega_j g(k - e_j) + i conj(Omega_j) (k_j + 1) g(k + e_j)
//        + i J_ij [(k_j + 1) g(k - e_i + e_j) + (k_i + 1) g(k - e_j + e_i)]
//   Ky:  [-i E(l) + sum_j (dk_j(l_j) - gamma_phi_j l_j^2)] g(l)
//        - i conj(Omega_j) g(l - e_j) - i Omega_j (l_j + 1) g(l + e_j)
//        - i J_ij [(l_j + 1) g(l - e_i + e_j) + (l_i + 1) g(l - e_j + e_i)]
//   P:   jumps g(k -+ e_j, l -+ e_j) (secular: where k_j = l_j) and the
//        dephasing cross term 2 gamma_phi_j k_j l_j
// with the tables of the full-grid network generator (FullTables: E_j, the
// damping dk, the jump coefficients adn and aup), so Kx + Ky + P is exactly
// that generator.  Classical RK4 on the joint state (Gx_i, Gy_i, R), FP64.
//
// Buffers per grid (2M grids of D points in one array each, gx_i at i D,
// gy_i at (M + i) D; R likewise): u (state), acc (RK4 sum), ya, yb (stage
// inputs: stage 1 reads u and writes ya, 2 reads ya and writes yb, 3 reads yb
// and writes ya, 4 reads ya and writes u).
#include <hip/hip_runtime.h>

#include "hgf_internal.h"
#include "hgf_kernels.h"

#define HGF_CONST __attribute__((address_space(4)))

namespace hgf {

namespace {

__device__ __forceinline__ double2 c_add(double2 a, double2 b) { return make_double2(a.x + b.x, a.y + b.y); }
__device__ __forceinline__ double2 c_sub_(double2 a, double2 b) { return make_double2(a.x - b.x, a.y - b.y); }
__device__ __forceinline__ double2 c_scale(double s, double2 a) { return make_double2(s * a.x, s * a.y); }
__device__ __forceinline__ double2 c_mul(double2 a, double2 b) {
  return make_double2(a.x * b.x - a.y * b.y, a.x * b.y + a.y * b.x);
}
// a + i s b
__device__ __forceinline__ double2 c_addi(double2 a, double s, double2 b) {
  return make_double2(a.x - s * b.y, a.y + s * b.x);
}

// coordinates of flat index f of the N-mode box, 5 bits per mode
__device__ __forceinline__ uint64_t pack_coords(const HGF_CONST FullTables* ft, int64_t f) {
  uint64_t p = 0;
  for (int j = ft->n - 1; j >= 0; --j) {
    const int nc = ft->nc[j];
    p |= (uint64_t)(f % nc) << (5 * j);
    f /= nc;
  }
  return p;
}
__device__ __forceinline__ int coord(uint64_t p, int j) { return (int)((p >> (5 * j)) & 31u); }

// one-sided operator (side 0: Kx; 1: Ky) at flat index f of grid `in`; the
// point's occupations, damping and energy come from the per-point table
__device__ __forceinline__ double2 side_op(const HGF_CONST FullTables* ft, const SepDims& d, int side,
                                           const SepPoint& q, const double2* __restrict__ in, int64_t f) {
  const uint64_t p = q.coords;
  const double sg = side == 0 ? 1.0 : -1.0;
  const double2 c = in[f];
  double2 r = c_addi(c_scale(q.dks - q.g2, c), sg * q.energy, c);
  for (int j = 0; j < ft->n; ++j) {
    const double orr = ft->drive_re[j], oi = ft->drive_im[j];
    if (orr == 0.0 && oi == 0.0) continue;
    const int kj = coord(p, j), nc = ft->nc[j];
    const int64_t s = d.stride[j];
    // x side: i Omega g(k - e) + i conj(Omega) (k + 1) g(k + e)
    // y side: -i conj(Omega) g(l - e) - i Omega (l + 1) g(l + e)
    const double2 om = make_double2(orr, oi), omc = make_double2(orr, -oi);
    if (kj >= 1) r = c_addi(r, sg, c_mul(side == 0 ? om : omc, in[f - s]));
    if (kj + 1 < nc) r = c_addi(r, sg * (double)(kj + 1), c_mul(side == 0 ? omc : om, in[f + s]));
  }
  for (int i = 0; i < ft->n; ++i)
    for (int j = i + 1; j < ft->n; ++j) {
      const double J = ft->exch[i][j];
      if (J == 0.0) continue;
      const int ki = coord(p, i), kj = coord(p, j);
      double2 t = make_double2(0.0, 0.0);
      if (ki >= 1 && kj + 1 < ft->nc[j]) t = c_add(t, c_scale((double)(kj + 1), in[f - d.stride[i] + d.stride[j]]));
      if (kj >= 1 && ki + 1 < ft->nc[i]) t = c_add(t, c_scale((double)(ki + 1), in[f - d.stride[j] + d.stride[i]]));
      r = c_addi(r, sg * J, t);
    }
  return r;
}

// classical RK4 bookkeeping of one element: k is the derivative at this stage
__device__ __forceinline__ void rk4_update(int stage, double h, double2 k, double2* __restrict__ u,
                                           double2* __restrict__ acc, double2* __restrict__ yout, int64_t f,
                                           int& bad) {
  if (stage == 1) {
    const double2 uv = u[f];
    acc[f] = c_add(uv, c_scale(h / 6.0, k));
    yout[f] = c_add(uv, c_scale(0.5 * h, k));
  } else if (stage == 2 || stage == 3) {
    acc[f] = c_add(acc[f], c_scale(h / 3.0, k));
    yout[f] = c_add(u[f], c_scale(stage == 2 ? 0.5 * h : h, k));
  } else {
    const double2 v = c_add(acc[f], c_scale(h / 6.0, k));
    bad |= !(isfinite(v.x) && isfinite(v.y));
    u[f] = v;
  }
}

}  // namespace

// ---- Gx and Gy of every monomial: blockIdx.y is the grid (gx_i for i < M,
// gy_{i - M} otherwise), with its separation constant +C_i or -C_i
__global__ __launch_bounds__(256) void k_sep_sides(const FullTables* __restrict__ ftg,
                                                   const SepPoint* __restrict__ pt, SepDims d, int stage,
                                                   double h, const double2* __restrict__ cst, double2* __restrict__ u,
                                                   double2* __restrict__ acc, const double2* __restrict__ yin,
                                                   double2* __restrict__ yout, int* __restrict__ flag) {
  const HGF_CONST FullTables* ft = (const HGF_CONST FullTables*)ftg;
  const int g = blockIdx.y;
  const int side = g < d.nmono ? 0 : 1;
  const double2 cg = cst[g];
  const int64_t base = (int64_t)g * d.dim;
  int bad = 0;
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < d.dim; f += (int64_t)gridDim.x * blockDim.x) {
    const double2* in = (stage == 1 ? u : yin) + base;
    double2 k = side_op(ft, d, side, pt[f], in, f);
    k = c_add(k, c_mul(cg, in[f]));
    rk4_update(stage, h, k, u + base, acc + base, yout + base, f, bad);
  }
  if (bad) atomicOr(flag, 1);
}

// ---- source of the diagonal R: S(m) = sum_i c_i Gx_i(m) Gy_i(m) at the stage
// inputs (the diagonal of sum_i c_i Gx_i Gy_i).  The grids are small (D
// points) and the monomials many, so a workgroup of 16 wavefronts takes 64
// points: wavefront w sums monomials w, w + 16, ... in order, and the 16
// partial sums are added in wavefront order (deterministic).
constexpr int kSdiagWaves = 16;
__global__ __launch_bounds__(64 * kSdiagWaves) void k_sep_sdiag(SepDims d, const double2* __restrict__ coef,
                                                                const double2* __restrict__ x,
                                                                double2* __restrict__ s) {
  __shared__ double2 part[kSdiagWaves][64];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t m = (int64_t)blockIdx.x * 64 + lane;
  double2 a = make_double2(0.0, 0.0);
  if (m < d.dim)
    for (int i = w; i < d.nmono; i += kSdiagWaves)
      a = c_add(a, c_mul(coef[i], c_mul(x[(int64_t)i * d.dim + m], x[(int64_t)(d.nmono + i) * d.dim + m])));
  part[w][lane] = a;
  __syncthreads();
  if (w == 0 && m < d.dim) {
    double2 t = part[0][lane];
    for (int q = 1; q < kSdiagWaves; ++q) t = c_add(t, part[q][lane]);
    s[m] = t;
  }
}

// ---- source of the whole-box R: S(K, L) = sum_i c_i Gx_i(K) Gy_i(L), an
// outer-product sum (a complex matrix product over the monomials), in tiles
// of 16 x 16 outputs staged through LDS
__global__ __launch_bounds__(256) void k_sep_souter(SepDims d, const double2* __restrict__ coef,
                                                    const double2* __restrict__ x, double2* __restrict__ s) {
  __shared__ double2 A[16][17], B[16][17];
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  const int64_t K = (int64_t)blockIdx.y * 16 + ty, L = (int64_t)blockIdx.x * 16 + tx;
  double2 a = make_double2(0.0, 0.0);
  for (int i0 = 0; i0 < d.nmono; i0 += 16) {
    // A[ii][kk] = c_{i0+ii} Gx_{i0+ii}(K0 + kk), B[ii][ll] = Gy_{i0+ii}(L0 + ll)
    {
      const int ii = ty, kk = tx;
      const int i = i0 + ii;
      const int64_t Kr = (int64_t)blockIdx.y * 16 + kk, Lr = (int64_t)blockIdx.x * 16 + kk;
      A[ii][kk] = (i < d.nmono && Kr < d.dim) ? c_mul(coef[i], x[(int64_t)i * d.dim + Kr]) : make_double2(0.0, 0.0);
      B[ii][kk] = (i < d.nmono && Lr < d.dim) ? x[(int64_t)(d.nmono + i) * d.dim + Lr] : make_double2(0.0, 0.0);
    }
    __syncthreads();
#pragma unroll 4
    for (int ii = 0; ii < 16; ++ii) a = c_add(a, c_mul(A[ii][ty], B[ii][tx]));
    __syncthreads();
  }
  if (K < d.dim && L < d.dim) s[K * d.dim + L] = a;
}

// ---- R on the diagonal: derivative (Kx + Ky + P) R + P S restricted to
// k = l (the drive and exchange shifts leave the diagonal and are dropped;
// the dephasing terms of Kx + Ky and P cancel on R there)
__global__ __launch_bounds__(256) void k_sep_rz(const FullTables* __restrict__ ftg, const SepPoint* __restrict__ pt,
                                                SepDims d, int stage, double h,
                                                const double2* __restrict__ src, double2* __restrict__ u,
                                                double2* __restrict__ acc, const double2* __restrict__ yin,
                                                double2* __restrict__ yout, int* __restrict__ flag) {
  const HGF_CONST FullTables* ft = (const HGF_CONST FullTables*)ftg;
  const double2* in = stage == 1 ? u : yin;
  int bad = 0;
  for (int64_t m = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; m < d.dim; m += (int64_t)gridDim.x * blockDim.x) {
    const uint64_t p = pt[m].coords;
    double2 k = c_scale(2.0 * pt[m].dks, in[m]);
    for (int j = 0; j < ft->n; ++j) {
      const int mj = coord(p, j), nc = ft->nc[j];
      const int64_t s = d.stride[j];
      if (mj >= 1) k = c_add(k, c_scale(ft->adn[j][ft->secular ? mj : 0], c_add(in[m - s], src[m - s])));
      if (mj + 1 < nc) {
        const double b = ft->secular ? ft->aup[j][mj] : ft->aup[j][0] * (double)((mj + 1) * (mj + 1));
        k = c_add(k, c_scale(b, c_add(in[m + s], src[m + s])));
      }
      if (ft->gphi[j] != 0.0) k = c_add(k, c_scale(2.0 * ft->gphi[j] * (double)(mj * mj), src[m]));
    }
    rk4_update(stage, h, k, u, acc, yout, m, bad);
  }
  if (bad) atomicOr(flag, 1);
}

// ---- R on the whole (k, l) box: the full generator on R plus P on S
__global__ __launch_bounds__(256) void k_sep_rfull(const FullTables* __restrict__ ftg, const SepPoint* __restrict__ pt,
                                                   SepDims d, int stage,
                                                   double h, const double2* __restrict__ src,
                                                   double2* __restrict__ u, double2* __restrict__ acc,
                                                   const double2* __restrict__ yin, double2* __restrict__ yout,
                                                   int* __restrict__ flag) {
  const HGF_CONST FullTables* ft = (const HGF_CONST FullTables*)ftg;
  const double2* in = stage == 1 ? u : yin;
  const int64_t D = d.dim, tot = D * D;
  int bad = 0;
  for (int64_t f = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; f < tot; f += (int64_t)gridDim.x * blockDim.x) {
    const int64_t K = f / D, L = f - K * D;
    const uint64_t pk = pt[K].coords, pl = pt[L].coords;
    double dr = 0.0;
    for (int j = 0; j < ft->n; ++j) {
      const int kj = coord(pk, j), lj = coord(pl, j);
      dr += ft->dk[j][kj] + ft->dk[j][lj] - ft->gphi[j] * (double)((kj - lj) * (kj - lj));
    }
    double2 k = c_addi(c_scale(dr, in[f]), pt[K].energy - pt[L].energy, in[f]);
    for (int j = 0; j < ft->n; ++j) {
      const int kj = coord(pk, j), lj = coord(pl, j), nc = ft->nc[j];
      const int64_t s = d.stride[j];
      if (!ft->secular || kj == lj) {
        if (kj >= 1 && lj >= 1)
          k = c_add(k, c_scale(ft->adn[j][ft->secular ? kj : 0], c_add(in[f - s * D - s], src[f - s * D - s])));
        if (kj + 1 < nc && lj + 1 < nc) {
          const double b = ft->secular ? ft->aup[j][kj] : ft->aup[j][0] * (double)((kj + 1) * (lj + 1));
          k = c_add(k, c_scale(b, c_add(in[f + s * D + s], src[f + s * D + s])));
        }
      }
      if (ft->gphi[j] != 0.0) k = c_add(k, c_scale(2.0 * ft->gphi[j] * (double)(kj * lj), src[f]));
      const double orr = ft->drive_re[j], oi = ft->drive_im[j];
      if (orr != 0.0 || oi != 0.0) {
        const double2 om = make_double2(orr, oi), omc = make_double2(orr, -oi);
        if (kj >= 1) k = c_addi(k, 1.0, c_mul(om, in[f - s * D]));
        if (kj + 1 < nc) k = c_addi(k, (double)(kj + 1), c_mul(omc, in[f + s * D]));
        if (lj >= 1) k = c_addi(k, -1.0, c_mul(omc, in[f - s]));
        if (lj + 1 < nc) k = c_addi(k, -(double)(lj + 1), c_mul(om, in[f + s]));
      }
    }
    for (int i = 0; i < ft->n; ++i)
      for (int j = i + 1; j < ft->n; ++j) {
        const double J = ft->exch[i][j];
        if (J == 0.0) continue;
        const int ki = coord(pk, i), kj = coord(pk, j), li = coord(pl, i), lj = coord(pl, j);
        const int64_t si = d.stride[i], sj = d.stride[j];
        double2 t = make_double2(0.0, 0.0);
        if (ki >= 1 && kj + 1 < ft->nc[j]) t = c_add(t, c_scale((double)(kj + 1), in[f + (sj - si) * D]));
        if (kj >= 1 && ki + 1 < ft->nc[i]) t = c_add(t, c_scale((double)(ki + 1), in[f + (si - sj) * D]));
        if (li >= 1 && lj + 1 < ft->nc[j]) t = c_sub_(t, c_scale((double)(lj + 1), in[f + sj - si]));
        if (lj >= 1 && li + 1 < ft->nc[i]) t = c_sub_(t, c_scale((double)(li + 1), in[f + si - sj]));
        k = c_addi(k, J, t);
      }
    rk4_update(stage, h, k, u, acc, yout, f, bad);
  }
  if (bad) atomicOr(flag, 1);
}

// ---- readout.  Weights of a product state: wx(k) = prod_j wt[j][k_j] with
// wt = sqrt(k!) conj(c_j(k)) (x side) and sqrt(l!) c_j(l) (y side), per-mode
// tables of 2 * kMaxCutoff entries each (x then y).
__device__ __forceinline__ double2 state_weight(const HGF_CONST FullTables* ft, const double2* __restrict__ wt,
                                                int side, uint64_t p) {
  double2 w = make_double2(1.0, 0.0);
  for (int j = 0; j < ft->n; ++j) w = c_mul(w, wt[(2 * j + side) * kMaxCutoff + coord(p, j)]);
  return w;
}

__device__ __forceinline__ double2 block_reduce(double2 v) {
  __shared__ double2 part[4];
  for (int off = 32; off > 0; off >>= 1) {
    v.x += __shfl_down(v.x, off, 64);
    v.y += __shfl_down(v.y, off, 64);
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  if (lane == 0) part[wv] = v;
  __syncthreads();
  double2 t = make_double2(0.0, 0.0);
  if (threadIdx.x == 0)
    for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t = c_add(t, part[i]);
  return t;
}

// partial sums: block b < 2M is the dot of grid b with its side's weights;
// the remaining blocks cover R (rows K of the whole box, or the diagonal)
__global__ __launch_bounds__(256) void k_sep_expect_partial(const FullTables* __restrict__ ftg, SepDims d, int rmode,
                                                            const double2* __restrict__ wt,
                                                            const double2* __restrict__ x,
                                                            const double2* __restrict__ r,
                                                            double2* __restrict__ part) {
  const HGF_CONST FullTables* ft = (const HGF_CONST FullTables*)ftg;
  const int b = blockIdx.x;
  double2 a = make_double2(0.0, 0.0);
  if (b < 2 * d.nmono) {
    const int side = b < d.nmono ? 0 : 1;
    for (int64_t f = threadIdx.x; f < d.dim; f += blockDim.x)
      a = c_add(a, c_mul(state_weight(ft, wt, side, pack_coords(ft, f)), x[(int64_t)b * d.dim + f]));
  } else {
    const int64_t rb = b - 2 * d.nmono, nrb = gridDim.x - 2 * d.nmono;
    if (rmode == 1) {
      for (int64_t m = rb * blockDim.x + threadIdx.x; m < d.dim; m += nrb * blockDim.x) {
        const uint64_t p = pack_coords(ft, m);
        a = c_add(a, c_mul(c_mul(state_weight(ft, wt, 0, p), state_weight(ft, wt, 1, p)), r[m]));
      }
    } else {
      for (int64_t K = rb; K < d.dim; K += nrb) {
        const double2 wk = state_weight(ft, wt, 0, pack_coords(ft, K));
        for (int64_t L = threadIdx.x; L < d.dim; L += blockDim.x)
          a = c_add(a, c_mul(c_mul(wk, state_weight(ft, wt, 1, pack_coords(ft, L))), r[K * d.dim + L]));
      }
    }
  }
  const double2 t = block_reduce(a);
  if (threadIdx.x == 0) part[b] = t;
}

// J = sum_i c_i dot(gx_i) dot(gy_i) + sum of the R partials, in a fixed order
__global__ void k_sep_expect_final(SepDims d, int nparts, const double2* __restrict__ coef,
                                   const double2* __restrict__ part, double2* __restrict__ out) {
  if (threadIdx.x != 0 || blockIdx.x != 0) return;
  double2 a = make_double2(0.0, 0.0);
  for (int i = 0; i < d.nmono; ++i) a = c_add(a, c_mul(coef[i], c_mul(part[i], part[d.nmono + i])));
  for (int b = 2 * d.nmono; b < nparts; ++b) a = c_add(a, part[b]);
  *out = a;
}

// number-basis elements <k|A|l> = sqrt(k! l!) (sum_i c_i gx_i(k) gy_i(l) + R(k, l))
// for k, l below `levels` in every mode: out[row * ln + col], row and col
// the mixed-radix (levels) indices of k and l; fac[j][k] = sqrt(k!)
__global__ __launch_bounds__(256) void k_sep_gather(const FullTables* __restrict__ ftg, SepDims d, int rmode,
                                                    int levels, int64_t ln, const double* __restrict__ fac,
                                                    const double2* __restrict__ coef,
                                                    const double2* __restrict__ x, const double2* __restrict__ r,
                                                    double2* __restrict__ out) {
  const HGF_CONST FullTables* ft = (const HGF_CONST FullTables*)ftg;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < ln * ln; e += (int64_t)gridDim.x * blockDim.x) {
    int64_t row = e / ln, col = e - (e / ln) * ln;
    int64_t K = 0, L = 0;
    double sc = 1.0;
    for (int j = ft->n - 1; j >= 0; --j) {
      const int kj = (int)(row % levels), lj = (int)(col % levels);
      row /= levels;
      col /= levels;
      K += kj * d.stride[j];
      L += lj * d.stride[j];
      sc *= fac[j * kMaxCutoff + kj] * fac[j * kMaxCutoff + lj];
    }
    double2 g = make_double2(0.0, 0.0);
    for (int i = 0; i < d.nmono; ++i)
      g = c_add(g, c_mul(coef[i], c_mul(x[(int64_t)i * d.dim + K], x[(int64_t)(d.nmono + i) * d.dim + L])));
    if (rmode == 0)
      g = c_add(g, r[K * d.dim + L]);
    else if (K == L)
      g = c_add(g, r[K]);
    out[e] = c_scale(sc, g);
  }
}

// initial monomials: x[idx[t]] = 1 (the grids are zero otherwise)
__global__ void k_sep_ones(int64_t n, const int64_t* __restrict__ idx, double2* __restrict__ x) {
  for (int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; t < n; t += (int64_t)gridDim.x * blockDim.x)
    x[idx[t]] = make_double2(1.0, 0.0);
}

// ------------------------------------------------------------ launchers
void launch_sep_ones(int64_t n, const int64_t* idx, double2* x, hipStream_t st) {
  if (n <= 0) return;
  const int b = (int)std::min<int64_t>((n + 255) / 256, 1024);
  hipLaunchKernelGGL(k_sep_ones, dim3(b), dim3(256), 0, st, n, idx, x);
}
void launch_sep_sides(const SepLaunch& L, int stage, double h, const double2* cst, double2* u, double2* acc,
                      const double2* yin, double2* yout, int* flag, hipStream_t st) {
  const int bx = (int)std::min<int64_t>((L.d.dim + 255) / 256, 64);
  hipLaunchKernelGGL(k_sep_sides, dim3(bx, 2 * L.d.nmono), dim3(256), 0, st, L.ft, L.pt, L.d, stage, h, cst, u, acc, yin,
                     yout, flag);
}
void launch_sep_source(const SepLaunch& L, int rmode, const double2* coef, const double2* x, double2* s,
                       hipStream_t st) {
  if (rmode == 1) {
    hipLaunchKernelGGL(k_sep_sdiag, dim3((unsigned)((L.d.dim + 63) / 64)), dim3(64 * kSdiagWaves), 0, st, L.d, coef,
                       x, s);
  } else {
    const int nb = (int)((L.d.dim + 15) / 16);
    hipLaunchKernelGGL(k_sep_souter, dim3(nb, nb), dim3(256), 0, st, L.d, coef, x, s);
  }
}
void launch_sep_r(const SepLaunch& L, int rmode, int stage, double h, const double2* src, double2* u,
                  double2* acc, const double2* yin, double2* yout, int* flag, hipStream_t st) {
  const int64_t tot = rmode == 1 ? L.d.dim : L.d.dim * L.d.dim;
  const int b = (int)std::min<int64_t>((tot + 255) / 256, 4096);
  if (rmode == 1)
    hipLaunchKernelGGL(k_sep_rz, dim3(b), dim3(256), 0, st, L.ft, L.pt, L.d, stage, h, src, u, acc, yin, yout, flag);
  else
    hipLaunchKernelGGL(k_sep_rfull, dim3(b), dim3(256), 0, st, L.ft, L.pt, L.d, stage, h, src, u, acc, yin, yout, flag);
}
int sep_expect_parts(const SepDims& d) { return 2 * d.nmono + 64; }
void launch_sep_expect(const SepLaunch& L, int rmode, const double2* wt, const double2* coef, const double2* x,
                       const double2* r, double2* part, double2* out, hipStream_t st) {
  const int np = sep_expect_parts(L.d);
  hipLaunchKernelGGL(k_sep_expect_partial, dim3(np), dim3(256), 0, st, L.ft, L.d, rmode, wt, x, r, part);
  hipLaunchKernelGGL(k_sep_expect_final, dim3(1), dim3(64), 0, st, L.d, np, coef, part, out);
}
void launch_sep_gather(const SepLaunch& L, int rmode, int levels, int64_t ln, const double* fac, const double2* coef,
                       const double2* x, const double2* r, double2* out, hipStream_t st) {
  const int b = (int)std::min<int64_t>((ln * ln + 255) / 256, 4096);
  hipLaunchKernelGGL(k_sep_gather, dim3(b), dim3(256), 0, st, L.ft, L.d, rmode, levels, ln, fac, coef, x, r, out);
}

}  // namespace hgf
