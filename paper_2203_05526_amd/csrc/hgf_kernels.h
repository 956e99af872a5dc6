// Launch wrappers for the HIP kernels (host-callable).
#pragma once

#include <hip/hip_runtime.h>

#include "hgf_internal.h"

namespace hgf {

// Digits of a grid-stride loop's stride in the grid's mixed radix.
struct StrideDigits {
  int64_t total;
  int digit[kMaxModes];
};

struct LaunchShape {
  int blocks;
  int threads;
};

// Point sources of the split layout: K(m) += scale * value at up to
// kMaxSources grid points.
constexpr int kMaxSources = 2 * kMaxModes + 1;
struct PointSources {
  int count;
  int64_t index[kMaxSources];
  double re[kMaxSources], im[kMaxSources];
  double scale_re, scale_im;
};

LaunchShape shape_for(const GridArgs& g, int max_blocks);

void launch_horner(int stage, int precision, const GridArgs& g, const void* in, const void* x1, void* y, void* yf,
                   void* out, double h, int* flag, hipStream_t st);
void launch_shadow(int precision, const GridArgs& g, const void* y, void* yf, hipStream_t st);
// Integrating-factor RK4 over many functions in one launch per stage (all the
// functions of an operator that share element types): one row of blocks per
// function, device array of items.
struct LawsonItem {
  GridArgs g;
  StrideDigits sd;     // loop stride: (blocks per row) * threads
  void* y;             // state
  void* yf;            // stage-precision copy of y (mixed) or NULL
  void* s1;            // v2, then v4
  void* s2;            // v3
  void* s3;            // the step's increment
  const double2* eh;   // per-axis exp(lam_j(m) h/2)
  double2 e0;          // exp(lam0 h/2)
};
void launch_lawson_group(int stage, int precision, bool real, const LawsonItem* items, int nitems, int row_blocks,
                         double h, int* flag, hipStream_t st);
int lawson_row_blocks(const GridArgs& g);
StrideDigits lawson_row_digits(const GridArgs& g, int row_blocks);
// Horner RK4 stage of a network operator on its full (k, l) grid (g.full set).
void launch_full_horner(int stage, int precision, const GridArgs& g, const void* in, const void* x1, void* y,
                        void* yf, void* out, double h, int* flag, hipStream_t st);
// Tiled form of the same stage (g.fblocks > 0): persistent grid, tile records
// at g.tiles; its LDS bytes for a tile of `tile_points`, its lane-round limit
// and its resident workgroups per CU.
void launch_full_tiled(int stage, int precision, const GridArgs& g, const void* in, const void* x1, void* y,
                       void* yf, void* out, double h, int* flag, hipStream_t st);
size_t full_tiled_lds_bytes(int precision, int tile_points);
int full_tiled_max_rounds();
int full_tiled_blocks_per_cu(int precision, int threads, int lds_bytes);
// form: 0 grouped kernel, 1 single-grid kernel, 2 single-grid pipelined kernel
int tiled_max_blocks_per_cu(int nfast, int nslow, int threads, int precision, int lds_bytes, bool real,
                            int form);
int tiled_max_slow_axes();
int tiled_max_lane_groups();
void launch_group(const GroupLaunch& gl, int stage, int* flag, hipStream_t st);
// resident (on-chip, many-step) integrator; grids of at most this many points
// lane rounds of the resident kernel's workgroup (1024 lanes, 512 in FP64)
int resident_max_rounds(bool fp64, bool real);
// LDS a resident workgroup may take: the CU's 160 KB on gfx950
constexpr int kResidentLdsMax = 160 * 1024;
// set the resident kernels' dynamic-LDS limit (for a function's element
// types) to `bytes`; a host call, made outside graph capture
hipError_t resident_allow_lds(bool real, int precision, int bytes);
// the gradient's on-chip segment kernels (complex FP64; csrc/hgf_resident.h):
// the recording forward integrator (items' rec set) and the reverse sweep,
// `count` items of `nf` axes, one workgroup of `threads` lanes and `lds` bytes
// each; grad_resident_allow_lds raises their dynamic-LDS limit (host call)
hipError_t grad_resident_allow_lds(int bytes);
void launch_grad_record(const ResidentItem* items, int count, int nf, int threads, int lds, int* flag,
                        hipStream_t st);
void launch_grad_reverse(const AdjointResidentItem* items, int count, int nf, int threads, int lds, int* flag,
                         hipStream_t st);
void launch_resident(const ResidentLaunch& rl, int* flag, hipStream_t st);
void launch_classical(int stage, int precision, const GridArgs& g, const void* in, void* y, void* acc, void* next,
                      double h, const PointSources& src, int* flag, hipStream_t st);
int expect_blocks(const GridArgs& g);
void launch_expect_partial(const GridArgs& g, const void* grid, bool grid_fp64, const double2* wtab,
                           double2* partial, hipStream_t st, bool real = false);
void launch_expect_final(const double2* partial, const int* start, const double2* coef, int nfun,
                         double2 analytic, double2* out, hipStream_t st);
// completes Xb1 of a reverse step in place and copies mu into mu_copy
void launch_adjoint_x(int64_t n, const double2* mu, const double2* vb2, const double2* vb1, double2* xb1,
                      double2* mu_copy, hipStream_t st);
// parameter products of a reverse step (Xb1 complete)
void launch_adjoint_q(const GridArgs& g, const double2* mu, const double2* vb2, const double2* vb1,
                      const double2* xb1, const double2* v2, const double2* v1, const double2* x1,
                      const double2* y, double2* Q, double h, hipStream_t st);
// parameter products of a reverse segment of L steps: step i's adjoint set
// (Vb2, Vb1, Xb1, mu) at adj + 4 i points, its grids (y, X1, V1, V2) at
// fwd + 4 i points
void launch_adjoint_q_segment(const GridArgs& g, const double2* adj, const double2* fwd, int L, double2* Q, double h,
                              hipStream_t st);
int marginal_bins(const GridArgs& g);
void launch_marginals(const GridArgs& g, const double2* Q, double2* bins, hipStream_t st);
void launch_fill_zero(double2* p, int64_t n, hipStream_t st);
// Number-basis matrix elements of one function on the lowest levels of every
// mode: the sub-box m_a < b[a] of the grid, scattered to out[row * ln + col]
// with row = sum_a (m_a + ur[a]) rp[a] and col = sum_a (m_a + uc[a]) cp[a]
// (a sector axis adds to both, a full grid's k axis to the row only and its l
// axis to the column only).
struct GatherBox {
  int b[kMaxModes];        // sub-box extents
  int ur[kMaxModes], uc[kMaxModes];
  int foff[kMaxModes];     // start of axis a in the factor table (sqrt(k! l!) per point)
  int64_t rp[kMaxModes], cp[kMaxModes];
  int64_t ln;              // levels^N: the output's row length
  int64_t total;           // prod_j b[j]
  int64_t pq;              // grid index that gets `add` (split layout), or -1
  double2 add;             // separable part at (p, q) (split layout)
  double2 coef;            // overall factor (g0 in split layout, else 1)
};
void launch_gather_levels(const GridArgs& g, const void* y, bool real, const GatherBox& box, const double* fac,
                          double2* out, hipStream_t st);
// device-to-device copy as a kernel (safe to record in a captured graph)
void launch_copy2(double2* dst, const double2* src, int64_t n, hipStream_t st);
// checkpoint c of `count` grids in one launch: states into it (to_ckpt) or
// restored from it; max_points: the largest grid
void launch_checkpoint_batch(const CheckpointItem* items, int count, int64_t max_points, int64_t c, bool to_ckpt,
                             hipStream_t st);
void launch_fill_weights(const GridArgs& g, const double2* wtab, double2* out, hipStream_t st);
// Separated form (Eqs. (9a)-(9c)), classical RK4 stage by stage: every
// monomial's Gx and Gy (with +-C), the source P(sum_i c_i Gx_i Gy_i) of R
// (rmode 1: its diagonal products; 0: the whole outer-product sum), and R
// (rmode 1: on the diagonal k = l; 0: on the whole box); readout.
void launch_sep_sides(const SepLaunch& L, int stage, double h, const double2* cst, double2* u, double2* acc,
                      const double2* yin, double2* yout, int* flag, hipStream_t st);
void launch_sep_source(const SepLaunch& L, int rmode, const double2* coef, const double2* x, double2* s,
                       hipStream_t st);
void launch_sep_r(const SepLaunch& L, int rmode, int stage, double h, const double2* src, double2* u,
                  double2* acc, const double2* yin, double2* yout, int* flag, hipStream_t st);
int sep_expect_parts(const SepDims& d);
void launch_sep_expect(const SepLaunch& L, int rmode, const double2* wt, const double2* coef, const double2* x,
                       const double2* r, double2* part, double2* out, hipStream_t st);
void launch_sep_ones(int64_t n, const int64_t* idx, double2* x, hipStream_t st);
void launch_sep_gather(const SepLaunch& L, int rmode, int levels, int64_t ln, const double* fac, const double2* coef,
                       const double2* x, const double2* r, double2* out, hipStream_t st);
// Thresholded representation: zero every coefficient with |g| <= thr and add
// the survivors to *count; then peak = max(peak, count) and count = 0.
// Thresholded representation: zero |g| <= thr in g[0, n) and add the kept
// count to counters[0]; with tile > 0 (n a multiple of it) also add the
// number of tiles of `tile` points that keep a coefficient to counters[2].
// launch_threshold_peak folds counters[0] into the peak counters[1] and
// counters[2] into counters[3], and clears the counts.
void launch_threshold(double2* g, int64_t n, double thr, int64_t tile, unsigned long long* counters,
                      hipStream_t st);
void launch_threshold_peak(unsigned long long* counters, hipStream_t st);
// Device address of the current device's copy of the static scratch
// (kScratchBytes), looked up once per device.
void* scratch_address();

}  // namespace hgf
