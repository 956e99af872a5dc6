// Internal structures shared by the host runtime and the HIP kernels.
#pragma once

#include <hip/hip_runtime.h>

#include <complex>
#include <cstdint>
#include <string>
#include <vector>

#include "hgf.h"

namespace hgf {

constexpr int kMaxModes = HGF_MAX_MODES;
constexpr int kMaxCutoff = HGF_MAX_CUTOFF;
// Points of a tile handled by one thread of the tiled stage kernel:
// lane groups of a tile <= kTileRounds * 512.
constexpr int kTileRounds = 8;
// Bytes of the static device scratch of the entry points that allocate
// nothing (hgf_expectation_noalloc); every GPU holds one copy.
constexpr size_t kScratchBytes = (size_t)4 << 20;

using cd = std::complex<double>;

// ------------------------------------------------------------------ errors
struct Error {
  hgf_status code;
  std::string msg;
};
void set_error(hgf_status code, const std::string& msg);
[[noreturn]] void fail(hgf_status code, const std::string& msg);
void hip_check(hipError_t e, const char* what);

// ------------------------------------------------------------------ system
struct System {
  int n = 0;
  int nc[kMaxModes] = {};
  double det[kMaxModes] = {}, kerr[kMaxModes] = {}, g1[kMaxModes] = {}, gphi[kMaxModes] = {},
         nth[kMaxModes] = {};
  double chi[kMaxModes][kMaxModes] = {};
  // HGF_DISS_SECULAR: one emission and one absorption channel per transition
  // n <-> n+1 of each mode, bath occupation nlev[j][n]
  int secular = 0;
  double nlev[kMaxModes][kMaxCutoff] = {};
  // driven, exchange-coupled network: H += Omega_j a_j^+ + conj(Omega_j) a_j
  // + sum_{i<j} J_ij (a_i^+ a_j + a_j^+ a_i); `full` when any is non-zero (the
  // sectors are then coupled and an operator is one full (k, l) grid)
  int full = 0;
  double drive_re[kMaxModes] = {}, drive_im[kMaxModes] = {};
  double exch[kMaxModes][kMaxModes] = {};
};

// Full (k, l) grid of a network operator: g(k, l) = <k|A|l> / sqrt(k! l!) on
// 2N axes, the k and l axes of each mode side by side (k, l of the mode at
// position 0, then position 1, ...), row-major: the (k, l) blocks of the last
// positions are contiguous, so a tile of the last two holds every neighbour
// along their axes.  The modes are placed by coupling (Function::fperm); the
// per-mode tables of the generator are in position order (device copy read
// by the kernels).
constexpr int kMaxFullModes = kMaxModes / 2;
struct FullTables {
  int n, secular;
  int nc[kMaxFullModes];
  double e[kMaxFullModes][kMaxCutoff];    // E_j(k) = Delta_j k + (K_j / 2) k (k - 1)
  double dk[kMaxFullModes][kMaxCutoff];   // minus half the rate out of level k (damping)
  double adn[kMaxFullModes][kMaxCutoff];  // coefficient of g(k - e_j, l - e_j)
  double aup[kMaxFullModes][kMaxCutoff];  // coefficient of g(k + e_j, l + e_j) (Lindblad: per (k+1)(l+1))
  double chi[kMaxFullModes][kMaxFullModes];
  double gphi[kMaxFullModes];
  double drive_re[kMaxFullModes], drive_im[kMaxFullModes];
  double exch[kMaxFullModes][kMaxFullModes];
};

// Separated form (Eqs. (9a)-(9c)): sizes of the N-mode boxes of Gx, Gy (and
// of R's rows and columns), and the number of monomials.
struct SepDims {
  int n;
  int nmono;
  int64_t dim;                       // prod_j Nc_j
  int64_t stride[kMaxFullModes];     // row-major strides of the box (last mode fastest)
};
// Per point of the N-mode box of a separated operator, precomputed on the
// host: the occupations (5 bits per mode), sum_j dk_j(k_j),
// sum_j gamma_phi_j k_j^2 and the energy E(k) with the cross-Kerr products.
struct SepPoint {
  uint64_t coords;
  double dks;
  double g2;
  double energy;
};
// One separated operator's launch arguments: dimensions, the device copy of
// its generator tables and its per-point table.
struct SepLaunch {
  SepDims d;
  const FullTables* ft;
  const SepPoint* pt;
};

// Coefficients of the generator restricted to one occupation-difference
// sector d (Eq. (17) with the dissipators of Eq. (3); derivation in the
// sector form): for grid point m,
//   (L g)(m) = [lam0 + sum_j lam_j(m_j)] g(m)
//            + sum_j [ alpha_j(m_j) g(m - e_j) [m_j >= 1] + beta_j(m_j) g(m + e_j) [m_j + 1 < ext_j] ]
// (alpha_j is the same at every level in the Lindblad form)
struct SectorTables {
  int n = 0;
  int d[kMaxModes] = {};
  int ext[kMaxModes] = {};
  int u[kMaxModes] = {}, v[kMaxModes] = {};  // k = m + u, l = m + v
  cd lam0;
  std::vector<cd> lam[kMaxModes];      // [ext_j]
  std::vector<double> beta[kMaxModes];  // [ext_j]; zero at the top of the axis
  std::vector<double> alpha[kMaxModes]; // [ext_j]; zero at m = 0
  int64_t points() const {
    int64_t p = 1;
    for (int j = 0; j < n; ++j) p *= ext[j];
    return p;
  }
};
SectorTables sector_tables(const System& s, const int* d);
System unit_system(const System& s, int p);  // only parameter p set to 1 (n_th kept)
int num_params(int n);

// spectral-radius bound used for the RK4 stability check
double generator_bound(const SectorTables& t);

// ------------------------------------------------------------------ device layout
// Everything a stage kernel needs to know about one grid; passed by value.
struct GridArgs {
  int n;                    // number of axes
  int nfast;                // trailing axes held inside one tile
  int ext[kMaxModes];
  int64_t stride[kMaxModes];
  int64_t points;
  int64_t tile_points;      // product of the fast extents
  int64_t ntiles;
  int off[kMaxModes];       // start of axis j in the concatenated tables (lam, alpha, beta)
  // tiled stage kernel: the trailing `nfast` axes form one tile held in LDS
  // with a zero halo of one point on each side of every fast axis
  int pstride[4];           // padded LDS strides of the fast axes
  int lds_elems;            // padded tile size in elements
  int cbits;                // bits per packed fast coordinate
  int blocks;               // persistent grid size (0: generic kernel)
  int threads;              // workgroup size of the tiled kernel
  int real;                 // tiled kernel on a real grid (real generator and data)
  int lds_bytes;            // dynamic LDS of the tiled kernel
  int xblock;               // tile order across XCDs: 0 contiguous eighths, B > 0 blocks of B tiles
  int pipe;                 // single-grid kernel issues the loads of the next lane round early
  int occ_cap;              // resident workgroups per CU requested for the persistent grid (0: all that fit)
  int occ_max;              // resident workgroups per CU that fit (registers, LDS, waves)
  int wblock;               // tile walk order: 0 row-major, B >= 2 blocks of B along every slow axis
  const void* tiles;        // per-tile records of the slow-axis terms (tiled kernel)
  const uint32_t* walk;     // tile index at each walk position (NULL: the identity)
  double lam0_re, lam0_im;
  const double2* lam;       // concatenated lam_j(m)
  double phase_slope[kMaxModes];  // Im lam_j(m) = m * phase_slope[j] (linear within a sector)
  int phase_linear;         // the tables have that form (else mixed precision runs the generic kernel)
  const double* beta;       // concatenated beta_j(m)
  const double* alpha;      // concatenated alpha_j(m) (0 at m = 0)
  const float* beta_f;
  const float* alpha_f;
  const FullTables* full;   // network operator on the full (k, l) grid, else NULL
  // tiled stage kernel of a network operator (tiles: the last two modes'
  // (k, l) block; records at `tiles`, walk order at `walk`)
  int fblocks;              // persistent grid size (0: the untiled kernel)
  int fthreads;             // workgroup size
  int flds;                 // dynamic LDS bytes
  int ftile;                // points per tile
  int frec;                 // bytes per tile record
  int fwblock;              // walk order: 0 row-major, B >= 2 blocks of B along every slow axis
  int fwgs;                 // resident workgroups per CU requested (0: all that fit)
  int64_t fntiles;          // tiles
};

// Per-tile record of a network operator's tiled stage kernel (host-built, read
// with scalar loads), followed by `nterms` FullTerm entries: the slow modes'
// part of the diagonal (real: damping and dephasing; imaginary: E(k) - E(l)
// with the cross-Kerr products among slow modes), the cross-Kerr sums that
// multiply the fast coordinates (ck[m] = sum_i chi_{i,P+m} k_i over slow i,
// cl[m] the same with l_i), and the neighbour terms that leave the tile.
struct FullTileRec {
  double lam_re, lam_im;
  double ck[2], cl[2];
  int32_t nterms, pad;
};
// One neighbour term: element offset from the point (slow and fast shifts),
// complex coefficient, and an optional shift of one fast axis (meta bits 0-1:
// axis k_P, l_P, k_Q, l_Q; kFullShift: a shift is present; kFullUp: +1, else
// -1; kFullFactor: the coefficient takes the factor (x + 1) of that axis'
// coordinate x).  The kernel drops the term where the shifted coordinate
// leaves the grid.
struct FullTerm {
  int32_t off;
  int32_t meta;
  double cr, ci;
};
constexpr int32_t kFullShift = 4, kFullUp = 8, kFullFactor = 16;

// Bits per fast coordinate in the tiled kernels' per-position words (16 bits
// hold NF coordinates): 4 for four fast axes (extents <= 16), else 5.
__host__ __device__ constexpr int tile_coord_bits(int nf) { return nf == 4 ? 4 : 5; }

// LDS carve-up of the tiled stage kernels, shared by the host (sizing) and
// the kernels (pointers), in bytes from the start of dynamic LDS: the padded
// tile (lds_elems stage elements of `ts` bytes), the per-position diagonal
// rate (T stage elements, 16-byte aligned), the per-position slot and
// coordinate words (T uint32, rounded up to an even count), and the fast
// axes' beta and alpha tables (esum values of `rs` bytes each), plus slack.
struct TiledLds {
  int lam_at, info_at, btab_at, bytes;
};
__host__ __device__ inline TiledLds tiled_lds(int lds_elems, int T, int esum, int ts, int rs) {
  TiledLds l;
  l.lam_at = (lds_elems * ts + 15) & ~15;
  l.info_at = l.lam_at + T * ts;
  l.btab_at = l.info_at + ((T + 1) & ~1) * 4;
  l.bytes = l.btab_at + 2 * esum * rs + 64;
  return l;
}

// Arguments of one member of a grouped (tiled) stage launch, kept in device
// memory: the member's grid, its buffers per stage and its step size.
struct MemberArgs {
  GridArgs g;
  const void* in[4];  // stencil input of stages 1..4
  const void* x1;     // X1 (stages 2..4)
  void* y;            // state
  void* yf;           // stage-precision copy of y (mixed) or NULL
  void* out[4];       // output of stages 1..3 (stage 4 writes y)
  double h;
  int64_t tile_begin;  // first tile of the member in the group's tile space
};

// One function integrated on chip by the resident kernel (the whole grid is
// one LDS tile): its grid, state buffers, step count and step size.
struct ResidentItem {
  GridArgs g;
  void* y;   // state
  void* yf;  // stage-precision copy of y (mixed) or NULL
  void* x1;  // network operators: X1 of the current step (the function's stage grid)
  int steps;
  double h;
  void* rec;  // complex FP64 only, or NULL: step s's y, X1, V1, V2 written at rec + 4 s P (the gradient's records)
};

// One grid of a batched checkpoint copy: the state y and the checkpoint array
// (checkpoint c of `points` complex values at ckpt + c points).
struct CheckpointItem {
  double2* y;
  double2* ckpt;
  int64_t points;
};

// One function's reverse sweep over a segment of the discrete adjoint, on chip
// (complex FP64): the transposed generator's layout and tables, the adjoint
// state, the segment's forward records (step i's y, X1, V1, V2 at
// seg + 4 i P) and the accumulator planes (1 + 2N planes of P points).
struct AdjointResidentItem {
  GridArgs g;
  void* mu;
  const void* seg;
  void* Q;
  int steps;
  double h;
};

// One resident launch: one workgroup per item, items sharing the number of
// axes and element types.
struct ResidentLaunch {
  const ResidentItem* items;  // device array
  int count;
  int nfast, threads, lds_bytes;  // network operators (full = 1): nfast is the number of modes
  int real, precision;
  int full;
};

// One grouped launch: members sharing the axis split and element types.
struct GroupLaunch {
  MemberArgs single;          // the member itself when nmem == 1 (passed by value)
  const MemberArgs* members;  // device array
  int nmem;
  int64_t total_tiles;
  int nfast, nslow, threads, lds_bytes, blocks;
  int real, precision;
};

// ------------------------------------------------------------------ functions
struct Function {
  SectorTables tab;
  GridArgs ga{};
  // device buffers (owned)
  void* y = nullptr;   // complex128 state
  void* ybak = nullptr;  // complex128 copy of y taken at the start of each evolve
  void* s1 = nullptr;  // stage buffers: complex128 (FP64) or complex64 (MIXED)
  void* s2 = nullptr;
  void* s3 = nullptr;
  void* s4 = nullptr;  // classical (split) form only: RK accumulator, complex128
  void* yf = nullptr;  // mixed precision: complex64 copy of y, the stencil input of stage 1
  void* dtab = nullptr;  // device tables
  void* ttab = nullptr;  // per-tile records of the tiled stage kernel
  // split mode
  bool split = false;
  bool real = false;  // real generator and data: real grids, half the bytes
  int p[kMaxModes] = {}, q[kMaxModes] = {};
  int64_t mono_index = 0;  // flat index of (p, q) in the grid
  cd g0 = 0.0, cx = 1.0, cy = 1.0;
  cd ax = 0.0, ay = 0.0;   // dc_x/dt = ax c_x, dc_y/dt = ay c_y
  std::vector<std::pair<int64_t, cd>> sources;  // R' = L R + c_x c_y S
  double tuned_us = 0.0;  // stage time measured by the autotuner for the current shape
  bool resident = false;  // integrated on chip by the resident kernel
  int res_threads = 0;    // workgroup size of the resident kernel
  int res_lds_bytes = 0;  // its LDS (two padded copies of the grid)
  GridArgs rga{};         // the resident kernel's layout (ga with every axis in LDS)
  bool precision_fp64 = false;
  // integrating-factor scheme: per-axis factors exp(lam_j(m) h/2) on the
  // device (concatenated like lam), exp(lam0 h/2), and the h they are for
  void* ehtab = nullptr;
  cd eh0 = 0.0;
  double eh_h = 0.0;
  // network operator: one full (k, l) grid, generator tables in ftab
  bool full = false;
  void* ftab = nullptr;
  double full_bound = 0.0;  // bound on the spectral radius of its generator
  int fperm[kMaxFullModes] = {};   // mode held at each position of the grid (slowest first)
  std::vector<FullTables> fhost;   // host copy of the tables (one entry), in position order
};

struct StepPlan;
struct SepState;

}  // namespace hgf

struct hgf_system_s {
  hgf::System sys;
};

struct hgf_operator_s {
  hgf::System sys;
  int precision = HGF_FP64;
  int layout = HGF_MERGED;
  int device = 0;
  std::vector<hgf::Function> fn;
  int64_t steps_done = 0;
  double time_us = 0.0;
  int64_t underflow = 0;
  int error_state = 0;
  int* dflag = nullptr;  // device non-finite flag
  // launch plan and cached graph of merged-mode steps
  hgf::StepPlan* plan = nullptr;
  void* graph_exec = nullptr;
  int graph_steps = 0;
  double graph_dt = 0.0;
  hipStream_t cap_stream = nullptr;
  // separated layout (Eqs. (9a)-(9c)): the monomials' Gx, Gy grids and R
  hgf::SepState* sep = nullptr;
  // thresholded representation (hgf_set_threshold): coefficients with
  // |g| <= threshold are dropped after every step; device counters of the
  // survivors (count of the last step, peak since the threshold was set)
  double threshold = 0.0;
  unsigned long long* dcount = nullptr;  // [4]: count, peak, tile count, tile peak
};
