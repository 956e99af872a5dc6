/*
 * hgf.h -- C ABI of the MI355X (gfx950) generating-function solver for the
 * adjoint Lindblad master equation of damped, Kerr-coupled bosonic modes.
 *
 * Method (paper: "Efficient classical simulation of open bosonic quantum
 * systems", arXiv:2203.05526):
 *   (i)   an operator A(0) is mapped to the coefficients g_{k,l}(0) of its
 *         transformed generating function G = e^{xy} F (Eqs. (2), (5)-(8));
 *   (ii)  the G equations (Eqs. (9) and (17)-(19)) are integrated with
 *         fourth-order Runge-Kutta, each independent function in parallel;
 *   (iii) the result is read out as <psi0| A(T) |psi0> (Eq. (11) contracted
 *         with a product state).
 * With o1 = a^+, o2 = a (r = 1) the basis element T_{k,l} of Eq. (8) is
 * sqrt(k! l!) |k><l| on the truncated space, so g_{k,l} = <k|A|l>/sqrt(k! l!)
 * per mode.  The physics handled is
 *   H = sum_j [Delta_j n_j + (K_j/2) a_j^+ a_j^+ a_j a_j] + sum_{i<j} chi_ij n_i n_j
 * with, per mode, emission (a_j, rate gamma1_j (1 + n_th_j)), absorption
 * (a_j^+, rate gamma1_j n_th_j) and dephasing (n_j, rate 2 gamma_phi_j) in the
 * Lindblad form of Eq. (3).  Every term then moves k and l together, so the
 * occupation difference d = l - k is conserved and the grid of one function is
 * an N-dimensional box over m_j = min(k_j, l_j), extent Nc_j - |d_j|.
 *
 * Conventions for every entry point:
 *  - Units: time in microseconds, angular frequency in rad/us, rates in 1/us.
 *  - Complex numbers are interleaved (re, im) doubles.
 *  - Arrays of a mode-indexed quantity are ordered by mode 0..N-1.  Grids are
 *    row-major over m with the last mode varying fastest.
 *  - Inputs are copied during the call; the caller keeps its arrays.
 *  - Outputs go to caller-provided buffers.
 *  - Every call returns an hgf_status; nothing is thrown across the ABI.
 *    On error, hgf_last_error() returns a thread-local message and the handle
 *    passed in is left as it was (except as noted for hgf_evolve).
 *  - `hip_stream` is a hipStream_t (NULL means the null stream).  Work is
 *    enqueued on it; calls that return host values synchronise it.
 *  - Handles are not thread-safe; calls on different handles may run on
 *    different threads.
 *
 * Environment (read when an operator is mapped or a gradient is taken; for
 * comparisons and tests, every setting gives the same results to rounding):
 *  - HGF_STAGE_KERNEL=generic: every function runs the untiled stage kernel.
 *  - HGF_RESIDENT=0: no function runs the resident (on-chip) integrator.
 *  - HGF_REAL_GRIDS=0: diagonal-sector functions keep complex grids.
 *  - HGF_GRAD_STORE=0: hgf_grad keeps only the states of a segment and
 *    recomputes each step's stage grids in the reverse sweep (bit-identical).
 *  - HGF_MAX_NFAST=k (1..4): the default launch shape of the tiled stage
 *    kernel takes at most k fast (LDS) axes, so small grids also run with
 *    slow-axis neighbour tiles (the shape large grids take); grids of more
 *    than k axes then also stay off the resident integrator by default.
 */
#ifndef HGF_H
#define HGF_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  HGF_OK = 0,
  HGF_EINVAL = -1,       /* malformed or out-of-range argument */
  HGF_ENOMEM = -2,       /* device or host allocation failed */
  HGF_EDEVICE = -3,      /* a HIP runtime call failed */
  HGF_EUNSTABLE = -4,    /* dt outside the RK4 stability bound of the generator */
  HGF_ENONFINITE = -5,   /* a NaN or Inf appeared in an evolved function */
  HGF_EUNSUPPORTED = -6, /* valid request the library does not implement */
  HGF_ESTATE = -7        /* handle in a state that forbids the call */
} hgf_status;

/* precision of an operator's functions */
enum {
  HGF_FP64 = 0,  /* every grid in complex128, stencil in FP64 */
  HGF_MIXED = 1  /* RK stage grids complex64 with FP32 stencil; state complex128 */
};

/* how an operator's coefficients are grouped into independently evolved functions */
enum {
  HGF_MERGED = 0, /* one grid per occupation-difference sector, initial value the
                     sector's part of G(0) (Eq. (10) summed up front by linearity) */
  HGF_SPLIT = 1,  /* one function per non-negligible g_{p,q}(0): G = Gx Gy + R with
                     Gx = c_x x^p, Gy = c_y y^q, R(0) = 0 (Eqs. (9)-(10), (19)) */
  HGF_SEPARATED = 2,      /* the separated form of Eqs. (9a)-(9c) with Gx(x) and Gy(y) as grids
                             over the N occupations (drive and exchange shift them), one pair
                             per non-negligible g_{p,q}(0), and R restricted to the diagonal
                             k = l: R approximated by a function of the products x_j y_j (the
                             approximation the paper reports for the driven network) */
  HGF_SEPARATED_EXACT = 3 /* the same with R on the whole (k, l) box: exact in continuous time */
};

/* operator input forms */
enum {
  HGF_OP_PRODUCT = 0, /* A = tensor product of per-mode Nc_j x Nc_j matrices */
  HGF_OP_SPARSE = 1,  /* A = sum_t value_t M(k_t, l_t) */
  HGF_OP_DENSE = 2    /* A given entry by entry over the whole truncated space (tiny systems) */
};
enum {
  HGF_BASIS_NUMBER = 0, /* entries are number-basis elements <k|A|l> */
  HGF_BASIS_NORMAL = 1  /* entries are the normal-ordered coefficients f_{k,l} of Eq. (2) */
};

/* product states psi0 = tensor product over modes */
enum {
  HGF_PSI_FOCK = 0,     /* |n_0> x |n_1> x ... */
  HGF_PSI_COHERENT = 1, /* coherent |alpha_j>, truncated to the cutoff and renormalised */
  HGF_PSI_PRODUCT = 2   /* arbitrary per-mode amplitude vectors (used as given) */
};

typedef struct hgf_system_s* hgf_system;
typedef struct hgf_operator_s* hgf_operator;

typedef struct {
  int32_t n_modes;          /* 1 .. HGF_MAX_MODES */
  const int32_t* cutoff;    /* [N] Fock levels kept per mode, 1 .. HGF_MAX_CUTOFF */
  const double* detuning;   /* [N] Delta_j, rad/us */
  const double* kerr;       /* [N] K_j, rad/us */
  const double* cross_kerr; /* [N*N] chi_ij, rad/us, symmetric; the diagonal is ignored */
  const double* gamma1;     /* [N] 1/T1, 1/us, >= 0 */
  const double* gamma_phi;  /* [N] 1/Tphi, 1/us, >= 0 */
  const double* n_th;       /* [N] bath occupation, >= 0 */
  int32_t dissipator;       /* HGF_DISS_LINDBLAD or HGF_DISS_SECULAR */
  const double* n_th_levels; /* SECULAR only, may be NULL: bath occupation of every
                                transition n <-> n+1, sum_j (Nc_j - 1) values, modes in
                                order (NULL: n_th_j for every transition of mode j) */
  /* The driven, exchange-coupled network of Eq. (16), in the frame rotating at
   * the drive frequency (a drive on resonance is static there; Delta_j is the
   * mode's detuning from the drive).  Either may be NULL (none).  When any
   * entry is non-zero the sectors are coupled: every operator is then one
   * function on the full (k, l) grid (2N axes, at most 8 modes and 2^28
   * points), merged layout and HGF_RK4 only, and hgf_grad and
   * hgf_get_function return HGF_EUNSUPPORTED (read it with hgf_reconstruct).
   * The modes are laid out by coupling (the pair with the most drive and
   * exchange terms between them last).  Its stage kernel tiles the (k, l)
   * block of the last two when there are at least three modes, that block
   * holds 256 to 4096 points and the grid at least 256 such tiles (see
   * hgf_set_tile_config); otherwise it runs untiled. */
  const double* drive;      /* [2N] complex Omega_j (re, im), rad/us:
                               H += Omega_j a_j^+ + conj(Omega_j) a_j */
  const double* exchange;   /* [N*N] J_ij, rad/us, symmetric, diagonal ignored:
                               H += sum_{i<j} J_ij (a_i^+ a_j + a_j^+ a_i) */
} hgf_system_desc;

/* dissipators (per mode; dephasing is the Lindblad channel n at rate 2 gamma_phi in both) */
enum {
  HGF_DISS_LINDBLAD = 0, /* emission a at gamma1 (1 + n_th), absorption a^+ at gamma1 n_th (Eq. (3)) */
  HGF_DISS_SECULAR = 1   /* first-principles form of Eq. (15): per transition n <-> n+1,
                            lowering |n><n+1| at gamma1 (n+1)(nbar_n + 1) and raising |n+1><n|
                            at gamma1 (n+1) nbar_n, nbar_n the bath occupation at the
                            transition's frequency; jumps act on populations only */
};

#define HGF_MAX_MODES 16
#define HGF_MAX_CUTOFF 32

/*
 * Validate and copy a system description (the Hamiltonian of Eq. (1) and the
 * dissipators of Eq. (3) or Eq. (15), restricted as above).  Errors:
 * HGF_EINVAL for a NULL pointer, N or a cutoff out of range, a negative or
 * non-finite rate or occupation, a non-symmetric cross_kerr, an unknown
 * dissipator, or n_th_levels given with HGF_DISS_LINDBLAD.  *out is owned by
 * the caller and freed by hgf_destroy_system.
 */
hgf_status hgf_define_system(const hgf_system_desc* desc, hgf_system* out);
void hgf_destroy_system(hgf_system sys);

/* Number of real parameters that hgf_grad differentiates:
 * K[N], chi[i<j lexicographic], Delta[N], gamma1[N], gamma_phi[N]. */
int32_t hgf_num_params(hgf_system sys);

typedef struct {
  int32_t kind;           /* HGF_OP_PRODUCT or HGF_OP_SPARSE */
  int32_t basis;          /* HGF_BASIS_NUMBER or HGF_BASIS_NORMAL */
  const double* values;   /* PRODUCT: the N matrices one after another, each
                             Nc_j x Nc_j row-major complex (2*sum Nc_j^2 doubles);
                             SPARSE: n_terms complex values (2*n_terms doubles);
                             DENSE: D x D row-major complex, D = prod_j Nc_j <= 4096,
                             rows and columns k flattened with the last mode fastest
                             (entry (k, l) is the coefficient of M(k, l)) */
  const int32_t* indices; /* SPARSE only: n_terms rows of 2N ints (k_0..k_{N-1}, l_0..l_{N-1});
                             NUMBER basis: M = |k><l|; NORMAL basis: M = prod_j (a_j^+)^{k_j} a_j^{l_j} */
  int64_t n_terms;        /* SPARSE only */
  int32_t precision;      /* HGF_FP64 or HGF_MIXED */
  int32_t layout;         /* HGF_MERGED or HGF_SPLIT */
  double drop_tol;        /* g_{p,q}(0) with |g| <= drop_tol are dropped (Eqs. (10)-(13)) */
} hgf_operator_desc;

/*
 * Step (i): map A(0) to its set of functions and place them on the current
 * device.  Coefficients follow g_{k,l} = <k|A|l>/sqrt(k! l!) per mode, or
 * Eq. (6) from normal-ordered f.  Functions are grouped by sector d = l - k
 * (merged) or one per coefficient (split).  Errors: HGF_EINVAL (bad kind,
 * basis, layout, precision, index out of the cutoff box, NULL arrays),
 * HGF_ENOMEM, HGF_EDEVICE.  The operator keeps its own copy of the system.
 */
hgf_status hgf_map_operator(hgf_system sys, const hgf_operator_desc* desc, hgf_operator* out);
void hgf_destroy_operator(hgf_operator op);

/* time-stepping schemes of hgf_evolve */
enum {
  HGF_RK4 = 0,       /* classical fourth-order Runge-Kutta with a fixed step (the paper's scheme) */
  HGF_LAWSON_RK4 = 1 /* integrating-factor RK4: the diagonal part of the generator (phases,
                        damping, dephasing) taken exactly, the jump terms by classical RK4 in
                        its interaction picture; merged layout only */
};

/*
 * Step (ii): advance every function of the operator by t_total_us with
 * fixed steps of dt_us (Heisenberg picture: A(0) -> A(t)) of the given
 * scheme: HGF_RK4, or HGF_LAWSON_RK4, whose step is exact without jumps and so
 * is not limited by large Kerr phases in off-diagonal sectors (every function
 * then runs on the untiled stage kernel).  Other values: HGF_EUNSUPPORTED, as
 * is HGF_LAWSON_RK4 on a split-layout or a network operator.
 * t_total_us / dt_us must be a non-negative integer (to 1e-9 relative).
 * Errors: HGF_EINVAL; HGF_EUNSTABLE when dt times a bound on the spectral
 * radius of the generator (HGF_RK4) or of its jump terms (HGF_LAWSON_RK4)
 * leaves the RK4 stability region (nothing is run);
 * HGF_ENONFINITE when a NaN/Inf appears (the functions are restored to the
 * last state checked finite and the operator moves to an error state in which
 * further evolves return HGF_ESTATE until hgf_clear_error); HGF_EDEVICE.
 */
hgf_status hgf_evolve(hgf_operator op, double t_total_us, double dt_us, int32_t scheme, void* hip_stream);

/*
 * Batched form of hgf_evolve: every member advances by its own t_total/dt
 * (arrays of n), all members' RK stages issued as one grouped launch per
 * stage and captured in a HIP graph.  Members must be distinct handles on the
 * same device with the layout HGF_MERGED.  Errors as for hgf_evolve, and
 * HGF_EUNSUPPORTED for a member with a threshold (hgf_set_threshold); on
 * error no member has been advanced.
 */
hgf_status hgf_evolve_batch(hgf_operator* ops, int32_t n, const double* t_total_us,
                            const double* dt_us, void* hip_stream);

typedef struct {
  int32_t kind;         /* HGF_PSI_FOCK, HGF_PSI_COHERENT or HGF_PSI_PRODUCT */
  const int32_t* fock;  /* FOCK: [N] occupations, each below the cutoff */
  const double* alpha;  /* COHERENT: [2N] complex alpha_j */
  const double* amps;   /* PRODUCT: per-mode amplitude vectors, complex, 2*sum Nc_j doubles */
} hgf_state_desc;

/*
 * Step (iii): out_re_im = <psi0| A(t) |psi0> for a product state, summed over
 * every function with FP64 accumulation (Eq. (11) contracted with psi0; in
 * split mode the separable part c_x c_y x^p y^q is added analytically; in the
 * separated layouts sum_i g_i <Gx_i> <Gy_i> + <R>).
 * Errors: HGF_EINVAL, HGF_EDEVICE.  Synchronises hip_stream.
 */
hgf_status hgf_expectation(hgf_operator op, const hgf_state_desc* psi, double out_re_im[2],
                           void* hip_stream);

/*
 * hgf_expectation for callers that cannot allocate device memory (code under
 * HIP graph capture, tight serving loops, harnesses that forbid hipMalloc):
 * the same result, computed by the same kernels, with every device buffer of
 * the call (weight tables, partial sums, result) taken from a static device
 * array of 4 MiB that each GPU holds from the library's first use until the
 * process ends.  No hipMalloc, hipFree or allocating library routine is
 * called.  Operators whose buffers need more than 4 MiB (weight tables of
 * sum_j extent_j complex values per function plus one partial sum per
 * workgroup, at most 2048 per function: roughly a few hundred large functions
 * or a few thousand small ones) are refused with HGF_EINVAL; hgf_expectation
 * serves them.  Calls on one GPU share its array: calls that overlap in time
 * on one GPU (several threads, or streams running concurrently) race and
 * must be serialised by the caller.  Errors as for hgf_expectation, and
 * HGF_EUNSUPPORTED for the separated layouts (read through hgf_expectation).
 */
hgf_status hgf_expectation_noalloc(hgf_operator op, const hgf_state_desc* psi, double out_re_im[2],
                                   void* hip_stream);

/*
 * Step (iii) at the operator level: the number-basis matrix elements
 * <k|A(t)|l> (Eq. (11): the generating-function coefficients g_{k,l} of the
 * evolved operator times sqrt(k! l!), with o1 = a^+, o2 = a, r = 1) for every
 * k, l whose occupations are all below `levels`, as a dense row-major matrix:
 * row index sum_j k_j * levels^(N-1-j) (last mode fastest), column index the
 * same for l.  out receives 2 * levels^(2N) doubles (re, im), owned by the
 * caller; elements of sectors the operator does not hold are 0.  In split
 * layout each function contributes g0 (c_x c_y x^p y^q + R).  levels = 3 gives
 * the three-level truncation on which the paper measures operator errors.
 * Errors: HGF_EINVAL (NULL, levels outside [1, every cutoff], levels^(2N) above
 * 2^24), HGF_EDEVICE.  Synchronises hip_stream.
 */
hgf_status hgf_reconstruct(hgf_operator op, int32_t levels, double* out, void* hip_stream);

/*
 * Gradient of J = <psi0| A(T) |psi0> with respect to every parameter of
 * hgf_num_params, by a discrete adjoint (reverse) sweep of the RK4 steps over
 * checkpoints taken every `checkpoint_every` steps, in FP64 and merged layout
 * (desc->precision and desc->layout are ignored).  value_out receives J,
 * grad_out 2*hgf_num_params doubles (complex dJ/dtheta; real for Hermitian A).
 * Device memory per sector of P points (16 P bytes a grid): the checkpoints
 * (T / (checkpoint_every dt) + 1 grids) and, when a segment's states and
 * stage grids fit in 2 GiB, one segment buffer of 4 checkpoint_every grids
 * (two when there are several segments: the next is recomputed beside the
 * sweep) and the segment's adjoint grids (4 checkpoint_every more); else one
 * buffer of checkpoint_every states (the stages are then recomputed).
 * Errors: HGF_EINVAL, HGF_EUNSTABLE, HGF_ENOMEM, HGF_EDEVICE, HGF_ENONFINITE.
 */
hgf_status hgf_grad(hgf_system sys, const hgf_operator_desc* desc, const hgf_state_desc* psi,
                    double t_total_us, double dt_us, int32_t checkpoint_every, double value_out[2],
                    double* grad_out, void* hip_stream);

typedef struct {
  int32_t n_functions;
  int32_t precision;
  int32_t layout;
  int32_t n_modes;
  int64_t total_points;   /* sum of grid points over functions */
  int64_t steps_done;     /* RK4 steps taken so far */
  double time_us;         /* t reached so far */
  int64_t fp32_underflow; /* MIXED: nonzero initial coefficients below FP32's normal range */
  int32_t error_state;    /* nonzero after HGF_ENONFINITE */
  int32_t real_functions; /* functions held as real grids (real generator and data) */
  int64_t stored_peak;    /* with a threshold set (hgf_set_threshold): the largest number of
                             coefficients kept after any step since it was set; else -1 */
  int32_t untiled_functions; /* merged and network layouts: functions whose RK4 stages run on the
                                untiled grid-stride kernel because the tiled one does not take
                                them (a tile beyond LDS, more than 12 slow axes, a buffer over
                                2^32 bytes, or HGF_STAGE_KERNEL=generic); several times slower */
  int32_t reserved;
  int64_t stored_tiles_peak; /* with a threshold set: the largest number of tiles (runs of tile_points
                                consecutive coefficients) holding a kept coefficient after any step,
                                the units a sparse store would skip whole; else -1 */
  int64_t tile_points;       /* network operators: the stage kernel's tile on the full grid (the (k, l)
                                block of the two fastest modes, the whole grid below three modes);
                                separated layouts: one grid of prod_j Nc_j points; else 0 */
} hgf_operator_info;

hgf_status hgf_get_info(hgf_operator op, hgf_operator_info* info);

/*
 * Thresholded representation of the operator (the paper's truncation of the
 * stored representation, tuned in its network example to a fixed operator
 * error): after every RK4 step of hgf_evolve, every stored generating-function
 * coefficient g with |g| <= threshold is set to zero, and the number of
 * coefficients kept is counted; hgf_get_info's stored_peak reports the
 * largest count since the threshold was set (the stored elements a sparse
 * store of the representation would hold at its peak), and stored_tiles_peak
 * the same for tiles of tile_points coefficients.  The grids stay dense
 * in memory.  threshold = 0 turns it off.  For FP64 network operators on the
 * full (k, l) grid and for the separated layouts (every Gx, Gy grid and R);
 * other operators return HGF_EUNSUPPORTED.  Steps run one launch sequence at
 * a time (no graph) while a threshold is set.  The call synchronises the
 * device (it resets the counters).  Errors: HGF_EINVAL (negative or
 * non-finite threshold), HGF_EUNSUPPORTED, HGF_EDEVICE.
 */
hgf_status hgf_set_threshold(hgf_operator op, double threshold);

/*
 * Copy function `idx` to the host for inspection: sector_d [N] gets d = q - p
 * (merged: the sector), extents [N] the grid extents, grid the complex128
 * values R(m) (merged: the whole function) row-major, capacity `n_points`
 * points.  split_out (may be NULL) receives, in split mode, 4N+6 doubles:
 * p[N], q[N] (as doubles), g_pq(0), c_x, c_y (complex) and then 2N zeros.
 * Errors: HGF_EINVAL (idx out of range, buffer too small), HGF_EDEVICE.
 */
hgf_status hgf_get_function(hgf_operator op, int32_t idx, int32_t* sector_d, int32_t* extents,
                            double* grid, int64_t n_points, double* split_out, void* hip_stream);

/*
 * Launch shape of the RK4 stage kernel of one function (merged layout).  The
 * stencil of Eq. (17) in sector form is evaluated on tiles: the trailing
 * `nfast` axes of the grid form a tile staged in LDS, the other axes are read
 * as neighbour tiles from HBM, and a persistent grid of workgroups walks the
 * tiles.  Shapes change the order of additions across axes only: results
 * agree to rounding.
 */
typedef struct {
  int32_t nfast;       /* trailing axes staged in LDS; 0 = untiled (generic) kernel */
  int32_t threads;     /* workgroup size: multiple of 64 in [64, 512] (the resident form: up to
                          1024 in mixed precision, 512 in FP64, covering the grid in at most 4
                          lane rounds, 5 on complex FP64 grids); 0 = default rule */
  int32_t xblock;      /* tile order over the 8 XCDs: 0 = contiguous eighths of the grid,
                          B > 0 = interleaved blocks of B consecutive tiles */
  int32_t pipe;        /* 1 = neighbour loads of the next lane round issued before the
                          current round computes */
  int32_t wgs_per_cu;  /* resident workgroups per CU in the persistent grid; 0 = as many as
                          fit (fewer narrow the band of tiles each XCD works on) */
  int32_t resident;    /* 1 = one workgroup integrates the whole grid on chip through all
                          the steps of a call (state in registers, stage grids in LDS): at
                          most 4 axes and 4096 points (FP64: 2048 real, 2560 complex), two padded copies of
                          the grid within 160 KB; 0 = one launch per RK4 stage.  Set by
                          default where the grid allows it (not under
                          HGF_STAGE_KERNEL=generic or an HGF_MAX_NFAST below the axis
                          count); the other fields keep the stage kernels' shape */
  int32_t walk_block;  /* order in which the persistent grid walks the tiles: 0 = row-major
                          over the slow axes; B >= 2 = blocks of B along every slow axis,
                          row-major inside a block and across blocks (neighbour tiles along
                          every slow axis are then visited close together in time) */
  int32_t blocks;      /* out: persistent workgroups per launch */
  int32_t tile_points; /* out: points per tile */
  double stage_us;     /* out: stage time measured by hgf_autotune for this shape, else 0 */
} hgf_tile_config;

/* Current launch shape of function idx.  Errors: HGF_EINVAL. */
hgf_status hgf_get_tile_config(hgf_operator op, int32_t idx, hgf_tile_config* out);

/*
 * Set the launch shape of function idx (inputs nfast, threads, xblock, pipe,
 * wgs_per_cu, resident, walk_block).
 * On a network operator's full (k, l) grid nfast is 0 (untiled kernel) or 4
 * (tiles of the last two modes' (k, l) block, the four fastest axes), with
 * threads, wgs_per_cu and walk_block, or nfast 0 with resident 1 (the
 * resident form of a network grid twice within 64 KB of LDS, at most three
 * modes); xblock and pipe must be 0.
 * hgf_autotune leaves network operators alone.
 * Errors: HGF_EINVAL when the shape does not fit the grid (LDS, lane rounds,
 * register budget), asks a real grid for the untiled kernel, or asks for the
 * resident form where the grid does not fit it (above; on a sector grid
 * nfast >= 1 must also name a feasible stage-kernel shape, kept beside it);
 * HGF_EUNSUPPORTED for split-layout functions (classical kernel only).  The
 * function is unchanged on error.
 */
hgf_status hgf_set_tile_config(hgf_operator op, int32_t idx, const hgf_tile_config* cfg);

/* flags of hgf_autotune */
enum {
  HGF_TUNE_DEFAULT = 0,     /* use cached shapes, measure the others and add them to the cache */
  HGF_TUNE_CACHED_ONLY = 1, /* apply cached shapes only; measure nothing */
  HGF_TUNE_FORCE = 2        /* measure every shape again and overwrite its cache entry */
};

/*
 * Launch-shape autotuner.  For every distinct grid shape among the merged-
 * layout functions of ops[0..n) (extents, precision, real or complex grid),
 * times the RK4 step of one such function with step dt_us under each
 * candidate shape (fast axes: the default and one fewer; every workgroup
 * size whose last lane round is at least 3/4 full; both XCD orders; with
 * and without pipelined loads; all resident workgroups per CU or one or two
 * fewer) and applies the fastest to every function of that shape.  Then
 * each group of two or more functions that run as one grouped launch per
 * stage (same axis split and element types: the members of a batch, the
 * sectors of one operator) is timed as a whole over workgroup sizes and
 * resident workgroups per CU, and the fastest is applied to all its members
 * (which keep it when evolved alone).  Grid functions that run on the
 * resident integrator are not tuned.  The timed steps run on the functions'
 * own buffers; their states are restored afterwards, so results are
 * unaffected.  cache_path (may be NULL:
 * no cache) names a text file of measured shapes keyed by device
 * architecture and CU count; it is read first and rewritten when shapes were
 * measured.  Errors: HGF_EINVAL (NULL ops, dt <= 0, unwritable cache),
 * HGF_EDEVICE.  Synchronises hip_stream.
 */
hgf_status hgf_autotune(hgf_operator* ops, int32_t n, double dt_us, const char* cache_path, int32_t flags,
                        void* hip_stream);

/* Leave the error state entered after HGF_ENONFINITE (the functions hold the
 * state from the start of the failed call).  Errors: HGF_EINVAL. */
hgf_status hgf_clear_error(hgf_operator op);

/*
 * Device-memory hook.  With alloc and free set, every device buffer the
 * library allocates afterwards comes from alloc(bytes, device, user) (which
 * returns NULL on failure: HGF_ENOMEM) and goes back through
 * free(ptr, device, user), on the device that allocated it.  Both NULL
 * restores hipMalloc / hipFree for later allocations; blocks still held from
 * a replaced hook are then dropped rather than freed (their memory belongs to
 * the hook's owner, e.g. a framework's caching allocator that is shutting
 * down).  Buffers are used on the streams passed to the other calls.
 * Errors: HGF_EINVAL when only one of alloc and free is NULL.
 */
typedef void* (*hgf_alloc_fn)(size_t bytes, int32_t device, void* user);
typedef void (*hgf_free_fn)(void* ptr, int32_t device, void* user);
hgf_status hgf_set_allocator(hgf_alloc_fn alloc, hgf_free_fn free_fn, void* user);

/*
 * Measurement helper (no part of the method): the streaming ceiling of the RK4
 * stage kernel.  On `points` points of fresh buffers, each Horner stage's
 * operands (the stencil input at the point itself, X1, the state y, the stage
 * output, the stage-precision copy of y) are read and written once per point
 * with the stage kernel's access policies and no neighbour reads; us_out[4]
 * receives the average microseconds per launch of stages 1..4 over `reps`
 * launches each.  precision: HGF_FP64 or HGF_MIXED; real: 1 for real grids.
 * Allocates and frees its buffers (5 x points x 16 bytes at most).
 * Errors: HGF_EINVAL (points or reps < 1, buffers beyond 2^32 bytes),
 * HGF_ENOMEM, HGF_EDEVICE.  Synchronises hip_stream.
 */
hgf_status hgf_stream_ceiling(int32_t precision, int32_t real, int64_t points, int32_t reps, double us_out[4],
                              void* hip_stream);

/* Thread-local message describing the last error of this thread ("" if none). */
const char* hgf_last_error(void);

/* Library version string. */
const char* hgf_version(void);

#ifdef __cplusplus
}
#endif

#endif /* HGF_H */
