// Declarations shared by the host runtime modules (hgf_api.cpp, hgf_functions.cpp,
// hgf_network.cpp, hgf_step.cpp, hgf_autotune.cpp, hgf_readout.cpp, hgf_grad.cpp).
#pragma once

#include <hip/hip_runtime.h>

#include <map>
#include <set>
#include <string>
#include <vector>

#include "hgf.h"
#include "hgf_host.h"
#include "hgf_internal.h"
#include "hgf_kernels.h"

namespace hgf {

// Launch shape of the tiled stage kernel.  Fields at -1 (nfast, xblock, pipe)
// or 0 (threads) take the default rule below.
struct TileChoice {
  int nfast = -1;
  int threads = 0;
  int xblock = -1;
  int pipe = -1;
  int wgs_per_cu = 0;  // resident workgroups per CU in the persistent grid (0: as many as fit)
  int wblock = -1;     // tile walk order (-1, 0: row-major; B >= 2: blocks of B per slow axis)
};

// Pipelined neighbour loads keep the register budget only up to this many
// slow axes (more spill to scratch).
constexpr int kPipeMaxSlow = 9;

// ---- merged-layout stepping
// A StepPlan runs one RK4 step of a set of (function, precision, step size)
// items: functions with a tiled configuration as grouped launches (one launch
// per axis split, element type and precision, covering every member's tiles),
// the others with the generic kernel.
struct PlanItem {
  Function* f;
  int precision;
  double h;
};

struct StepPlan {
  std::vector<GroupLaunch> groups;
  std::vector<void*> dmem;
  std::vector<PlanItem> generic;
  // resident launches, with host copies of their items (the step count is set
  // per call)
  std::vector<ResidentLaunch> resident;
  std::vector<std::vector<ResidentItem>> res_host;
  ~StepPlan() {
    for (auto& p : dmem) dfree(p);
  }
};

// Owns an executable graph.
struct GraphHolder {
  hipGraphExec_t e;
  explicit GraphHolder(hipGraphExec_t x) : e(x) {}
  ~GraphHolder() { (void)hipGraphExecDestroy(e); }
  GraphHolder(const GraphHolder&) = delete;
  GraphHolder& operator=(const GraphHolder&) = delete;
};

// Most steps of one resident launch.
constexpr int64_t kResidentChunk = 8192;

// Most kernel nodes in one captured graph.
constexpr int64_t kMaxGraphNodes = 16384;

struct TuneEntry {
  TileChoice c;
  double us = 0.0;
};

// Largest number of grid points in one operator (summed over its functions).
// Every kernel indexes a grid with 64-bit element counts; the cap keeps the
// point counts, their byte sizes and the sums over sectors far from int64
// overflow, and is beyond what HBM holds anyway (2^32 points of the smallest
// element set, a real mixed grid with its stage grids, take over 100 GB).
constexpr int64_t kMaxOperatorPoints = (int64_t)1 << 32;

// ---- hgf_functions.cpp: functions of an operator, tile configuration
bool stage_kernel_generic();
bool configure_tiles(GridArgs& g, int precision, bool real, const TileChoice& c);
std::vector<uint32_t> walk_order(const GridArgs& g);
void* upload_tile_records(GridArgs& g, const SectorTables& t, int precision);
void build_tile_records(Function& f, int precision);
bool resident_eligible(Function& f, int threads = 0);
void fill_grid_args(Function& f, int precision, bool want_real);
size_t state_bytes(const Function& f);
void alloc_function_buffers(Function& f, int precision);
void free_function(Function& f);
int64_t flat_index(const SectorTables& t, const int* m);
std::vector<cd> mode_g(const double* vals, int nc, int basis);
void precheck_operator_size(const System& s, const hgf_operator_desc* d);
void upload_state(Function& f, const std::vector<cd>& grid, int precision);
double energy(const System& s, const int* k);
void setup_split(Function& f, const System& s, const Coeff& c);
void build_functions(hgf_operator_s* op, const hgf_operator_desc* d, bool allow_real = true);

// ---- hgf_network.cpp: network operators on the full (k, l) grid
std::vector<char> full_tile_records(const GridArgs& g, const FullTables& ft, int& rec_bytes);
bool configure_full_tiles(Function& f, const FullTables& ft, int precision, const TileChoice& c);
void drop_full_tiles(Function& f);
void full_mode_order(const System& s, int* perm);
System permute_modes(const System& s, const int* perm);
void build_full_function(hgf_operator_s* op, const hgf_operator_desc* d);
bool full_resident_eligible(Function& f, int precision);

// ---- hgf_step.cpp: launch plans, graphs, RK4 stepping, batches
MemberArgs member_args(const PlanItem& it);
StepPlan* build_plan(const std::vector<PlanItem>& items, bool allow_resident = true);
void run_resident(StepPlan& plan, int64_t steps, int* flag, hipStream_t st);
void stage_launch(const Function& f, int precision, int stage, const void* in, const void* x1, void* y,
    void* yf, void* out, double h, int* flag, hipStream_t st);
void generic_stage(const PlanItem& it, int s, int* flag, hipStream_t st);
void run_plan_step(const StepPlan& plan, int* flag, hipStream_t st);
void drop_graph(hgf_operator_s* op);
void drop_plan(hgf_operator_s* op);
void ensure_plan(hgf_operator_s* op, double h);
hipGraphExec_t capture_steps(const StepPlan& plan, int* flag, int chunk, hipStream_t cap);
int graph_chunk(const StepPlan& plan, int64_t steps);
void ensure_graph(hgf_operator_s* op, double h, int chunk);
void split_step(hgf_operator_s* op, Function& f, double h, hipStream_t st);
void ensure_lawson_tables(Function& f, double h, hipStream_t st);
void lawson_steps(hgf_operator_s* op, int64_t steps, double h, hipStream_t st);
int64_t full_tile_points(const Function& f);
void apply_threshold(hgf_operator_s* op, hipStream_t st);
void evolve_impl(hgf_operator_s* op, int64_t steps, double h, hipStream_t st, int scheme = HGF_RK4);
void batch_impl(hgf_operator* ops, int n, const std::vector<int64_t>& steps, const double* dt, hipStream_t st);

// ---- hgf_autotune.cpp: launch-shape autotuner
void retile(Function& f, int precision, const TileChoice& c);
std::string device_tag();
std::string tune_key(const std::string& dev, const Function& f, int precision);
std::map<std::string, TuneEntry> read_tune_cache(const char* path);
void write_tune_cache(const char* path, const std::map<std::string, TuneEntry>& m);
std::vector<TileChoice> tune_candidates(const Function& f, int precision);
TuneEntry pick_shape(const std::vector<TileChoice>& cands, const std::vector<double>& times);
double time_function_steps(Function& f, int precision, double h, int* flag, int steps, hipStream_t st);
TileChoice current_choice(const Function& f);
double time_plan_steps(const std::vector<PlanItem>& items, int* flag, int steps, hipStream_t st);
void tune_groups(hgf_operator* ops, int n, double h, const std::string& dev,
    std::map<std::string, TuneEntry>& cache, std::set<std::string>& fresh, int flags,
    bool& measured, int* flag, hipStream_t st);
void autotune_impl(hgf_operator* ops, int n, double h, const char* cache_path, int flags, hipStream_t st);

// ---- hgf_readout.cpp: expectation values and the operator readout
std::vector<cd> mode_amps(const hgf_state_desc* psi, int j, int nc, size_t amp_off);
std::vector<cd> sector_weights(const System& s, const Function& f, const std::vector<std::vector<cd>>& amps);
cd expectation_impl(hgf_operator_s* op, const hgf_state_desc* psi, hipStream_t st, void* ws = nullptr,
    size_t ws_bytes = 0);
void reconstruct_impl(hgf_operator_s* op, int levels, double* out, hipStream_t st);

// ---- hgf_grad.cpp: discrete-adjoint gradient
SectorTables transposed_tables(const SectorTables& t);
void grad_impl(const System& sys, const hgf_operator_desc* desc, const hgf_state_desc* psi, double T,
    double dt, int ce, double* value_out, double* grad_out, hipStream_t st);

// ---- hgf_api.cpp: argument checks
double factorial(int n);
int64_t checked_points(const int* ext, int n);
void add_points(int64_t& total, int64_t add);
void check_stability(const std::vector<Function>& fns, double dt, bool jumps_only = false);

}  // namespace hgf
