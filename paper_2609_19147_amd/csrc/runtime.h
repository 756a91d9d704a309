// Runtime objects behind the C ABI: states, plans with their device tables,
// layer execution and the reduction drivers.
#pragma once
#include <hip/hip_runtime.h>

#include <complex>
#include <string>
#include <memory>
#include <vector>

#include "fround.h"
#include "kernels.h"
#include "planner.h"
#include "qs.h"

// A plan's whole layer sequence recorded as a HIP graph for one state
// (qs_apply_graph): valid for the plan's parameter version and the buffer the
// state starts from (gathers flip between the two buffers).
struct PlanGraphEntry {
  uint64_t plan_uid = 0;
  uint64_t version = 0;
  int cur0 = 0, cur1 = 0;
  hipGraphExec_t exec = nullptr;
};

struct qs_state {
  int n = 0;
  qs_dtype dtype = QS_C64;
  int device = 0;
  void* buf[2] = {nullptr, nullptr};
  bool owned[2] = {false, false};
  int cur = 0;
  bool view = false;  // owned by a batch
  hipStream_t stream = nullptr;
  double* red_partials = nullptr;
  double* red_out = nullptr;
  double* norm_part = nullptr;  // per-tile norm partials of a fused apply-and-norm
  uint64_t norm_cap = 0;
  std::vector<PlanGraphEntry> graphs;  // recorded plans, most recent last
  hipStream_t capture_stream = nullptr;  // private stream graphs are recorded on
  void* matbuf = nullptr;  // device staging for dense plain gates
  qs::NormAcc plain_acc;   // norm compensation of the per-gate path's complex64 rounding
  // adjoint sweeps: the two work states (phi, lambda) and a device scratch
  // area, made by the first call and kept until the state is freed
  std::unique_ptr<qs_state> work[2];
  void* work_buf = nullptr;
  size_t work_cap = 0;

  size_t amp_bytes() const;
  size_t state_bytes() const;
  void* cur_ptr() const { return buf[cur]; }
  void ensure_other();
  void ensure_red();
  void ensure_norm(uint64_t tiles);
  void* ensure_work_buf(size_t bytes);  // at least `bytes` of device scratch (waits for the stream to grow it)
  void sync();
  ~qs_state();
};

namespace qs {

// Device tables of a plan for one precision.
struct PlanDev {
  void* blob = nullptr;
  size_t bytes = 0;
  bool valid = false;
  std::vector<size_t> diag_terms, diag_groups, diag_lut;
  std::vector<int> diag_ngroups;
  std::vector<size_t> diag_theta;   // per diagonal layer: reduced group angles (double)
  std::vector<double> diag_global;  // per diagonal layer: reduced global phase angle
  std::vector<size_t> pass_rounds, pass_ops, pass_coef;
  std::vector<size_t> pass_diag;  // per pass: its diagonal slots as DiagDev[] (0: none)
  std::vector<size_t> pass_qtab;  // per pass: pair coefficients of its diagonal rounds
  std::vector<uint32_t> pass_nrounds;  // per pass: device rounds (diagonals as rounds of their own)
  std::vector<double> pass_scale;      // per pass: the store's scale (butterflies, factored rotations)
  std::vector<size_t> dense_mat, dense_mat_dagger;  // per dense block
  std::vector<size_t> plain_mat;  // per layer (only dense plain gates), else 0
};

void check_hip(hipError_t e, const char* what);
extern thread_local std::string g_last_error;

// A profiler range (rocTX) over a scope: planner phases, table builds and
// updates, applies, batch recording and adjoint sweeps appear under these
// names in rocprofv3 --marker-trace.
struct Range {
  explicit Range(const char* name);
  ~Range();
  Range(const Range&) = delete;
  Range& operator=(const Range&) = delete;
};

// Amplitude buffers the library allocates (states, their scratch halves,
// adjoint work states and scratch, batch arenas) count against the cap
// QS_MAX_BYTES (environment variable, bytes, read once; unset or 0: none).
// The allocation also fails with QS_ENOMEM when the device's free memory is
// short.  free_amplitudes takes the size that was allocated.
void* alloc_amplitudes(size_t bytes, const char* what);
void free_amplitudes(void* p, size_t bytes);
size_t amplitude_bytes_held();
size_t amplitude_cap();

}  // namespace qs

namespace qs {
uint64_t new_plan_uid();
}

struct qs_plan {
  qs::PlanIR ir;
  std::vector<double> params;
  bool bound = false;
  qs::PlanDev dev[2];
  std::vector<qs::Gf2Args> gf2;  // host-side kernel arguments per GF(2) layer
  uint64_t version = 0;          // bumped whenever the parameters change
  uint64_t uid = qs::new_plan_uid();  // unique per plan object (keys recorded graphs)
  qs_plan* inv = nullptr;        // inverse plan (adjoint sweeps), built on demand
  uint64_t inv_version = 0;

  // Stream ordering of the device tables (per precision).  Every stream that
  // runs work reading the tables is listed with an event recorded after its
  // latest such work (release); a parameter update stages the new tables in
  // pinned memory, makes the library's upload stream wait for those events
  // (device-side waits: neither the host nor other streams stall) and uploads
  // there, recording `ready`; each reading stream waits for `ready` once per
  // update before its next work (acquire).  A batch lists its stream with an
  // event it records itself after every run (external: not owned here).
  struct TableUser {
    hipStream_t stream = nullptr;
    hipEvent_t done = nullptr;
    uint64_t seen = 0;      // uploads this stream has waited for
    bool external = false;  // event owned by the caller (a batch)
    qs_batch* batch = nullptr;  // that caller, told when the plan is freed first
  };
  std::vector<TableUser> users[2];
  hipEvent_t ready[2] = {nullptr, nullptr};
  uint64_t uploads[2] = {0, 0};
  void* staging[2] = {nullptr, nullptr};  // pinned host image of the last upload
  size_t staging_cap[2] = {0, 0};

  void refresh_device();  // rebuild the tables of every precision already on the device
  const qs::PlanDev& device_for(qs_dtype dt);
  // device tables for work about to be enqueued on s (waits, on s, for a
  // pending update), and the mark after that work is enqueued
  const qs::PlanDev& acquire(qs_dtype dt, hipStream_t s);
  void release(qs_dtype dt, hipStream_t s);
  // a batch's stream and completion event as a user of the tables
  void add_external_user(qs_dtype dt, hipStream_t s, hipEvent_t done, qs_batch* b);
  void remove_external_user(qs_dtype dt, hipEvent_t done);
  // that user's stream waits for an upload it has not seen yet
  void sync_external_user(qs_dtype dt, hipEvent_t done, hipStream_t s);
  qs_plan& inverse();     // the inverse plan with the current parameters
  ~qs_plan();
};

namespace qs {

// A plan of batch b is being freed: the batch drops its pointer to it and
// refuses to run from then on (its recorded launches read the plan's tables).
void batch_plan_freed(qs_batch* b, const qs_plan* p);

// acquire on construction, release on scope exit (also when an error unwinds
// a sequence of enqueued work).
struct TableUse {
  qs_plan& p;
  qs_dtype dt;
  hipStream_t s;
  TableUse(qs_plan& p_, qs_dtype dt_, hipStream_t s_) : p(p_), dt(dt_), s(s_) { p.acquire(dt, s); }
  ~TableUse() {
    try {
      p.release(dt, s);
    } catch (...) {
    }
  }
  TableUse(const TableUse&) = delete;
  TableUse& operator=(const TableUse&) = delete;
};

// Layers [first, last) on the state's stream.  track: order the work against
// parameter updates of p (acquire / release; skipped while the stream is
// being captured); callers that bracket a sequence of calls themselves pass
// false.
void apply_layers(qs_state& s, qs_plan& p, size_t first, size_t last, bool track = true);
// Kernel arguments of tile pass `pass` of plan p applied to state s (device
// tables made on first use); norm_part unset.
template <class R>
TileKArgs<R> tile_args(qs_state& s, qs_plan& p, int pass);
// Apply every layer and return ||psi||^2 of the result (FP64).  When the last
// layer is a tile pass or a gather, its kernel sums |psi|^2 over what it
// writes (no separate read of the state); otherwise a reduction follows.
double apply_norm2(qs_state& s, qs_plan& p);
// Apply every layer through a HIP graph recorded on first use for this state,
// plan and parameter version, replayed afterwards (one launch for the whole
// plan).  Plans with host-staged gates (plain gates on 3 or more qubits) run
// eagerly instead.
void apply_graph(qs_state& s, qs_plan& p);
void free_graphs(qs_state& s);
void apply_plain_gate(qs_state& s, const NGate& g, const std::vector<double>& params, bool inverse = false);
double state_norm2(qs_state& s);
std::complex<double> state_overlap(qs_state& a, qs_state& b);
double state_infidelity(qs_state& a, qs_state& b);
std::vector<double> state_expect(qs_state& s, const qs_pauli* terms, size_t n_terms);

}  // namespace qs
