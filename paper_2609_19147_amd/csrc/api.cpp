// C ABI of libqs: states, plans, layer application, reductions, profiling.
// Validation happens before any device work; errors are reported through
// qs_status and a thread-local message.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <new>
#include <string>
#include <vector>

#include "kernels.h"
#include "planner.h"
#include "qs.h"
#include "runtime.h"

#include <rocprofiler-sdk-roctx/roctx.h>

#include <atomic>
#include <cstdlib>

using namespace qs;

namespace qs {

thread_local std::string g_last_error = "";

void check_hip(hipError_t e, const char* what) {
  if (e != hipSuccess) fail(QS_EDEVICE, std::string(what) + ": " + hipGetErrorString(e));
}

void allow_dynamic_lds(const void* kernel, int bytes, const char* name) {
  const hipError_t e = hipFuncSetAttribute(kernel, hipFuncAttributeMaxDynamicSharedMemorySize, bytes);
  if (e != hipSuccess) {
    (void)hipGetLastError();
    fail(QS_EDEVICE, std::string("LDS limit of ") + name + ": " + hipGetErrorString(e));
  }
}

void check_launch(const char* name) {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) fail(QS_EDEVICE, std::string("launch of ") + name + ": " + hipGetErrorString(e));
}

// ---------------------------------------------------------------- profiling
namespace {
struct ProfRec {
  const char* name;
  hipEvent_t a, b;
};
std::mutex g_prof_mu;
bool g_prof_on = false;
std::vector<ProfRec> g_prof_pending;
std::map<std::string, std::pair<long, double>> g_prof_stats;
thread_local hipEvent_t g_prof_cur = nullptr;
thread_local const char* g_prof_name = nullptr;
}  // namespace

// Graph capture must not record profiling events.
static bool g_prof_suspended = false;
void prof_suspend(bool on) { g_prof_suspended = on; }

void prof_begin(const char* name, hipStream_t s) {
  if (!g_prof_on || g_prof_suspended) return;
  hipEvent_t e;
  check_hip(hipEventCreate(&e), "hipEventCreate");
  check_hip(hipEventRecord(e, s), "hipEventRecord");
  g_prof_cur = e;
  g_prof_name = name;
}
void prof_end(hipStream_t s) {
  if (!g_prof_on || g_prof_suspended || !g_prof_cur) return;
  hipEvent_t e;
  check_hip(hipEventCreate(&e), "hipEventCreate");
  check_hip(hipEventRecord(e, s), "hipEventRecord");
  std::lock_guard<std::mutex> lk(g_prof_mu);
  g_prof_pending.push_back({g_prof_name, g_prof_cur, e});
  g_prof_cur = nullptr;
}
static void prof_drain() {
  std::lock_guard<std::mutex> lk(g_prof_mu);
  for (auto& r : g_prof_pending) {
    check_hip(hipEventSynchronize(r.b), "hipEventSynchronize");
    float ms = 0;
    check_hip(hipEventElapsedTime(&ms, r.a, r.b), "hipEventElapsedTime");
    auto& st = g_prof_stats[r.name];
    st.first += 1;
    st.second += ms;
    hipEventDestroy(r.a);
    hipEventDestroy(r.b);
  }
  g_prof_pending.clear();
}

}  // namespace qs

// ---------------------------------------------------------------- error wrapper
template <class F>
static qs_status guarded(F&& f) {
  try {
    f();
    return QS_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_last_error = "host allocation failed";
    return QS_ENOMEM;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return QS_EINVAL;
  }
}

extern "C" const char* qs_last_error(void) { return g_last_error.c_str(); }
extern "C" const char* qs_version(void) { return "qs 0.1 (gfx950, wave64)"; }

extern "C" qs_status qs_memory_info(size_t* held, size_t* cap) {
  return guarded([&] {
    if (held) *held = qs::amplitude_bytes_held();
    if (cap) *cap = qs::amplitude_cap();
  });
}

// ---------------------------------------------------------------- profiler ranges
namespace qs {
Range::Range(const char* name) { roctxRangePushA(name); }
Range::~Range() { roctxRangePop(); }

namespace {
void plan_phase_range(const char* phase, bool begin) {
  if (begin) roctxRangePushA(phase);
  else roctxRangePop();
}
// the planner's phases report to rocTX from the moment the library is loaded
const bool g_phase_hook_set = (set_plan_phase_hook(&plan_phase_range), true);
}  // namespace
}  // namespace qs

// ---------------------------------------------------------------- device memory
namespace qs {
namespace {
std::atomic<size_t> g_amp_held{0};

size_t amp_cap_read() {
  static const size_t cap = [] {
    const char* e = std::getenv("QS_MAX_BYTES");
    if (!e || !*e) return (size_t)0;
    char* end = nullptr;
    const unsigned long long v = std::strtoull(e, &end, 10);
    return (end && *end == '\0') ? (size_t)v : (size_t)0;
  }();
  return cap;
}
}  // namespace

size_t amplitude_cap() { return amp_cap_read(); }

void* alloc_amplitudes(size_t bytes, const char* what) {
  const size_t cap = amp_cap_read();
  if (cap) {
    size_t held = g_amp_held.load();
    do {
      if (held + bytes > cap)
        fail(QS_ENOMEM, std::string(what) + ": over the QS_MAX_BYTES cap (" + std::to_string(held) + " + " +
                            std::to_string(bytes) + " > " + std::to_string(cap) + " bytes)");
    } while (!g_amp_held.compare_exchange_weak(held, held + bytes));
  } else {
    g_amp_held += bytes;
  }
  size_t fr = 0, tot = 0;
  void* p = nullptr;
  if (hipMemGetInfo(&fr, &tot) != hipSuccess || bytes > fr || hipMalloc(&p, bytes) != hipSuccess) {
    g_amp_held -= bytes;
    fail(QS_ENOMEM, std::string(what) + ": not enough free device memory");
  }
  return p;
}

void free_amplitudes(void* p, size_t bytes) {
  if (!p) return;
  hipFree(p);
  g_amp_held -= bytes;
}

size_t amplitude_bytes_held() { return g_amp_held.load(); }
}  // namespace qs

// ---------------------------------------------------------------- states
size_t qs_state::amp_bytes() const { return dtype == QS_C64 ? 8 : 16; }
size_t qs_state::state_bytes() const { return amp_bytes() << n; }

void qs_state::ensure_other() {
  if (buf[1 - cur]) return;
  buf[1 - cur] = alloc_amplitudes(state_bytes(), "permutation scratch buffer");
  owned[1 - cur] = true;
}

void qs_state::ensure_red() {
  if (red_partials) return;
  check_hip(hipMalloc(&red_partials, sizeof(double) * 2 * kMaxTermsPerLaunch * kRedBlocks), "hipMalloc");
  check_hip(hipMalloc(&red_out, sizeof(double) * 16), "hipMalloc");
}

void qs_state::ensure_norm(uint64_t tiles) {
  if (norm_cap >= tiles) return;
  if (norm_part) {
    check_hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
    check_hip(hipFree(norm_part), "hipFree");
    norm_part = nullptr;
    norm_cap = 0;
  }
  check_hip(hipMalloc(&norm_part, sizeof(double) * tiles), "hipMalloc");
  norm_cap = tiles;
}

void* qs_state::ensure_work_buf(size_t bytes) {
  if (work_cap >= bytes) return work_buf;
  if (work_buf) {
    check_hip(hipStreamSynchronize(stream), "hipStreamSynchronize");
    free_amplitudes(work_buf, work_cap);
    work_buf = nullptr;
    work_cap = 0;
  }
  work_buf = alloc_amplitudes(bytes, "adjoint scratch");
  work_cap = bytes;
  return work_buf;
}

void qs_state::sync() { check_hip(hipStreamSynchronize(stream), "hipStreamSynchronize"); }

static qs_state* check_state(qs_state* s) {
  if (!s) fail(QS_EINVAL, "state is NULL");
  return s;
}

extern "C" qs_status qs_alloc(int n, qs_dtype dtype, void* buf, void* scratch, size_t bytes, void* stream,
                              qs_state** out) {
  return guarded([&] {
    if (!out) fail(QS_EINVAL, "out is NULL");
    if (n < 1 || n > QS_MAX_QUBITS) fail(QS_EINVAL, "qubit count out of range");
    if (dtype != QS_C64 && dtype != QS_C128) fail(QS_EINVAL, "unknown dtype");
    auto s = std::make_unique<qs_state>();
    s->n = n;
    s->dtype = dtype;
    s->stream = (hipStream_t)stream;
    const size_t need = s->state_bytes();
    if ((buf && bytes < need) || (scratch && bytes < need)) fail(QS_EINVAL, "given buffer smaller than 2^n amplitudes");
    if (buf) {
      s->buf[0] = buf;
    } else {
      s->buf[0] = alloc_amplitudes(need, "state");  // the cap is checked before any device call
      s->owned[0] = true;
    }
    check_hip(hipGetDevice(&s->device), "hipGetDevice");
    if (scratch) s->buf[1] = scratch;
    *out = s.release();
  });
}

qs_state::~qs_state() {
  for (int k = 0; k < 2; ++k)
    if (owned[k] && buf[k]) free_amplitudes(buf[k], state_bytes());
  if (red_partials) hipFree(red_partials);
  if (red_out) hipFree(red_out);
  if (norm_part) hipFree(norm_part);
  free_graphs(*this);
  if (matbuf) hipFree(matbuf);
  if (work_buf) free_amplitudes(work_buf, work_cap);
}

extern "C" qs_status qs_free(qs_state* s) {
  return guarded([&] {
    if (!s) return;
    if (!s->view) {
      hipStreamSynchronize(s->stream);
      delete s;
    }
  });
}

extern "C" qs_status qs_state_buffers(const qs_state* s, void** current, void** other) {
  return guarded([&] {
    if (!s) fail(QS_EINVAL, "state is NULL");
    if (current) *current = s->buf[s->cur];
    if (other) *other = s->buf[1 - s->cur];
  });
}

extern "C" qs_status qs_state_info(const qs_state* s, int* n, int* dtype) {
  return guarded([&] {
    if (!s) fail(QS_EINVAL, "state is NULL");
    if (n) *n = s->n;
    if (dtype) *dtype = s->dtype;
  });
}

extern "C" qs_status qs_set_basis(qs_state* s, uint64_t index) {
  return guarded([&] {
    check_state(s);
    if (index >> s->n) fail(QS_EINVAL, "basis index out of range");
    uint64_t N = 1ull << s->n;
    if (s->dtype == QS_C64) launch_fill_basis<float>((cplx<float>*)s->cur_ptr(), N, index, s->stream);
    else launch_fill_basis<double>((cplx<double>*)s->cur_ptr(), N, index, s->stream);
  });
}

extern "C" qs_status qs_set_uniform(qs_state* s) {
  return guarded([&] {
    check_state(s);
    uint64_t N = 1ull << s->n;
    double v = std::ldexp(1.0, -s->n / 2) * ((s->n & 1) ? std::sqrt(0.5) : 1.0);
    if (s->dtype == QS_C64) launch_fill_uniform<float>((cplx<float>*)s->cur_ptr(), N, v, s->stream);
    else launch_fill_uniform<double>((cplx<double>*)s->cur_ptr(), N, v, s->stream);
  });
}

extern "C" qs_status qs_upload(qs_state* s, const void* host, size_t bytes) {
  return guarded([&] {
    check_state(s);
    if (!host || bytes != s->state_bytes()) fail(QS_EINVAL, "host buffer size must be 2^n amplitudes");
    check_hip(hipMemcpyAsync(s->cur_ptr(), host, bytes, hipMemcpyHostToDevice, s->stream), "hipMemcpyAsync");
    s->sync();
  });
}

extern "C" qs_status qs_download(const qs_state* cs, void* host, size_t bytes) {
  return guarded([&] {
    qs_state* s = const_cast<qs_state*>(cs);
    check_state(s);
    if (!host || bytes != s->state_bytes()) fail(QS_EINVAL, "host buffer size must be 2^n amplitudes");
    check_hip(hipMemcpyAsync(host, s->cur_ptr(), bytes, hipMemcpyDeviceToHost, s->stream), "hipMemcpyAsync");
    s->sync();
  });
}

extern "C" qs_status qs_copy(qs_state* dst, const qs_state* csrc) {
  return guarded([&] {
    qs_state* src = const_cast<qs_state*>(csrc);
    check_state(dst);
    check_state(src);
    if (dst->n != src->n) fail(QS_EINVAL, "qubit counts differ");
    if (src->stream != dst->stream) src->sync();
    uint64_t N = 1ull << dst->n;
    if (dst->dtype == QS_C64 && src->dtype == QS_C64)
      launch_convert<float, float>((cplx<float>*)dst->cur_ptr(), (const cplx<float>*)src->cur_ptr(), N, dst->stream);
    else if (dst->dtype == QS_C64)
      launch_convert<float, double>((cplx<float>*)dst->cur_ptr(), (const cplx<double>*)src->cur_ptr(), N, dst->stream);
    else if (src->dtype == QS_C64)
      launch_convert<double, float>((cplx<double>*)dst->cur_ptr(), (const cplx<float>*)src->cur_ptr(), N, dst->stream);
    else
      launch_convert<double, double>((cplx<double>*)dst->cur_ptr(), (const cplx<double>*)src->cur_ptr(), N,
                                     dst->stream);
  });
}

extern "C" qs_status qs_sync(qs_state* s) {
  return guarded([&] {
    check_state(s);
    s->sync();
  });
}

// ---------------------------------------------------------------- plans
extern "C" qs_status qs_plan_create(int n, const qs_gate* gates, size_t n_gates, size_t n_params,
                                    const qs_plan_opts* opts, qs_plan** out) {
  return guarded([&] {
    const Range range("qs.plan_create");
    if (!out) fail(QS_EINVAL, "out is NULL");
    PlanOptions o;
    int low = 0;
    if (opts) {
      if (opts->mode != QS_PLAIN && opts->mode != QS_FUSED) fail(QS_EINVAL, "unknown plan mode");
      o.mode = opts->mode;
      o.max_tile_bits = opts->max_tile_bits;
      if (opts->dense_k_max) o.dense_k_max = opts->dense_k_max;
      if (opts->window_k < -1 || (opts->window_k > 0 && (opts->window_k < 4 || opts->window_k > 6)))
        fail(QS_EINVAL, "window_k must be -1, 0 or 4..6");
      if (opts->window_k) o.window_k = opts->window_k;
      if (opts->low_bits && (opts->low_bits < 2 || opts->low_bits > 8)) fail(QS_EINVAL, "low_bits must be 0 or 2..8");
      if (opts->low_bits) low = opts->low_bits;
      if (opts->coset_order < 0 || opts->coset_order > 2) fail(QS_EINVAL, "coset_order must be 0, 1 or 2");
      o.coset_order = opts->coset_order;
      if (opts->diag_low_bits != 0 && opts->diag_low_bits != -1 && (opts->diag_low_bits < 2 || opts->diag_low_bits > 8))
        fail(QS_EINVAL, "diag_low_bits must be -1, 0 or 2..8");
      o.diag_low_bits = opts->diag_low_bits;
      if (opts->balance_passes < -1 || opts->balance_passes > 0) fail(QS_EINVAL, "balance_passes must be -1 or 0");
      o.balance_passes = opts->balance_passes;
    }
    int tb = o.max_tile_bits ? o.max_tile_bits : 13;
    if (tb < kRoundBits + 1 || tb > kMaxTileBits) fail(QS_EINVAL, "max_tile_bits out of range");
    auto g = normalise_gates(n, gates, n_gates, n_params);
    auto p = std::make_unique<qs_plan>();
    p->ir = build_plan(n, std::move(g), n_params, o, tb, low);
    p->bound = n_params == 0;
    *out = p.release();
  });
}

extern "C" qs_status qs_plan_set_params(qs_plan* p, const double* params, size_t n_params) {
  return guarded([&] {
    if (!p) fail(QS_EINVAL, "plan is NULL");
    if (n_params != p->ir.n_params) fail(QS_EINVAL, "parameter count does not match the plan");
    if (n_params && !params) fail(QS_EINVAL, "params is NULL");
    for (size_t i = 0; i < n_params; ++i)
      if (!std::isfinite(params[i])) fail(QS_EINVAL, "non-finite parameter");
    p->params.assign(params, params + n_params);
    p->bound = true;
    p->version += 1;
    p->refresh_device();
  });
}

extern "C" qs_status qs_plan_num_layers(const qs_plan* p, size_t* out) {
  return guarded([&] {
    if (!p || !out) fail(QS_EINVAL, "NULL argument");
    *out = p->ir.layers.size();
  });
}

extern "C" qs_status qs_plan_describe(const qs_plan* p, char* buf, size_t cap, size_t* needed) {
  return guarded([&] {
    if (!p) fail(QS_EINVAL, "plan is NULL");
    std::string js = describe_json(p->ir, p->params, p->bound);
    if (needed) *needed = js.size() + 1;
    if (buf && cap) {
      size_t k = std::min(cap - 1, js.size());
      std::memcpy(buf, js.data(), k);
      buf[k] = 0;
    }
  });
}

qs_plan::~qs_plan() {
  // work that reads the tables, and a pending upload, finish first
  for (int k = 0; k < 2; ++k) {
    for (auto& u : users[k]) {
      if (u.done) hipEventSynchronize(u.done);
      if (u.done && !u.external) hipEventDestroy(u.done);
      if (u.external && u.batch) qs::batch_plan_freed(u.batch, this);
    }
    if (ready[k]) {
      hipEventSynchronize(ready[k]);
      hipEventDestroy(ready[k]);
    }
    if (staging[k]) hipHostFree(staging[k]);
  }
  for (auto& d : dev)
    if (d.blob) hipFree(d.blob);
  delete inv;
}

extern "C" qs_status qs_plan_inverse(const qs_plan* p, qs_plan** out) {
  return guarded([&] {
    if (!p || !out) fail(QS_EINVAL, "NULL argument");
    auto q = std::make_unique<qs_plan>();
    q->ir = invert_plan(p->ir);
    q->params = p->params;
    q->bound = p->bound;
    *out = q.release();
  });
}

extern "C" qs_status qs_plan_free(qs_plan* p) {
  return guarded([&] { delete p; });
}

extern "C" qs_status qs_apply_layer(qs_state* s, const qs_plan* p, size_t first, size_t count) {
  return guarded([&] {
    check_state(s);
    if (!p) fail(QS_EINVAL, "plan is NULL");
    if (p->ir.n != s->n) fail(QS_EINVAL, "plan and state qubit counts differ");
    if (!p->bound) fail(QS_EINVAL, "plan parameters are not bound");
    size_t L = p->ir.layers.size();
    if (first > L) fail(QS_EINVAL, "first layer out of range");
    size_t last = (count == (size_t)-1 || count > L - first) ? L : first + count;
    apply_layers(*s, const_cast<qs_plan&>(*p), first, last);
  });
}

extern "C" qs_status qs_apply_graph(qs_state* s, const qs_plan* p) {
  return guarded([&] {
    check_state(s);
    if (!p) fail(QS_EINVAL, "plan is NULL");
    if (p->ir.n != s->n) fail(QS_EINVAL, "plan and state qubit counts differ");
    if (!p->bound) fail(QS_EINVAL, "plan parameters are not bound");
    apply_graph(*s, const_cast<qs_plan&>(*p));
  });
}

extern "C" qs_status qs_apply_norm2(qs_state* s, const qs_plan* p, double* norm2) {
  return guarded([&] {
    check_state(s);
    if (!p) fail(QS_EINVAL, "plan is NULL");
    if (!norm2) fail(QS_EINVAL, "norm2 is NULL");
    if (p->ir.n != s->n) fail(QS_EINVAL, "plan and state qubit counts differ");
    if (!p->bound) fail(QS_EINVAL, "plan parameters are not bound");
    *norm2 = apply_norm2(*s, const_cast<qs_plan&>(*p));
  });
}

extern "C" qs_status qs_apply_gates(qs_state* s, const qs_gate* gates, size_t n_gates, const double* params,
                                    size_t n_params) {
  return guarded([&] {
    check_state(s);
    auto g = normalise_gates(s->n, gates, n_gates, n_params);
    if (n_params && !params) fail(QS_EINVAL, "params is NULL");
    std::vector<double> pv(params, params + n_params);
    s->plain_acc = NormAcc{};  // the rounding compensation restarts with every call
    for (auto& ng : g) apply_plain_gate(*s, ng, pv);
  });
}

// ---------------------------------------------------------------- reductions
extern "C" qs_status qs_norm2(qs_state* s, double* out) {
  return guarded([&] {
    check_state(s);
    if (!out) fail(QS_EINVAL, "out is NULL");
    *out = state_norm2(*s);
  });
}

extern "C" qs_status qs_overlap(qs_state* a, qs_state* b, double out[2]) {
  return guarded([&] {
    check_state(a);
    check_state(b);
    if (!out) fail(QS_EINVAL, "out is NULL");
    if (a->n != b->n) fail(QS_EINVAL, "qubit counts differ");
    auto v = state_overlap(*a, *b);
    out[0] = v.real();
    out[1] = v.imag();
  });
}

extern "C" qs_status qs_infidelity(qs_state* a, qs_state* b, double* out) {
  return guarded([&] {
    check_state(a);
    check_state(b);
    if (!out) fail(QS_EINVAL, "out is NULL");
    if (a->n != b->n) fail(QS_EINVAL, "qubit counts differ");
    *out = state_infidelity(*a, *b);
  });
}

extern "C" qs_status qs_expect(qs_state* s, const qs_pauli* terms, size_t n_terms, double* per_term, double* total) {
  return guarded([&] {
    check_state(s);
    if (n_terms && !terms) fail(QS_EINVAL, "terms is NULL");
    std::vector<double> v = state_expect(*s, terms, n_terms);
    double tot = 0.0, c = 0.0;
    for (size_t i = 0; i < n_terms; ++i) {
      if (per_term) per_term[i] = v[i];
      double y = v[i] - c, t = tot + y;
      c = (t - tot) - y;
      tot = t;
    }
    if (total) *total = tot;
  });
}

extern "C" qs_status qs_amplitudes(qs_state* s, const uint64_t* idx, size_t count, void* host_amps) {
  return guarded([&] {
    check_state(s);
    if (count == 0) return;
    if (!idx || !host_amps) fail(QS_EINVAL, "NULL argument");
    for (size_t i = 0; i < count; ++i)
      if (idx[i] >> s->n) fail(QS_EINVAL, "index out of range");
    uint64_t* didx = nullptr;
    void* dout = nullptr;
    check_hip(hipMalloc(&didx, count * 8), "hipMalloc");
    if (hipMalloc(&dout, count * s->amp_bytes()) != hipSuccess) {
      hipFree(didx);
      fail(QS_ENOMEM, "hipMalloc");
    }
    struct Guard {
      void* a;
      void* b;
      ~Guard() { hipFree(a); hipFree(b); }
    } guard{didx, dout};
    check_hip(hipMemcpyAsync(didx, idx, count * 8, hipMemcpyHostToDevice, s->stream), "hipMemcpyAsync");
    if (s->dtype == QS_C64)
      launch_gather<float>((const cplx<float>*)s->cur_ptr(), didx, (cplx<float>*)dout, count, s->stream);
    else
      launch_gather<double>((const cplx<double>*)s->cur_ptr(), didx, (cplx<double>*)dout, count, s->stream);
    check_hip(hipMemcpyAsync(host_amps, dout, count * s->amp_bytes(), hipMemcpyDeviceToHost, s->stream),
              "hipMemcpyAsync");
    s->sync();
  });
}

// ---------------------------------------------------------------- read-out
extern "C" qs_status qs_sample(qs_state* s, const double* u, size_t count, uint64_t* out) {
  return guarded([&] {
    check_state(s);
    if (count == 0) return;
    if (!u || !out) fail(QS_EINVAL, "NULL argument");
    for (size_t k = 0; k < count; ++k)
      if (!(u[k] >= 0.0 && u[k] < 1.0)) fail(QS_EINVAL, "uniform numbers must lie in [0, 1)");
    const double nrm = state_norm2(*s);
    if (!(nrm > 0.0) || !std::isfinite(nrm)) fail(QS_EINVAL, "the state has no probability mass");
    const size_t nscr = sample_scratch_doubles(s->n);
    void* buf = nullptr;
    check_hip(hipMalloc(&buf, (nscr + 2 * count) * 8), "hipMalloc");
    struct Guard {
      void* p;
      ~Guard() { hipFree(p); }
    } guard{buf};
    double* scratch = (double*)buf;
    double* du = scratch + nscr;
    uint64_t* dout = (uint64_t*)(du + count);
    check_hip(hipMemcpyAsync(du, u, count * 8, hipMemcpyHostToDevice, s->stream), "hipMemcpyAsync");
    if (s->dtype == QS_C64)
      launch_sample<float>((const cplx<float>*)s->cur_ptr(), s->n, du, count, dout, scratch, s->stream);
    else
      launch_sample<double>((const cplx<double>*)s->cur_ptr(), s->n, du, count, dout, scratch, s->stream);
    check_hip(hipMemcpyAsync(out, dout, count * 8, hipMemcpyDeviceToHost, s->stream), "hipMemcpyAsync");
    s->sync();
  });
}

// The same draws as qs_sample, with every device buffer in the library's
// static per-GPU scratch: no device memory is allocated or freed.
extern "C" qs_status qs_sample_noalloc(qs_state* s, const double* u, size_t count, uint64_t* out) {
  return guarded([&] {
    check_state(s);
    if (count == 0) return;
    if (!u || !out) fail(QS_EINVAL, "NULL argument");
    if (s->n > kNoAllocSampleMaxQubits)
      fail(QS_EINVAL, "qs_sample_noalloc: the state has " + std::to_string(s->n) + " qubits; its static scratch "
                      "holds the sums of at most " + std::to_string(kNoAllocSampleMaxQubits) + " qubits");
    if (count > kNoAllocSampleMaxDraws)
      fail(QS_EINVAL, "qs_sample_noalloc: " + std::to_string(count) + " draws requested; at most " +
                      std::to_string(kNoAllocSampleMaxDraws) + " per call");
    for (size_t k = 0; k < count; ++k)
      if (!(u[k] >= 0.0 && u[k] < 1.0)) fail(QS_EINVAL, "uniform numbers must lie in [0, 1)");
    const NoAllocSampleScratch S = noalloc_sample_scratch(s->device);
    const uint64_t N = 1ull << s->n;
    if (s->dtype == QS_C64)
      launch_norm2<float>((const cplx<float>*)s->cur_ptr(), N, S.norm_partials, S.norm_out, s->stream);
    else
      launch_norm2<double>((const cplx<double>*)s->cur_ptr(), N, S.norm_partials, S.norm_out, s->stream);
    double nrm = 0.0;
    check_hip(hipMemcpyAsync(&nrm, S.norm_out, sizeof nrm, hipMemcpyDeviceToHost, s->stream), "hipMemcpyAsync");
    s->sync();
    if (!(nrm > 0.0) || !std::isfinite(nrm)) fail(QS_EINVAL, "the state has no probability mass");
    check_hip(hipMemcpyAsync(S.u, u, count * 8, hipMemcpyHostToDevice, s->stream), "hipMemcpyAsync");
    if (s->dtype == QS_C64)
      launch_sample<float>((const cplx<float>*)s->cur_ptr(), s->n, S.u, count, S.out, S.sums, s->stream);
    else
      launch_sample<double>((const cplx<double>*)s->cur_ptr(), s->n, S.u, count, S.out, S.sums, s->stream);
    check_hip(hipMemcpyAsync(out, S.out, count * 8, hipMemcpyDeviceToHost, s->stream), "hipMemcpyAsync");
    s->sync();
  });
}

extern "C" qs_status qs_marginal(qs_state* s, uint64_t qubit_mask, double* out) {
  return guarded([&] {
    check_state(s);
    if (!out) fail(QS_EINVAL, "NULL argument");
    if (s->n < 64 && (qubit_mask >> s->n)) fail(QS_EINVAL, "qubit mask out of range");
    const int k = __builtin_popcountll(qubit_mask);
    if (k > 16) fail(QS_EINVAL, "at most 16 qubits in a marginal");
    if (k == 0) {
      out[0] = state_norm2(*s);
      return;
    }
    int sel[16], m = 0;
    for (int b = 0; b < s->n; ++b)  // ascending state bits = descending qubits
      if ((qubit_mask >> (s->n - 1 - b)) & 1) sel[m++] = b;
    const MarginalArgs A = marginal_geometry(s->n, sel, k);
    const size_t np = marginal_partials(A), bins = (size_t)1 << k;
    void* buf = nullptr;
    check_hip(hipMalloc(&buf, (np + bins) * 8), "hipMalloc");
    struct Guard {
      void* p;
      ~Guard() { hipFree(p); }
    } guard{buf};
    double* part = (double*)buf;
    double* dout = part + np;
    if (s->dtype == QS_C64)
      launch_marginal<float>((const cplx<float>*)s->cur_ptr(), A, part, dout, s->stream);
    else
      launch_marginal<double>((const cplx<double>*)s->cur_ptr(), A, part, dout, s->stream);
    check_hip(hipMemcpyAsync(out, dout, bins * 8, hipMemcpyDeviceToHost, s->stream), "hipMemcpyAsync");
    s->sync();
  });
}

// ---------------------------------------------------------------- profiling
extern "C" qs_status qs_profile_enable(int on) {
  return guarded([&] {
    if (!on) prof_drain();
    g_prof_on = on != 0;
  });
}

extern "C" qs_status qs_profile_report(char* buf, size_t cap, size_t* needed) {
  return guarded([&] {
    prof_drain();
    std::string js = "[";
    bool first = true;
    for (auto& kv : g_prof_stats) {
      char line[256];
      std::snprintf(line, sizeof line, "%s{\"kernel\":\"%s\",\"launches\":%ld,\"total_ms\":%.6f}", first ? "" : ",",
                    kv.first.c_str(), kv.second.first, kv.second.second);
      js += line;
      first = false;
    }
    js += "]";
    if (needed) *needed = js.size() + 1;
    if (buf && cap) {
      size_t k = std::min(cap - 1, js.size());
      std::memcpy(buf, js.data(), k);
      buf[k] = 0;
    }
  });
}

extern "C" qs_status qs_profile_reset(void) {
  return guarded([&] {
    prof_drain();
    g_prof_stats.clear();
  });
}
