// Batched execution of many circuits: one device arena for all states, one
// launch per (qubit count, layer slot) covering every instance of that size,
// the whole sequence recorded once as a HIP graph.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <memory>
#include <string>
#include <vector>

#include "runtime.h"

using namespace qs;

namespace qs {
void prof_suspend(bool on);
}

struct qs_batch {
  size_t n_inst = 0;
  qs_dtype dtype = QS_C64;
  int init = 1;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  std::vector<int> nq;
  std::vector<qs_plan*> plans;
  void* arena = nullptr;
  size_t arena_bytes = 0;
  std::vector<size_t> offset;  // amplitude offset of each instance
  std::vector<std::unique_ptr<qs_state>> views;
  struct Group {
    int n;
    std::vector<size_t> inst;
  };
  std::vector<Group> groups;
  void* desc = nullptr;  // device descriptors of the batched tile launches
  size_t desc_bytes = 0;
  std::vector<std::vector<size_t>> slot_desc;  // per group, per layer: byte offset into desc (or -1)
  double* red = nullptr;
  size_t red_doubles = 0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;  // recorded after every run: the plans order table updates after it
  bool plan_freed = false;    // a plan was freed while the batch lived: it no longer runs
  // observables stored by qs_batch_set_observables: device tables, results
  // and partials in one allocation, descriptors in group order
  void* obs_dev = nullptr;
  size_t obs_out_off = 0, obs_part_off = 0, obs_desc_off = 0;
  std::vector<size_t> obs_pos;

  size_t amp_bytes() const { return dtype == QS_C64 ? 8 : 16; }
  ~qs_batch();
};

qs_batch::~qs_batch() {
  if (exec) hipGraphExecDestroy(exec);
  if (graph) hipGraphDestroy(graph);
  if (stream) hipStreamSynchronize(stream);
  if (done) {
    for (qs_plan* p : plans)
      if (p) p->remove_external_user(dtype, done);
    hipEventDestroy(done);
  }
  if (desc) hipFree(desc);
  if (red) hipFree(red);
  if (arena) free_amplitudes(arena, arena_bytes);
  if (obs_dev) hipFree(obs_dev);
  if (own_stream && stream) hipStreamDestroy(stream);
}

namespace {

std::string shape_signature(const PlanIR& P) {
  std::string sig;
  for (const LayerIR& L : P.layers) {
    char b[64];
    if (L.kind == L_TILE) {
      const TilePassIR& T = P.passes[L.index];
      std::snprintf(b, sizeof b, "T%d.%d.%d;", T.L, T.a, T.h);
    } else {
      std::snprintf(b, sizeof b, "K%d;", L.kind);
    }
    sig += b;
  }
  return sig;
}

// Every amplitude of |+>^n: 2^(-n/2).
double plus_amplitude(int n) { return std::ldexp(1.0, -n / 2) * ((n & 1) ? std::sqrt(0.5) : 1.0); }

template <class R>
void build_descs(qs_batch& B) {
  // one TileKArgs per (group, tile layer, instance), laid out contiguously per launch
  std::vector<unsigned char> host;
  B.slot_desc.assign(B.groups.size(), {});
  for (size_t gi = 0; gi < B.groups.size(); ++gi) {
    const auto& G = B.groups[gi];
    const PlanIR& P0 = B.plans[G.inst[0]]->ir;
    B.slot_desc[gi].assign(P0.layers.size(), (size_t)-1);
    for (size_t li = 0; li < P0.layers.size(); ++li) {
      if (P0.layers[li].kind != L_TILE) continue;
      size_t off = (host.size() + 255) & ~size_t(255);
      host.resize(off + G.inst.size() * sizeof(TileKArgs<R>));
      for (size_t k = 0; k < G.inst.size(); ++k) {
        size_t i = G.inst[k];
        qs_plan& p = *B.plans[i];
        const PlanDev& d = p.device_for(B.dtype);
        const char* base = (const char*)d.blob;
        const LayerIR& L = p.ir.layers[li];
        const TilePassIR& T = p.ir.passes[L.index];
        TileKArgs<R> A;
        std::memset(&A, 0, sizeof A);
        A.psi = (cplx<R>*)((char*)B.arena + B.offset[i] * B.amp_bytes());
        A.rounds = (const TileRound*)(base + d.pass_rounds[L.index]);
        A.ops = (const TileOp*)(base + d.pass_ops[L.index]);
        A.coef = (const cplx<R>*)(base + d.pass_coef[L.index]);
        A.diag = d.pass_diag[L.index] ? (const DiagDev*)(base + d.pass_diag[L.index]) : nullptr;
        A.qtab = (const int32_t*)(base + d.pass_qtab[L.index]);
        A.L = T.L;
        A.a = T.a;
        A.h = T.h;
        A.m = T.L + T.h;
        A.n_rounds = d.pass_nrounds[L.index];
        A.n = p.ir.n;
        A.scale = d.pass_scale[L.index];
        // |+>^n made by the first layer's tile loads (no separate fill)
        if (li == 0 && B.init == 1) A.init_amp = plus_amplitude(G.n);
        std::memcpy(host.data() + off + k * sizeof A, &A, sizeof A);
      }
      B.slot_desc[gi][li] = off;
    }
  }
  if (host.empty()) host.resize(16);
  if (B.desc && B.desc_bytes != host.size()) {
    hipFree(B.desc);
    B.desc = nullptr;
  }
  if (!B.desc) check_hip(hipMalloc(&B.desc, host.size()), "hipMalloc(batch descriptors)");
  B.desc_bytes = host.size();
  check_hip(hipMemcpy(B.desc, host.data(), host.size(), hipMemcpyHostToDevice), "hipMemcpy");
}

template <class R>
void record(qs_batch& B) {
  // initial states, then every layer slot of every group
  for (const auto& G : B.groups) {
    const size_t first = G.inst[0];
    cplx<R>* base = (cplx<R>*)((char*)B.arena + B.offset[first] * B.amp_bytes());
    const uint64_t N = (uint64_t)G.inst.size() << G.n;  // instances of a group are contiguous
    if (B.init == 1) {
      // a group whose first layer is a tile pass makes |+>^n in that pass's loads
      const PlanIR& P0 = B.plans[first]->ir;
      if (P0.layers.empty() || P0.layers[0].kind != L_TILE) launch_fill_uniform<R>(base, N, plus_amplitude(G.n), B.stream);
    } else {
      // |0...0> for each instance
      launch_fill_uniform<R>(base, N, 0.0, B.stream);
      for (size_t i : G.inst)
        launch_fill_basis<R>((cplx<R>*)((char*)B.arena + B.offset[i] * B.amp_bytes()), 1ull << G.n, 0, B.stream);
    }
  }
  for (size_t gi = 0; gi < B.groups.size(); ++gi) {
    const auto& G = B.groups[gi];
    const PlanIR& P0 = B.plans[G.inst[0]]->ir;
    for (size_t li = 0; li < P0.layers.size(); ++li) {
      const LayerIR& L0 = P0.layers[li];
      if (L0.kind == L_TILE) {
        const TilePassIR& T = P0.passes[L0.index];
        bool has_diag = false;
        for (size_t i : G.inst) {
          const qs_plan& p = *B.plans[i];
          has_diag = has_diag || !p.ir.passes[p.ir.layers[li].index].diag_slots.empty();
        }
        launch_tile_batched<R>((const TileKArgs<R>*)((char*)B.desc + B.slot_desc[gi][li]), (uint32_t)G.inst.size(),
                               (uint32_t)G.n, (uint32_t)(T.L + T.h), has_diag, B.stream);
      } else {
        // other layer kinds: one launch per instance
        for (size_t i : G.inst) apply_layers(*B.views[i], *B.plans[i], li, li + 1);
      }
    }
  }
}

}  // namespace

extern "C" qs_status qs_batch_create(size_t n_inst, const int* n_qubits, const qs_plan* const* plans, int init,
                                     qs_dtype dtype, void* stream, qs_batch** out) {
  qs_batch* raw = nullptr;
  try {
    if (!out || !n_qubits || !plans || n_inst == 0) fail(QS_EINVAL, "empty batch or NULL argument");
    if (dtype != QS_C64 && dtype != QS_C128) fail(QS_EINVAL, "unknown dtype");
    if (init != 0 && init != 1) fail(QS_EINVAL, "init must be 0 or 1");
    auto B = std::make_unique<qs_batch>();
    B->n_inst = n_inst;
    B->dtype = dtype;
    B->init = init;
    B->nq.assign(n_qubits, n_qubits + n_inst);
    for (size_t i = 0; i < n_inst; ++i) {
      qs_plan* p = const_cast<qs_plan*>(plans[i]);
      if (!p) fail(QS_EINVAL, "NULL plan");
      if (p->ir.n != n_qubits[i]) fail(QS_EINVAL, "plan and instance qubit counts differ");
      if (!p->bound) fail(QS_EINVAL, "plan parameters are not bound");
      for (const LayerIR& L : p->ir.layers) {
        if (L.kind == L_GF2) fail(QS_EUNSUPPORTED, "permutation layers are not supported in batches");
        if (L.kind == L_DENSE) fail(QS_EUNSUPPORTED, "dense blocks are not supported in batches");
        if (L.kind == L_PLAIN && p->ir.gates[L.index].bits.size() > 2)
          fail(QS_EUNSUPPORTED, "dense gates on more than two qubits are not supported in batches");
      }
      B->plans.push_back(p);
    }
    // group instances by qubit count and layer shape, lay states out group by group
    std::map<std::pair<int, std::string>, size_t> gidx;
    for (size_t i = 0; i < n_inst; ++i) {
      auto key = std::make_pair(n_qubits[i], shape_signature(B->plans[i]->ir));
      auto it = gidx.find(key);
      if (it == gidx.end()) {
        gidx[key] = B->groups.size();
        B->groups.push_back({n_qubits[i], {}});
        it = gidx.find(key);
      }
      B->groups[it->second].inst.push_back(i);
    }
    B->offset.assign(n_inst, 0);
    size_t total = 0;
    for (auto& G : B->groups)
      for (size_t i : G.inst) {
        B->offset[i] = total;
        total += 1ull << G.n;
      }
    const size_t bytes = total * B->amp_bytes();
    B->arena = alloc_amplitudes(bytes, "batch states");
    B->arena_bytes = bytes;
    if (stream) {
      B->stream = (hipStream_t)stream;
    } else {
      check_hip(hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking), "hipStreamCreate");
      B->own_stream = true;
    }
    int dev = 0;
    check_hip(hipGetDevice(&dev), "hipGetDevice");
    for (size_t i = 0; i < n_inst; ++i) {
      auto v = std::make_unique<qs_state>();
      v->n = n_qubits[i];
      v->dtype = dtype;
      v->device = dev;
      v->buf[0] = (char*)B->arena + B->offset[i] * B->amp_bytes();
      v->view = true;
      v->stream = B->stream;
      B->views.push_back(std::move(v));
    }
    raw = B.release();
    qs_status st = qs_batch_refresh(raw);
    if (st != QS_OK) {
      std::string msg = g_last_error;
      delete raw;
      fail(st, msg);
    }
    *out = raw;
    return QS_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  } catch (const std::exception& e) {
    g_last_error = e.what();
    return QS_EINVAL;
  }
}

namespace qs {
void batch_plan_freed(qs_batch* b, const qs_plan* p) {
  for (auto& q : b->plans)
    if (q == p) {
      q = nullptr;
      b->plan_freed = true;
    }
}
}  // namespace qs

extern "C" qs_status qs_batch_refresh(qs_batch* b) {
  try {
    if (!b) fail(QS_EINVAL, "batch is NULL");
    if (b->plan_freed) fail(QS_EINVAL, "a plan of the batch has been freed");
    const Range range("qs.batch.record");
    for (auto* p : b->plans)
      if (!p->bound) fail(QS_EINVAL, "plan parameters are not bound");
    check_hip(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    if (!b->done) check_hip(hipEventCreateWithFlags(&b->done, hipEventDisableTiming), "hipEventCreateWithFlags");
    for (qs_plan* p : b->plans) p->add_external_user(b->dtype, b->stream, b->done, b);
    if (b->exec) {
      hipGraphExecDestroy(b->exec);
      b->exec = nullptr;
    }
    if (b->graph) {
      hipGraphDestroy(b->graph);
      b->graph = nullptr;
    }
    if (b->dtype == QS_C64) build_descs<float>(*b);
    else build_descs<double>(*b);
    prof_suspend(true);
    check_hip(hipStreamBeginCapture(b->stream, hipStreamCaptureModeThreadLocal), "hipStreamBeginCapture");
    try {
      if (b->dtype == QS_C64) record<float>(*b);
      else record<double>(*b);
    } catch (...) {
      hipGraph_t g = nullptr;
      hipStreamEndCapture(b->stream, &g);
      if (g) hipGraphDestroy(g);
      prof_suspend(false);
      throw;
    }
    check_hip(hipStreamEndCapture(b->stream, &b->graph), "hipStreamEndCapture");
    prof_suspend(false);
    check_hip(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0), "hipGraphInstantiate");
    return QS_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  }
}

extern "C" qs_status qs_batch_run(qs_batch* b) {
  try {
    if (!b || !b->exec) fail(QS_EINVAL, "batch is NULL or not recorded");
    if (b->plan_freed) fail(QS_EINVAL, "a plan of the batch has been freed");
    // tables re-uploaded since the batch last read them: wait for them on the
    // batch's stream (device-side)
    for (qs_plan* p : b->plans) p->sync_external_user(b->dtype, b->done, b->stream);
    prof_begin("batch_graph", b->stream);
    check_hip(hipGraphLaunch(b->exec, b->stream), "hipGraphLaunch");
    prof_end(b->stream);
    check_hip(hipEventRecord(b->done, b->stream), "hipEventRecord");
    return QS_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  }
}

namespace {

// Device image of per-instance Z-type observables: count tables and
// descriptors (host bytes, uploaded as one block), then room for the results
// (256-byte aligned) and the batched reduction's partial sums.
struct ObsImage {
  std::vector<unsigned char> host;
  size_t desc_off = 0, out_off = 0, part_off = 0, bytes = 0;
  std::vector<size_t> pos;  // instance -> position in group order
  std::vector<size_t> t_off, g_off, w_off, nb_off;
  std::vector<double> c0;
  std::vector<int> ng;
};

// The neighbour tables of the batched observable kernel (layout of ObsDev::nbr).
std::vector<int32_t> obs_neighbours(const DiagNumeric& num, int n) {
  const std::vector<PairNeighbours> pn = pair_neighbours(num, n);
  std::vector<int32_t> nb(pn.size() * kObsNbrStride, 0);
  for (size_t g = 0; g < pn.size(); ++g) {
    int32_t* T = nb.data() + g * kObsNbrStride;
    for (int p = 0; p < 32; ++p) {
      T[p] = (int32_t)pn[g].mask[p];
      T[32 + p] = pn[g].deg[p];
    }
    T[64] = pn[g].ok ? 1 : 0;
  }
  return nb;
}

ObsImage build_obs(const qs_batch* b, const qs_pauli* const* obs, const size_t* n_terms) {
  ObsImage I;
  I.t_off.resize(b->n_inst);
  I.g_off.resize(b->n_inst);
  I.w_off.resize(b->n_inst);
  I.nb_off.resize(b->n_inst);
  I.c0.resize(b->n_inst);
  I.ng.resize(b->n_inst);
  auto put = [&](const void* src, size_t bytes) {
    size_t off = (I.host.size() + 15) & ~size_t(15);
    I.host.resize(off + bytes + 16);
    if (bytes) std::memcpy(I.host.data() + off, src, bytes);
    return off;
  };
  for (size_t i = 0; i < b->n_inst; ++i) {
    if (n_terms[i] && !obs[i]) fail(QS_EINVAL, "NULL observable");
    DiagIR D = diag_observable(b->nq[i], obs[i], n_terms[i]);
    DiagNumeric num = diag_numeric(D, {});
    std::vector<double> w;
    for (auto& G : D.groups) w.push_back(G.angle.c0);
    // diag_numeric's first group has lut entries; only terms/groups are used here
    I.t_off[i] = put(num.terms.data(), num.terms.size() * sizeof(DiagTerm));
    I.g_off[i] = put(num.groups.data(), num.groups.size() * sizeof(DiagGroup));
    I.w_off[i] = put(w.data(), w.size() * sizeof(double));
    const std::vector<int32_t> nb = obs_neighbours(num, b->nq[i]);
    I.nb_off[i] = put(nb.data(), nb.size() * sizeof(int32_t));
    I.c0[i] = D.global.c0;
    I.ng[i] = (int)D.groups.size();
  }
  I.desc_off = (I.host.size() + 255) & ~size_t(255);
  I.host.resize(I.desc_off + b->n_inst * sizeof(ObsDev));
  size_t need_red = 0;
  for (auto& G : b->groups) need_red = std::max(need_red, batch_observable_partials((uint32_t)G.inst.size(), G.n));
  I.out_off = (I.host.size() + 255) & ~size_t(255);
  I.part_off = I.out_off + sizeof(double) * (b->n_inst + 8);
  I.bytes = I.part_off + sizeof(double) * need_red;
  I.pos.resize(b->n_inst);
  size_t k = 0;
  for (auto& G : b->groups)
    for (size_t i : G.inst) I.pos[i] = k++;
  return I;
}

// Fills the descriptors for device base `dev` and uploads the tables.
void upload_obs(const qs_batch* b, ObsImage& I, void* dev) {
  char* base = (char*)dev;
  for (size_t i = 0; i < b->n_inst; ++i) {
    ObsDev o;
    std::memset(&o, 0, sizeof o);
    o.psi = b->views[i]->buf[0];
    o.terms = (const DiagTerm*)(base + I.t_off[i]);
    o.groups = (const DiagGroup*)(base + I.g_off[i]);
    o.w = (const double*)(base + I.w_off[i]);
    o.nbr = (const int32_t*)(base + I.nb_off[i]);
    o.n_groups = I.ng[i];
    o.c0 = I.c0[i];
    std::memcpy(I.host.data() + I.desc_off + I.pos[i] * sizeof(ObsDev), &o, sizeof o);
  }
  check_hip(hipMemcpyAsync(dev, I.host.data(), I.host.size(), hipMemcpyHostToDevice, b->stream), "hipMemcpyAsync");
}

// One batched reduction per qubit-count group over uploaded observables, the
// per-instance results copied back (waits for the stream).
void run_obs(const qs_batch* b, void* dev, size_t desc_off, size_t out_off, size_t part_off,
             const std::vector<size_t>& pos, double* out) {
  char* base = (char*)dev;
  double* dout = (double*)(base + out_off);
  double* partials = (double*)(base + part_off);
  size_t first = 0;
  for (auto& G : b->groups) {
    const ObsDev* od_dev = (const ObsDev*)(base + desc_off) + first;
    if (b->dtype == QS_C64)
      launch_batch_observable<float>(od_dev, (uint32_t)G.inst.size(), G.n, partials, dout + first, b->stream);
    else
      launch_batch_observable<double>(od_dev, (uint32_t)G.inst.size(), G.n, partials, dout + first, b->stream);
    first += G.inst.size();
  }
  std::vector<double> res(b->n_inst);
  check_hip(hipMemcpyAsync(res.data(), dout, b->n_inst * sizeof(double), hipMemcpyDeviceToHost, b->stream),
            "hipMemcpyAsync");
  check_hip(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
  for (size_t i = 0; i < b->n_inst; ++i) out[i] = res[pos[i]];
}

}  // namespace

extern "C" qs_status qs_batch_expect_diag(qs_batch* b, const qs_pauli* const* obs, const size_t* n_terms,
                                          double* out) {
  try {
    if (!b || !obs || !n_terms || !out) fail(QS_EINVAL, "NULL argument");
    ObsImage I = build_obs(b, obs, n_terms);
    void* dev = nullptr;
    check_hip(hipMalloc(&dev, I.bytes), "hipMalloc");
    struct Guard {
      void* p;
      ~Guard() { hipFree(p); }
    } guard{dev};
    upload_obs(b, I, dev);
    run_obs(b, dev, I.desc_off, I.out_off, I.part_off, I.pos, out);
    return QS_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  }
}

extern "C" qs_status qs_batch_set_observables(qs_batch* b, const qs_pauli* const* obs, const size_t* n_terms) {
  try {
    if (!b || !obs || !n_terms) fail(QS_EINVAL, "NULL argument");
    ObsImage I = build_obs(b, obs, n_terms);
    void* dev = nullptr;
    check_hip(hipMalloc(&dev, I.bytes), "hipMalloc");
    try {
      upload_obs(b, I, dev);
      check_hip(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
    } catch (...) {
      hipFree(dev);
      throw;
    }
    if (b->obs_dev) {
      check_hip(hipStreamSynchronize(b->stream), "hipStreamSynchronize");
      hipFree(b->obs_dev);
    }
    b->obs_dev = dev;
    b->obs_desc_off = I.desc_off;
    b->obs_out_off = I.out_off;
    b->obs_part_off = I.part_off;
    b->obs_pos = I.pos;
    return QS_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  }
}

extern "C" qs_status qs_batch_expect_stored(qs_batch* b, double* out) {
  try {
    if (!b || !out) fail(QS_EINVAL, "NULL argument");
    if (!b->obs_dev) fail(QS_EINVAL, "no observables stored: call qs_batch_set_observables first");
    run_obs(b, b->obs_dev, b->obs_desc_off, b->obs_out_off, b->obs_part_off, b->obs_pos, out);
    return QS_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  }
}

extern "C" qs_status qs_batch_expect(qs_batch* b, const qs_pauli* const* obs, const size_t* n_terms, double* out) {
  try {
    if (!b || !obs || !n_terms || !out) fail(QS_EINVAL, "NULL argument");
    // Z-type terms of every instance in one batched reduction; terms with X or
    // Y factors per instance (pair reads on its state view)
    std::vector<std::vector<qs_pauli>> zt(b->n_inst), xt(b->n_inst);
    std::vector<const qs_pauli*> zp(b->n_inst);
    std::vector<size_t> zn(b->n_inst);
    for (size_t i = 0; i < b->n_inst; ++i) {
      if (n_terms[i] && !obs[i]) fail(QS_EINVAL, "NULL observable");
      for (size_t t = 0; t < n_terms[i]; ++t) (obs[i][t].x_mask ? xt[i] : zt[i]).push_back(obs[i][t]);
      zp[i] = zt[i].data();
      zn[i] = zt[i].size();
    }
    const qs_status st = qs_batch_expect_diag(b, zp.data(), zn.data(), out);
    if (st != QS_OK) return st;
    for (size_t i = 0; i < b->n_inst; ++i) {
      if (xt[i].empty()) continue;
      const std::vector<double> v = state_expect(*b->views[i], xt[i].data(), xt[i].size());
      for (double x : v) out[i] += x;
    }
    return QS_OK;
  } catch (const Error& e) {
    g_last_error = e.msg;
    return e.code;
  }
}

extern "C" qs_status qs_batch_state(qs_batch* b, size_t i, qs_state** view) {
  if (!b || !view || i >= b->n_inst) {
    g_last_error = "bad batch index";
    return QS_EINVAL;
  }
  *view = b->views[i].get();
  return QS_OK;
}

extern "C" qs_status qs_batch_free(qs_batch* b) {
  delete b;
  return QS_OK;
}
