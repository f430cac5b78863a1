// C ABI of the PTHR library (declared in include/pthr.h): validation, the
// device state layout, step-wise and fused EMCS launches, read-back,
// checkpointing and the launch-shape autotuner.  All device memory belongs to
// the caller; nothing here calls hipMalloc.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <chrono>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "pthr.h"
#include "pthr_internal.h"

namespace {

constexpr size_t kLdsLimit = pthr::kLdsMax;
constexpr uint64_t kBlobMagic = 0x5054485253544154ull;  // "PTHRSTAT"
constexpr int kMaxGroup = 64;  // contexts per group
constexpr double kLog2e = 0x1.71547652b82fep+0;  // RN(log2 e)

size_t align256(size_t v) { return (v + 255) / 256 * 256; }

// Byte offsets of every region of the caller's state buffer.
struct Layout {
  size_t beta64, beta32, T64, spins, J, beta_clone, clone_at, er_head, pt_last, pt_count, pt_energy, e_now, rt_state,
      rt_count, status, walker, J_plane, total;
};

struct Derived {
  int V, NPT, NER, C, NW, NWPT;
};

Derived derive(const pthr_params& p) {
  Derived d{};
  d.V = p.L * p.L * p.L;
  d.NPT = p.n_replicas * p.n_temps;
  d.NER = p.n_replicas * p.n_reservoir;
  d.C = d.NPT + d.NER;
  d.NWPT = (d.NPT + 31) / 32;
  d.NW = d.NWPT + (d.NER + 31) / 32;
  return d;
}

Layout layout_of(const pthr_params& p) {
  const Derived d = derive(p);
  const size_t S = p.n_samples, NR = p.n_replicas, NT = p.n_temps;
  const size_t fp = p.precision == PTHR_FP64 ? 8 : 4;
  Layout l{};
  size_t o = 256;  // header: the EMCS counter t (uint32) at offset 0
  l.beta64 = o;    o = align256(o + 8 * NT);
  l.beta32 = o;    o = align256(o + 4 * NT);
  l.T64 = o;       o = align256(o + 8 * NT);
  l.spins = o;     o = align256(o + 4 * S * d.NW * d.V);
  l.J = o;         o = align256(o + fp * S * 3 * d.V);
  // + 16 bytes: the sweep reads the factors of a Philox block's clones as one
  // contiguous load, and a partial last block reaches up to 3 (FP32) or 1
  // (FP64) entries past the table
  l.beta_clone = o; o = align256(o + fp * S * d.C + 16);
  l.clone_at = o;  o = align256(o + 4 * S * NR * NT);
  l.er_head = o;   o = align256(o + 4 * S * NR);
  l.pt_last = o;   o = align256(o + S * NR * (NT - 1));
  l.pt_count = o;  o = align256(o + 4 * S * NR * (NT - 1));
  l.pt_energy = o; o = align256(o + 8 * S * d.NPT);
  l.e_now = o;     o = align256(o + 8 * S * d.NPT);
  l.rt_state = o;  o = align256(o + S * d.NPT);
  l.rt_count = o;  o = align256(o + 8 * S);
  l.status = o;    o = align256(o + 4 * S);
  l.walker = o;    o = align256(o + 8 * S * d.NPT);
  // FP32 MicSA whose row kernel reads the couplings through the scalar cache
  // (4 <= L <= 16, two samples' spin words fit in LDS): the couplings again,
  // in plane order
  const bool j_plane = p.precision == PTHR_FP32 && p.local_update == PTHR_MICSA &&
                       pthr::micsa_scalar_couplings(p.L, d.NWPT, int(NR * NT), d.NPT);
  l.J_plane = j_plane ? o : 0;
  if (j_plane) o = align256(o + 4 * S * 3 * d.V);
  l.total = o;
  return l;
}

pthr::Geo geo_of(const pthr_params& p, int K_acu) {
  const Derived d = derive(p);
  pthr::Geo g{};
  g.L = p.L;
  g.V = d.V;
  g.Vh = d.V / 2;
  g.S = p.n_samples;
  g.NR = p.n_replicas;
  g.NT = p.n_temps;
  g.NERG = p.n_reservoir;
  g.NPT = d.NPT;
  g.NER = d.NER;
  g.C = d.C;
  g.NW = d.NW;
  g.NWPT = d.NWPT;
  g.K_acu = K_acu;
  g.mode = p.houdayer_mode;
  g.update = p.local_update;
  g.micsa_refresh = p.micsa_refresh > 0 ? p.micsa_refresh : (p.sweeps_per_emcs > 0 ? p.sweeps_per_emcs : 1);
  g.exp_lo = 0x1.ffffep-1f;  // 1 - 2^-20
  g.exp_hi = 0x1.00001p+0f;  // 1 + 2^-20
  g.key0 = static_cast<uint32_t>(p.seed);
  g.key1 = static_cast<uint32_t>(p.seed >> 32);
  return g;
}

int threads_for(int V, int chunk) { return (V / chunk + 63) / 64 * 64; }
// Chunk sizes with a compiled kernel: FP64 keeps 12 doubles per pair of sites
// in registers, so it stops at 4 sites per work-item.
bool chunk_ok(int precision, int V, int chunk) {
  if (precision == PTHR_FP64 && chunk > 4) return false;
  return threads_for(V, chunk) <= 1024 && V / chunk >= 1;
}
// Smallest chunk (most work-items per sample) with a compiled kernel; 0 if none.
int default_chunk(int precision, int V) {
  for (int ch = 2; ch <= 8; ch *= 2)
    if (chunk_ok(precision, V, ch)) return ch;
  return 0;
}

thread_local std::string g_create_error;

constexpr int kMaxDevices = 64;
std::mutex& device_mu() {
  static std::mutex mu;
  return mu;
}
// Per device: address of the static autotuning workspace (null until the
// device's first set-up), which also marks the kernels as prepared there.
void** device_scratch() {
  static void* ptr[kMaxDevices] = {};
  return ptr;
}

const char* validate(const pthr_params& p) {
  if (p.L < 2 || p.L > 32) return "L must be in [2, 32]";
  if (p.L % 2) return "odd L is not supported on the GPU (the checkerboard is not a bipartition)";
  if (p.n_samples < 1 || p.n_samples > (1 << 24)) return "n_samples must be in [1, 2^24]";
  if (p.n_replicas < 2 || p.n_replicas > 32 || p.n_replicas % 2) return "n_replicas must be even, in [2, 32]";
  if (p.n_temps < 2 || p.n_temps > 1024) return "n_temps must be in [2, 1024]";
  if (p.n_reservoir < 0 || p.n_reservoir > 64) return "n_reservoir must be in [0, 64]";
  if (p.sweeps_per_emcs < 0 || p.sweeps_per_emcs > 256) return "sweeps_per_emcs must be in [0, 256]";
  if (p.er_sweeps_per_emcs < 0 || p.er_sweeps_per_emcs > 256) return "er_sweeps_per_emcs must be in [0, 256]";
  if (p.precision != PTHR_FP64 && p.precision != PTHR_FP32) return "precision must be PTHR_FP64 or PTHR_FP32";
  if (p.houdayer_mode != PTHR_ACU && p.houdayer_mode != PTHR_SINGLE_NEG) return "houdayer_mode must be PTHR_ACU or PTHR_SINGLE_NEG";
  if (p.local_update != PTHR_METROPOLIS && p.local_update != PTHR_HEAT_BATH && p.local_update != PTHR_MICSA)
    return "local_update must be PTHR_METROPOLIS, PTHR_HEAT_BATH or PTHR_MICSA";
  if (p.micsa_refresh < 0 || p.micsa_refresh > 256) return "micsa_refresh must be in [0, 256]";
  if (std::isnan(p.t_acu)) return "t_acu must not be NaN";
  return nullptr;
}

}  // namespace

struct pthr_ctx {
  pthr_params p{};
  Derived d{};
  Layout lay{};
  pthr::Geo g{};
  unsigned char* d_state = nullptr;
  bool ready = false;
  int64_t t = 0;
  int m_pt = 0, m_er = 0;
  // e_now in the state buffer holds the energies of the current configurations
  // (set by the PT step, cleared by anything that changes spins)
  bool e_current = false;
  int K_acu = 0;
  std::vector<double> T;
  pthr_schedule sch{};
  std::vector<std::pair<pthr_schedule, double>> tune;  // last autotuning: candidate, ms per EMCS
  std::string err;
  // captured EMCS window for pthr_run
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  int g_window = 0;
  void* g_obs = nullptr;
  unsigned char* g_state = nullptr;
  pthr_schedule g_sch{};

  int n_cu = 256;  // compute units of the device the context was made on
  // overlap_reservoir: the second stream and the fork / join events
  hipStream_t side_stream = nullptr;
  hipEvent_t ev_fork = nullptr, ev_join = nullptr;

  ~pthr_ctx() {
    drop_graph();
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (side_stream) (void)hipStreamDestroy(side_stream);
    if (ev_fork) (void)hipEventDestroy(ev_fork);
    if (ev_join) (void)hipEventDestroy(ev_join);
  }
  bool overlapping() const { return sch.overlap_reservoir && d.NER > 0 && p.er_sweeps_per_emcs > 0; }
  // Creates the second stream and its events (once; never inside a capture).
  int make_side() {
    hipError_t e = hipSuccess;
    if (!side_stream && (e = hipStreamCreateWithFlags(&side_stream, hipStreamNonBlocking)) != hipSuccess)
      return hip_fail(e, "second stream");
    if (!ev_fork && (e = hipEventCreateWithFlags(&ev_fork, hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e, "fork event");
    if (!ev_join && (e = hipEventCreateWithFlags(&ev_join, hipEventDisableTiming)) != hipSuccess)
      return hip_fail(e, "join event");
    return PTHR_OK;
  }
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
    g_window = 0;
  }

  int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return code;
  }
  int hip_fail(hipError_t e, const char* what) {
    return fail(PTHR_EHIP, "%s: %s", what, hipGetErrorString(e));
  }
  pthr::State state() const {
    pthr::State st{};
    unsigned char* b = d_state;
    st.t_dev = reinterpret_cast<uint32_t*>(b);  // first word of the reserved header
    st.spins = reinterpret_cast<uint32_t*>(b + lay.spins);
    st.J = b + lay.J;
    st.clone_at = reinterpret_cast<int32_t*>(b + lay.clone_at);
    st.er_head = reinterpret_cast<int32_t*>(b + lay.er_head);
    st.pt_last = b + lay.pt_last;
    st.pt_count = reinterpret_cast<uint32_t*>(b + lay.pt_count);
    st.pt_energy = reinterpret_cast<double*>(b + lay.pt_energy);
    st.e_now = reinterpret_cast<double*>(b + lay.e_now);
    st.rt_state = b + lay.rt_state;
    st.rt_count = reinterpret_cast<uint64_t*>(b + lay.rt_count);
    st.status = reinterpret_cast<uint32_t*>(b + lay.status);
    st.beta64 = reinterpret_cast<const double*>(b + lay.beta64);
    st.beta32 = reinterpret_cast<const float*>(b + lay.beta32);
    st.beta_clone = b + lay.beta_clone;
    st.T64 = reinterpret_cast<const double*>(b + lay.T64);
    st.walker = reinterpret_cast<double*>(b + lay.walker);
    st.J_plane = lay.J_plane ? reinterpret_cast<float*>(b + lay.J_plane) : nullptr;
    return st;
  }
  pthr::Obs obs(void* d_obs) const {
    pthr::Obs o{};
    if (d_obs) {
      unsigned char* b = static_cast<unsigned char*>(d_obs);
      o.n_meas = reinterpret_cast<uint64_t*>(b);
      o.acc = reinterpret_cast<double*>(b + pthr_obs_acc_offset(&p));
      o.hist = reinterpret_cast<uint64_t*>(b + pthr_obs_hist_offset(&p));
    }
    return o;
  }
  pthr::Shape shape() const {
    pthr::Shape sh{};
    sh.threads = sch.threads_per_sample;
    sh.split = sch.clone_split;
    sh.parts = sch.sample_split;
    sh.chunk = 2;  // smallest chunk giving this many work-items (checked by set_schedule)
    while (threads_for(d.V, sh.chunk) != sch.threads_per_sample && sh.chunk < 8) sh.chunk *= 2;
    return sh;
  }
  // Launches `run` over all samples, split by samples_per_launch;
  // `shared_gpu`: other contexts' kernels run beside these (a group).
  int launch(pthr::Run run, void* d_obs, hipStream_t stream, bool shared_gpu = false) {
    const pthr::State st = state();
    const pthr::Obs ob = obs(d_obs);
    const int per = sch.samples_per_launch > 0 ? sch.samples_per_launch : p.n_samples;
    // exp early-out for clones colder than exp_early_out/1000 (0 = never)
    // (the FP32 form keeps beta log2 e per clone)
    const double unit = p.precision == PTHR_FP32 ? kLog2e : 1.0;
    run.early_beta = sch.exp_early_out > 0 ? static_cast<float>(1000.0 / sch.exp_early_out * unit) : 3.0e38f;
    for (int s0 = 0; s0 < p.n_samples; s0 += per) {
      run.sample_begin = s0;
      const int nb = std::min(per, p.n_samples - s0);
      pthr::Geo gl = g;
      if (!sch.exp_filter) {
        gl.exp_lo = 0.0f;
        gl.exp_hi = INFINITY;
      }
      pthr::Shape sh = shape();
      // more sample workgroups than CUs, or other work beside them: the
      // Houdayer kernel may take fewer moves at once for more workgroups per CU
      sh.hou_occupancy = shared_gpu || nb > n_cu;
      hipError_t e = pthr::launch_emcs(p.precision, gl, st, ob, run, sh, nb, stream);
      if (e != hipSuccess) return hip_fail(e, "EMCS kernel launch");
    }
    return PTHR_OK;
  }
  // Once per device and process: raises the kernels' dynamic-LDS limit and
  // looks up the device address of the static autotuning workspace.
  int prepare() {
    std::lock_guard<std::mutex> lock(device_mu());
    int dev = 0;
    hipError_t e = hipGetDevice(&dev);
    if (e != hipSuccess) return hip_fail(e, "get device");
    if (dev < 0 || dev >= kMaxDevices) return fail(PTHR_EUNSUPPORTED, "device %d: at most %d devices", dev, kMaxDevices);
    if (device_scratch()[dev]) return PTHR_OK;
    e = pthr::prepare_kernels(kLdsLimit);
    if (e != hipSuccess) return hip_fail(e, "kernel attributes");
    void* ptr = nullptr;
    e = pthr::scratch_address(&ptr);
    if (e != hipSuccess || !ptr) return hip_fail(e, "workspace address");
    device_scratch()[dev] = ptr;
    return PTHR_OK;
  }
  // One whole EMCS on `stream`: sweeps, Houdayer, PT + reservoir (all
  // samples), t += 1, then the observables if d_obs is set.
  int emcs(void* d_obs, hipStream_t stream, bool shared_gpu = false) {
    pthr::Run run{};
    run.phases = pthr::kPhaseSweep | (K_acu ? pthr::kPhaseHoudayer : 0u) | pthr::kPhasePT;
    run.n_pt = p.sweeps_per_emcs;
    run.n_er = d.NER > 0 ? p.er_sweeps_per_emcs : 0;
    run.do_reservoir = 1;
    hipError_t e = hipSuccess;
    if (overlapping()) {
      // reservoir sweeps on the second stream, PT sweeps and the Houdayer step
      // on this one (disjoint spin words), joined before the PT step
      if (!side_stream || !ev_fork || !ev_join) return fail(PTHR_ESTATE, "second stream not created");
      if ((e = hipEventRecord(ev_fork, stream)) != hipSuccess ||
          (e = hipStreamWaitEvent(side_stream, ev_fork, 0)) != hipSuccess)
        return hip_fail(e, "fork");
      pthr::Run er{};
      er.phases = pthr::kPhaseSweep;
      er.n_er = run.n_er;
      if (int rc = launch(er, nullptr, side_stream, shared_gpu)) return rc;
      pthr::Run pt = run;
      pt.phases &= ~pthr::kPhasePT;
      pt.n_er = 0;
      if (int rc = launch(pt, nullptr, stream, shared_gpu)) return rc;
      if ((e = hipEventRecord(ev_join, side_stream)) != hipSuccess ||
          (e = hipStreamWaitEvent(stream, ev_join, 0)) != hipSuccess)
        return hip_fail(e, "join");
      pthr::Run ps{};
      ps.phases = pthr::kPhasePT;
      ps.do_reservoir = 1;
      if (int rc = launch(ps, nullptr, stream, shared_gpu)) return rc;
    } else {
      if (int rc = launch(run, nullptr, stream, shared_gpu)) return rc;
    }
    e = pthr::launch_advance_t(state(), stream);
    if (e != hipSuccess) return hip_fail(e, "advance t");
    if (d_obs) {
      pthr::Run m{};
      m.phases = pthr::kPhaseMeasure;
      m.e_current = 1;  // the PT step just left the current energies in e_now
      if (int rc = launch(m, d_obs, stream, shared_gpu)) return rc;
    }
    return PTHR_OK;
  }
  // Instantiates (or reuses) a graph of `window` EMCS for the current buffers
  // and schedule.  The graph reads t from the state buffer, so it can be
  // replayed any number of times.
  int graph(int window, void* d_obs) {
    if (gexec && g_window == window && g_obs == d_obs && g_state == d_state &&
        std::memcmp(&g_sch, &sch, sizeof sch) == 0)
      return PTHR_OK;
    drop_graph();
    hipError_t e = hipSuccess;
    if (!cap_stream) e = hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return hip_fail(e, "capture stream");
    if (overlapping()) return fail(PTHR_EUNSUPPORTED, "overlap_reservoir runs as plain launches (graph_window = 0)");
    if ((e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return hip_fail(e, "begin capture");
    int rc = PTHR_OK;
    for (int w = 0; w < window && rc == PTHR_OK; ++w) rc = emcs(d_obs, cap_stream);
    hipGraph_t gr = nullptr;
    e = hipStreamEndCapture(cap_stream, &gr);
    if (rc != PTHR_OK) {
      if (gr) (void)hipGraphDestroy(gr);
      return rc;
    }
    if (e != hipSuccess) return hip_fail(e, "end capture");
    e = hipGraphInstantiate(&gexec, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) {
      gexec = nullptr;
      return hip_fail(e, "graph instantiation");
    }
    g_window = window;
    g_obs = d_obs;
    g_state = d_state;
    g_sch = sch;
    return PTHR_OK;
  }
  int need_ready() {
    if (!ready) return fail(PTHR_ESTATE, "state buffer not initialised (call pthr_init_samples)");
    return PTHR_OK;
  }
};

extern "C" {

const char* pthr_create_error(void) { return g_create_error.c_str(); }

size_t pthr_state_bytes(const pthr_params* p) {
  if (!p || validate(*p)) return 0;
  return layout_of(*p).total;
}

size_t pthr_lds_bytes(const pthr_params* p) {
  if (!p || validate(*p)) return 0;
  return pthr::lds_bytes(geo_of(*p, 0), p->precision == PTHR_FP64 ? 8 : 4);
}

size_t pthr_obs_acc_offset(const pthr_params* p) { return p ? 256 : 0; }
size_t pthr_obs_hist_offset(const pthr_params* p) {
  if (!p) return 0;
  return align256(256 + sizeof(double) * size_t(p->n_samples) * p->n_temps * PTHR_NOBS);
}
size_t pthr_obs_bytes(const pthr_params* p) {
  if (!p || validate(*p)) return 0;
  const size_t V = size_t(p->L) * p->L * p->L;
  return align256(pthr_obs_hist_offset(p) + sizeof(uint64_t) * size_t(p->n_temps) * (V + 1));
}

int pthr_create(const pthr_params* p, pthr_ctx** out) {
  if (!out) {
    g_create_error = "out must not be NULL";
    return PTHR_EINVAL;
  }
  *out = nullptr;
  if (!p) {
    g_create_error = "params must not be NULL";
    return PTHR_EINVAL;
  }
  if (const char* msg = validate(*p)) {
    g_create_error = msg;
    return (p->L % 2 && p->L >= 2 && p->L <= 32) ? PTHR_EUNSUPPORTED : PTHR_EINVAL;
  }
  const Derived d = derive(*p);
  if (default_chunk(p->precision, d.V) == 0) {
    g_create_error = "lattice too large for one workgroup per sample (V > 8192, or V > 4096 in FP64)";
    return PTHR_EUNSUPPORTED;
  }
  const size_t lds = pthr::lds_bytes(geo_of(*p, 0), p->precision == PTHR_FP64 ? 8 : 4);
  if (lds > kLdsLimit) {
    char buf[256];
    snprintf(buf, sizeof buf, "sample does not fit in LDS: needs %zu bytes, limit %zu", lds, kLdsLimit);
    g_create_error = buf;
    return PTHR_EUNSUPPORTED;
  }
  pthr_ctx* c = new pthr_ctx();
  c->p = *p;
  c->d = d;
  c->lay = layout_of(*p);
  c->g = geo_of(*p, 0);
  int n_cu = 256, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || n_cu < 1) {
    n_cu = 256;                // no device visible here: size for an MI355X
    (void)hipGetLastError();   // and leave no error behind for later calls
  }
  c->n_cu = n_cu;
  int ch = default_chunk(p->precision, d.V);
  // FP32 sweeps a last reservoir word of 16 clones two sites at a time when a
  // work-item owns two sites of a colour: for batches of at least two samples
  // per CU, 4 sites per work-item is then the faster default wherever it
  // still gives a sample 4 or more waves
  if (p->precision == PTHR_FP32 && ch == 2 && d.NER % 32 == 16 && chunk_ok(PTHR_FP32, d.V, 4) &&
      threads_for(d.V, 4) >= 256 && int64_t(p->n_samples) >= 2 * int64_t(n_cu))
    ch = 4;
  c->sch.threads_per_sample = threads_for(d.V, ch);
  c->sch.samples_per_launch = 0;
  c->sch.exp_early_out = 0;  // the branch-free exponential for every clone (fastest on gfx950)
  c->sch.exp_filter = 1;
  c->sch.graph_window = 16;
  // Batches too small to fill the GPU with waves (4 per SIMD at the sweep's
  // register use): share each chunk's clone words among 2 or 4 waves, up to
  // 1024 work-items per workgroup and one GPU's worth of waves.
  const int64_t waves = int64_t(p->n_samples) * (c->sch.threads_per_sample / 64);
  c->sch.clone_split = 1;
  while (c->sch.clone_split < 4 && c->sch.threads_per_sample * c->sch.clone_split * 2 <= 1024 &&
         waves * c->sch.clone_split * 2 <= int64_t(n_cu) * 16)
    c->sch.clone_split *= 2;
  // Fewer sample workgroups than compute units (one GPU's share of a sharded
  // batch): the sweep takes 2 or 4 workgroups per sample.
  c->sch.sample_split = 1;
  while (c->sch.sample_split < 4 && int64_t(p->n_samples) * c->sch.sample_split < n_cu) c->sch.sample_split *= 2;
  *out = c;
  g_create_error.clear();
  return PTHR_OK;
}

int pthr_destroy(pthr_ctx* ctx) {
  delete ctx;
  return PTHR_OK;
}

const char* pthr_last_error(const pthr_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int pthr_init_samples(pthr_ctx* ctx, const double* J_host, const double* T_host, void* d_state, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (!J_host || !T_host || !d_state) return ctx->fail(PTHR_EINVAL, "J, T and d_state must not be NULL");
  if (int rc = ctx->prepare()) return rc;
  ctx->drop_graph();
  if (reinterpret_cast<uintptr_t>(d_state) % 256) return ctx->fail(PTHR_EINVAL, "d_state must be 256-byte aligned");
  const pthr_params& p = ctx->p;
  const int NT = p.n_temps;
  for (int k = 0; k < NT; ++k) {
    if (!(T_host[k] > 0.0) || !std::isfinite(T_host[k]))
      return ctx->fail(PTHR_EINVAL, "T[%d] must be finite and > 0", k);
    if (k > 0 && !(T_host[k] > T_host[k - 1])) return ctx->fail(PTHR_EINVAL, "T must be strictly increasing");
  }
  const size_t nJ = size_t(p.n_samples) * 3 * ctx->d.V;
  for (size_t n = 0; n < nJ; ++n)
    if (!std::isfinite(J_host[n])) return ctx->fail(PTHR_EINVAL, "J[%zu] is not finite", n);
  if (p.precision == PTHR_FP32) {
    // The FP32 sweep rounds its exponent t = -(beta log2 e) dE to an integer
    // with the float adder, exact while |t| < 2^22; |dE| <= 12 max|J|.
    double jmax = 0.0;
    for (size_t n = 0; n < nJ; ++n) jmax = std::max(jmax, std::fabs(static_cast<double>(static_cast<float>(J_host[n]))));
    const double tmax = static_cast<double>(static_cast<float>(1.0 / T_host[0] * kLog2e)) * 12.0 * jmax * 1.001;
    if (!(tmax < 4194304.0))
      return ctx->fail(PTHR_EINVAL,
                       "FP32 form: beta_max log2(e) 12 max|J| = %g must stay below 2^22 (raise T_min or use FP64)",
                       tmax);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  // host image of the small regions and the couplings
  std::vector<double> b64(NT);
  std::vector<float> b32(NT);
  for (int k = 0; k < NT; ++k) {
    b64[k] = 1.0 / T_host[k];
    b32[k] = static_cast<float>(b64[k] * kLog2e);  // the FP32 form's Metropolis factor beta log2 e
  }
  int K = 0;
  while (K < NT && T_host[K] < p.t_acu) ++K;
  ctx->K_acu = K;
  ctx->g = geo_of(p, K);
  ctx->T.assign(T_host, T_host + NT);
  ctx->d_state = static_cast<unsigned char*>(d_state);
  const Layout& l = ctx->lay;
  hipError_t e;
  e = hipMemcpyAsync(ctx->d_state + l.beta64, b64.data(), 8 * NT, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(ctx->d_state + l.beta32, b32.data(), 4 * NT, hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipMemcpyAsync(ctx->d_state + l.T64, T_host, 8 * NT, hipMemcpyHostToDevice, s);
  std::vector<float> J32;
  if (e == hipSuccess) {
    if (p.precision == PTHR_FP64) {
      e = hipMemcpyAsync(ctx->d_state + l.J, J_host, 8 * nJ, hipMemcpyHostToDevice, s);
    } else {
      J32.resize(nJ);
      for (size_t n = 0; n < nJ; ++n) J32[n] = static_cast<float>(J_host[n]);
      e = hipMemcpyAsync(ctx->d_state + l.J, J32.data(), 4 * nJ, hipMemcpyHostToDevice, s);
    }
  }
  const size_t S = p.n_samples, NR = p.n_replicas;
  // every clone starts at its own temperature; reservoir clones are at T_max
  std::vector<double> bc64(S * ctx->d.C);
  std::vector<float> bc32(S * ctx->d.C);
  for (size_t smp = 0; smp < S; ++smp)
    for (int c = 0; c < ctx->d.C; ++c) {
      const int k = c < ctx->d.NPT ? c % NT : NT - 1;
      bc64[smp * ctx->d.C + c] = b64[k];
      bc32[smp * ctx->d.C + c] = b32[k];
    }
  if (e == hipSuccess)
    e = p.precision == PTHR_FP64
            ? hipMemcpyAsync(ctx->d_state + l.beta_clone, bc64.data(), 8 * bc64.size(), hipMemcpyHostToDevice, s)
            : hipMemcpyAsync(ctx->d_state + l.beta_clone, bc32.data(), 4 * bc32.size(), hipMemcpyHostToDevice, s);
  std::vector<int32_t> cat(S * NR * NT);
  for (size_t x = 0; x < cat.size(); ++x) cat[x] = static_cast<int32_t>(x % (NR * NT));
  if (e == hipSuccess) e = hipMemcpyAsync(ctx->d_state + l.clone_at, cat.data(), 4 * cat.size(), hipMemcpyHostToDevice, s);
  if (e != hipSuccess) return ctx->hip_fail(e, "copy to the state buffer");
  // zero the header (t) and the counters and bookkeeping regions with a kernel
  const size_t zero_from = l.er_head, zero_to = l.total;
  e = pthr::launch_zero(ctx->d_state, 256, s);
  if (e == hipSuccess) e = pthr::launch_zero(ctx->d_state + zero_from, zero_to - zero_from, s);
  if (e == hipSuccess) e = pthr::launch_init(ctx->g, ctx->state(), s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // host staging buffers go out of scope
  if (e != hipSuccess) return ctx->hip_fail(e, "state initialisation");
  ctx->t = 0;
  ctx->m_pt = ctx->m_er = 0;
  ctx->e_current = false;
  ctx->ready = true;
  return PTHR_OK;
}

int pthr_sweep(pthr_ctx* ctx, int n_pt, int n_er, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (int rc = ctx->need_ready()) return rc;
  if (n_pt < 0 || n_er < 0) return ctx->fail(PTHR_EINVAL, "sweep counts must be >= 0");
  if (ctx->d.NER == 0) n_er = 0;
  if (ctx->m_pt + n_pt > 256 || ctx->m_er + n_er > 256)
    return ctx->fail(PTHR_ESTATE, "more than 256 sweeps in one EMCS (sweep counter field is 8 bits)");
  if (n_pt == 0 && n_er == 0) return PTHR_OK;
  pthr::Run run{};
  run.phases = pthr::kPhaseSweep;
  run.m_pt0 = ctx->m_pt;
  run.n_pt = n_pt;
  run.m_er0 = ctx->m_er;
  run.n_er = n_er;
  if (int rc = ctx->launch(run, nullptr, static_cast<hipStream_t>(stream))) return rc;
  ctx->m_pt += n_pt;
  ctx->m_er += n_er;
  ctx->e_current = false;
  return PTHR_OK;
}

int pthr_houdayer(pthr_ctx* ctx, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (int rc = ctx->need_ready()) return rc;
  if (ctx->K_acu == 0) return PTHR_OK;
  pthr::Run run{};
  run.phases = pthr::kPhaseHoudayer;
  ctx->e_current = false;
  return ctx->launch(run, nullptr, static_cast<hipStream_t>(stream));
}

int pthr_pt_swap(pthr_ctx* ctx, int do_reservoir, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (int rc = ctx->need_ready()) return rc;
  if (ctx->t >= 0xFFFFFFFFll) return ctx->fail(PTHR_ESTATE, "EMCS counter exhausted (2^32)");
  pthr::Run run{};
  run.phases = pthr::kPhasePT;
  run.do_reservoir = do_reservoir ? 1 : 0;
  if (int rc = ctx->launch(run, nullptr, static_cast<hipStream_t>(stream))) return rc;
  hipError_t e = pthr::launch_advance_t(ctx->state(), static_cast<hipStream_t>(stream));
  if (e != hipSuccess) return ctx->hip_fail(e, "advance t");
  ctx->t += 1;
  ctx->m_pt = ctx->m_er = 0;
  ctx->e_current = true;
  return PTHR_OK;
}

int pthr_measure(pthr_ctx* ctx, void* d_obs, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (int rc = ctx->need_ready()) return rc;
  if (!d_obs) return ctx->fail(PTHR_EINVAL, "d_obs must not be NULL");
  pthr::Run run{};
  run.phases = pthr::kPhaseMeasure;
  run.e_current = ctx->e_current ? 1 : 0;
  return ctx->launch(run, d_obs, static_cast<hipStream_t>(stream));
}

int pthr_obs_clear(pthr_ctx* ctx, void* d_obs, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (!d_obs) return ctx->fail(PTHR_EINVAL, "d_obs must not be NULL");
  hipError_t e = pthr::launch_zero(d_obs, pthr_obs_bytes(&ctx->p), static_cast<hipStream_t>(stream));
  return e == hipSuccess ? PTHR_OK : ctx->hip_fail(e, "obs clear");
}

int pthr_run(pthr_ctx* ctx, int64_t n_emcs, void* d_obs, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (int rc = ctx->need_ready()) return rc;
  if (n_emcs < 0) return ctx->fail(PTHR_EINVAL, "n_emcs must be >= 0");
  if (ctx->m_pt || ctx->m_er) return ctx->fail(PTHR_ESTATE, "an EMCS is in progress (sweep counters not at 0)");
  if (ctx->t + n_emcs > 0xFFFFFFFFll) return ctx->fail(PTHR_ESTATE, "EMCS counter would pass 2^32");
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int W = ctx->sch.graph_window;
  if (ctx->overlapping()) {
    if (W > 0) return ctx->fail(PTHR_EUNSUPPORTED, "overlap_reservoir runs as plain launches (graph_window = 0)");
    if (int rc = ctx->make_side()) return rc;
  }
  int64_t done = 0;
  if (W > 0 && n_emcs >= W) {
    if (int rc = ctx->graph(W, d_obs)) return rc;
    for (; done + W <= n_emcs; done += W) {
      hipError_t e = hipGraphLaunch(ctx->gexec, s);
      if (e != hipSuccess) return ctx->hip_fail(e, "graph launch");
      ctx->t += W;
    }
  }
  for (; done < n_emcs; ++done) {
    if (int rc = ctx->emcs(d_obs, s)) return rc;
    ctx->t += 1;
  }
  if (n_emcs > 0) ctx->e_current = true;
  return PTHR_OK;
}

int pthr_cluster_stats(pthr_ctx* ctx, void* d_sizes, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (int rc = ctx->need_ready()) return rc;
  if (!d_sizes) return ctx->fail(PTHR_EINVAL, "d_sizes must not be NULL");
  if (ctx->K_acu == 0) return PTHR_OK;
  if (pthr::houdayer_plan(ctx->g, ctx->sch.threads_per_sample, true, false, false).M < 1)
    return ctx->fail(PTHR_EUNSUPPORTED, "cluster statistics need more LDS than one workgroup has at this size");
  pthr::Run run{};
  run.phases = pthr::kPhaseClusterStats;
  run.labels = static_cast<int32_t*>(d_sizes);
  return ctx->launch(run, nullptr, static_cast<hipStream_t>(stream));
}

int pthr_cluster_labels(pthr_ctx* ctx, void* d_labels, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (int rc = ctx->need_ready()) return rc;
  if (!d_labels) return ctx->fail(PTHR_EINVAL, "d_labels must not be NULL");
  if (ctx->K_acu == 0) return PTHR_OK;
  pthr::Run run{};
  run.phases = pthr::kPhaseLabels;
  run.labels = static_cast<int32_t*>(d_labels);
  return ctx->launch(run, nullptr, static_cast<hipStream_t>(stream));
}

int pthr_read_spins(pthr_ctx* ctx, int8_t* spins, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (int rc = ctx->need_ready()) return rc;
  if (!spins) return ctx->fail(PTHR_EINVAL, "spins must not be NULL");
  const Derived& d = ctx->d;
  const size_t S = ctx->p.n_samples;
  std::vector<uint32_t> words(S * d.NW * d.V);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(words.data(), ctx->d_state + ctx->lay.spins, 4 * words.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return ctx->hip_fail(e, "read spins");
  const int L = ctx->p.L, Vh = d.V / 2;
  for (size_t smp = 0; smp < S; ++smp)
    for (int c = 0; c < d.C; ++c) {
      const int w = c < d.NPT ? c / 32 : d.NWPT + (c - d.NPT) / 32;
      const int b = c < d.NPT ? c % 32 : (c - d.NPT) % 32;
      const uint32_t* plane = words.data() + (smp * d.NW + w) * d.V;
      int8_t* out = spins + (smp * d.C + c) * d.V;
      for (int i = 0; i < d.V; ++i) {
        const int x = i % L, y = (i / L) % L, z = i / (L * L);
        const int j = ((x + y + z) & 1) * Vh + (i >> 1);
        out[i] = ((plane[j] >> b) & 1u) ? -1 : 1;
      }
    }
  return PTHR_OK;
}

int pthr_write_spins(pthr_ctx* ctx, const int8_t* spins, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (int rc = ctx->need_ready()) return rc;
  if (!spins) return ctx->fail(PTHR_EINVAL, "spins must not be NULL");
  const Derived& d = ctx->d;
  const size_t S = ctx->p.n_samples;
  const size_t n = S * d.C * d.V;
  for (size_t x = 0; x < n; ++x)
    if (spins[x] != 1 && spins[x] != -1) return ctx->fail(PTHR_EINVAL, "spins[%zu] = %d is not +1 or -1", x, spins[x]);
  // bit b of word w at plane index j: clone 32w+b (PT) or NPT+32(w-NWPT)+b (ER); set = spin down
  std::vector<uint32_t> words(S * d.NW * d.V, 0u);
  const int L = ctx->p.L, Vh = d.V / 2;
  for (size_t smp = 0; smp < S; ++smp)
    for (int c = 0; c < d.C; ++c) {
      const int w = c < d.NPT ? c / 32 : d.NWPT + (c - d.NPT) / 32;
      const int b = c < d.NPT ? c % 32 : (c - d.NPT) % 32;
      uint32_t* plane = words.data() + (smp * d.NW + w) * d.V;
      const int8_t* in = spins + (smp * d.C + c) * d.V;
      for (int i = 0; i < d.V; ++i) {
        const int x = i % L, y = (i / L) % L, z = i / (L * L);
        const int j = ((x + y + z) & 1) * Vh + (i >> 1);
        if (in[i] < 0) plane[j] |= 1u << b;
      }
    }
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(ctx->d_state + ctx->lay.spins, words.data(), 4 * words.size(), hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);  // the staging vector goes out of scope
  if (e != hipSuccess) return ctx->hip_fail(e, "write spins");
  ctx->e_current = false;
  return PTHR_OK;
}

int pthr_read_pt(pthr_ctx* ctx, int32_t* clone_at, int32_t* er_head, uint8_t* pt_last, uint32_t* pt_count,
                 double* pt_energy, uint8_t* rt_state, uint64_t* rt_count, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (int rc = ctx->need_ready()) return rc;
  const size_t S = ctx->p.n_samples, NR = ctx->p.n_replicas, NT = ctx->p.n_temps;
  const Layout& l = ctx->lay;
  hipStream_t s = static_cast<hipStream_t>(stream);
  struct Item {
    void* dst;
    size_t off, bytes;
  } items[] = {{clone_at, l.clone_at, 4 * S * NR * NT}, {er_head, l.er_head, 4 * S * NR},
               {pt_last, l.pt_last, S * NR * (NT - 1)},  {pt_count, l.pt_count, 4 * S * NR * (NT - 1)},
               {pt_energy, l.pt_energy, 8 * S * ctx->d.NPT}, {rt_state, l.rt_state, S * ctx->d.NPT},
               {rt_count, l.rt_count, 8 * S}};
  for (const Item& it : items) {
    if (!it.dst) continue;
    hipError_t e = hipMemcpyAsync(it.dst, ctx->d_state + it.off, it.bytes, hipMemcpyDeviceToHost, s);
    if (e != hipSuccess) return ctx->hip_fail(e, "read PT state");
  }
  hipError_t e = hipStreamSynchronize(s);
  return e == hipSuccess ? PTHR_OK : ctx->hip_fail(e, "read PT state");
}

int pthr_read_walkers(pthr_ctx* ctx, double* walker, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (int rc = ctx->need_ready()) return rc;
  if (!walker) return ctx->fail(PTHR_EINVAL, "walker must not be NULL");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(walker, ctx->d_state + ctx->lay.walker, 8 * size_t(ctx->p.n_samples) * ctx->d.NPT,
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? PTHR_OK : ctx->hip_fail(e, "read walkers");
}

int pthr_counters(const pthr_ctx* ctx, int64_t* t, int32_t* m_pt, int32_t* m_er) {
  if (!ctx) return PTHR_EINVAL;
  if (t) *t = ctx->t;
  if (m_pt) *m_pt = ctx->m_pt;
  if (m_er) *m_er = ctx->m_er;
  return PTHR_OK;
}

int pthr_check(pthr_ctx* ctx, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (int rc = ctx->need_ready()) return rc;
  std::vector<uint32_t> st(ctx->p.n_samples);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(st.data(), ctx->d_state + ctx->lay.status, 4 * st.size(), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return ctx->hip_fail(e, "read status");
  for (size_t i = 0; i < st.size(); ++i)
    if (st[i]) return ctx->fail(PTHR_EDEVICE, "sample %zu: status 0x%x (union-find iteration bound hit)", i, st[i]);
  return PTHR_OK;
}

namespace {
struct BlobHeader {
  uint64_t magic;
  pthr_params p;
  int64_t t;
  int32_t m_pt, m_er;
  uint64_t state_bytes;
};
}  // namespace

namespace {
// Field by field: the struct's tail padding is not part of the parameters.
bool same_params(const pthr_params& a, const pthr_params& b) {
  return a.L == b.L && a.n_samples == b.n_samples && a.n_replicas == b.n_replicas && a.n_temps == b.n_temps &&
         a.n_reservoir == b.n_reservoir && a.sweeps_per_emcs == b.sweeps_per_emcs &&
         a.er_sweeps_per_emcs == b.er_sweeps_per_emcs && a.precision == b.precision &&
         a.houdayer_mode == b.houdayer_mode && a.local_update == b.local_update &&
         std::memcmp(&a.t_acu, &b.t_acu, sizeof a.t_acu) == 0 && a.seed == b.seed &&
         a.micsa_refresh == b.micsa_refresh;
}
}  // namespace

size_t pthr_blob_bytes(const pthr_ctx* ctx) { return ctx ? sizeof(BlobHeader) + ctx->lay.total : 0; }

int pthr_get_state(pthr_ctx* ctx, void* blob, size_t bytes, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (int rc = ctx->need_ready()) return rc;
  if (!blob || bytes < pthr_blob_bytes(ctx)) return ctx->fail(PTHR_EINVAL, "blob too small");
  BlobHeader h{};
  h.magic = kBlobMagic;
  h.p = ctx->p;
  h.t = ctx->t;
  h.m_pt = ctx->m_pt;
  h.m_er = ctx->m_er;
  h.state_bytes = ctx->lay.total;
  std::memcpy(blob, &h, sizeof h);
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(static_cast<unsigned char*>(blob) + sizeof h, ctx->d_state, ctx->lay.total,
                                hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  return e == hipSuccess ? PTHR_OK : ctx->hip_fail(e, "get state");
}

int pthr_set_state(pthr_ctx* ctx, const void* blob, size_t bytes, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (int rc = ctx->need_ready()) return rc;
  if (!blob || bytes < sizeof(BlobHeader)) return ctx->fail(PTHR_EINVAL, "blob too small");
  BlobHeader h{};
  std::memcpy(&h, blob, sizeof h);
  if (h.magic != kBlobMagic || !same_params(h.p, ctx->p) || h.state_bytes != ctx->lay.total ||
      bytes < sizeof h + h.state_bytes)
    return ctx->fail(PTHR_EINVAL, "blob does not belong to a context with these parameters");
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e = hipMemcpyAsync(ctx->d_state, static_cast<const unsigned char*>(blob) + sizeof h, h.state_bytes,
                                hipMemcpyHostToDevice, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) return ctx->hip_fail(e, "set state");
  ctx->t = h.t;
  ctx->m_pt = h.m_pt;
  ctx->m_er = h.m_er;
  ctx->e_current = false;
  return PTHR_OK;
}

int pthr_get_schedule(const pthr_ctx* ctx, pthr_schedule* out) {
  if (!ctx || !out) return PTHR_EINVAL;
  *out = ctx->sch;
  return PTHR_OK;
}

int pthr_set_schedule(pthr_ctx* ctx, const pthr_schedule* sch) {
  if (!ctx || !sch) return PTHR_EINVAL;
  ctx->err.clear();
  bool ok = false;
  for (int ch = 2; ch <= 8; ch *= 2)
    if (chunk_ok(ctx->p.precision, ctx->d.V, ch) && threads_for(ctx->d.V, ch) == sch->threads_per_sample) ok = true;
  if (!ok)
    return ctx->fail(PTHR_EINVAL,
                     "threads_per_sample must be ceil(V/chunk / 64)*64 for chunk in {2,4,8} (FP64: {2,4}) and <= 1024");
  if (sch->samples_per_launch < 0) return ctx->fail(PTHR_EINVAL, "bad samples_per_launch");
  if (sch->graph_window < 0 || sch->graph_window > 4096) return ctx->fail(PTHR_EINVAL, "graph_window must be in [0, 4096]");
  if (sch->exp_early_out < 0) return ctx->fail(PTHR_EINVAL, "exp_early_out must be >= 0");
  if (sch->exp_filter != 0 && sch->exp_filter != 1) return ctx->fail(PTHR_EINVAL, "exp_filter must be 0 or 1");
  if (sch->clone_split != 1 && sch->clone_split != 2 && sch->clone_split != 4)
    return ctx->fail(PTHR_EINVAL, "clone_split must be 1, 2 or 4");
  if (sch->threads_per_sample * sch->clone_split > 1024)
    return ctx->fail(PTHR_EINVAL, "threads_per_sample * clone_split must be <= 1024");
  if (sch->sample_split != 1 && sch->sample_split != 2 && sch->sample_split != 4)
    return ctx->fail(PTHR_EINVAL, "sample_split must be 1, 2 or 4");
  if (sch->overlap_reservoir != 0 && sch->overlap_reservoir != 1)
    return ctx->fail(PTHR_EINVAL, "overlap_reservoir must be 0 or 1");
  ctx->sch = *sch;
  return PTHR_OK;
}

}  // extern "C"

namespace {
// Times candidate schedules on a copy of the state in `d_scratch` and keeps
// the fastest.  no_alloc: the trial EMCS run as plain launches (no graph is
// instantiated) and are timed with the host clock after a stream
// synchronisation (no events are created), so that nothing is allocated.
int autotune_impl(pthr_ctx* ctx, void* d_scratch, int n_emcs, double* best_ms, void* stream, bool no_alloc) {
  hipStream_t s = static_cast<hipStream_t>(stream);
  unsigned char* real = ctx->d_state;
  const int64_t t_saved = ctx->t;
  const bool e_saved = ctx->e_current;
  const pthr_schedule saved = ctx->sch;
  pthr_schedule best = saved;
  double best_t = 1e300;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (!no_alloc && (hipEventCreate(&e0) != hipSuccess || hipEventCreate(&e1) != hipSuccess)) {
    if (e0) (void)hipEventDestroy(e0);
    return ctx->fail(PTHR_EHIP, "event creation failed");
  }
  // elapsed milliseconds of n_emcs EMCS on the scratch state
  auto timed = [&](float* ms) -> int {
    if (no_alloc) {
      if (hipStreamSynchronize(s) != hipSuccess) return ctx->fail(PTHR_EHIP, "autotune synchronisation");
      const auto a = std::chrono::steady_clock::now();
      if (int rc = pthr_run(ctx, n_emcs, nullptr, stream)) return rc;
      if (hipStreamSynchronize(s) != hipSuccess) return ctx->fail(PTHR_EHIP, "autotune synchronisation");
      *ms = std::chrono::duration<float, std::milli>(std::chrono::steady_clock::now() - a).count();
      return PTHR_OK;
    }
    if (hipEventRecord(e0, s) != hipSuccess) return ctx->fail(PTHR_EHIP, "autotune event");
    if (int rc = pthr_run(ctx, n_emcs, nullptr, stream)) return rc;
    if (hipEventRecord(e1, s) != hipSuccess || hipEventSynchronize(e1) != hipSuccess ||
        hipEventElapsedTime(ms, e0, e1) != hipSuccess)
      return ctx->fail(PTHR_EHIP, "autotune timing");
    return PTHR_OK;
  };
  int n_cu = 256, dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n_cu, hipDeviceAttributeMultiprocessorCount, dev) !=
                                               hipSuccess)
    n_cu = 256;
  // Candidates: work-items per sample (chunk size) x waves per chunk
  // (clone_split) x workgroups per sample (sample_split, tried for batches of
  // fewer than two samples per compute unit), and the exp early-out below
  // T = 0.7 on the plain shapes.
  std::vector<pthr_schedule> cands;
  for (int ch = 2; ch <= 8; ch *= 2) {
    if (!chunk_ok(ctx->p.precision, ctx->d.V, ch)) continue;
    if (ch > 2 && threads_for(ctx->d.V, ch) == threads_for(ctx->d.V, ch / 2)) continue;
    for (int split = 1; split <= 4; split *= 2)
      for (int parts = 1; parts <= 4; parts *= 2)
        for (int early = 0; early <= 700; early += 700) {
          if (threads_for(ctx->d.V, ch) * split > 1024) continue;
          if (parts > 1 && int64_t(ctx->p.n_samples) >= 2 * int64_t(n_cu)) continue;
          if (early && (split > 1 || parts > 1)) continue;
          pthr_schedule cand = saved;
          cand.threads_per_sample = threads_for(ctx->d.V, ch);
          cand.exp_early_out = early;
          cand.clone_split = split;
          cand.sample_split = parts;
          cand.overlap_reservoir = 0;
          cands.push_back(cand);
        }
  }
  ctx->tune.clear();
  int rc = PTHR_OK;
  // then the fastest of them with the reservoir sweeps beside the Houdayer
  // step, for schedules that run plain launches (a second stream: not in the
  // allocation-free form)
  const bool try_overlap =
      !no_alloc && saved.graph_window == 0 && ctx->d.NER > 0 && ctx->p.er_sweeps_per_emcs > 0;
  const size_t n_base = cands.size();
  for (size_t ci = 0; ci <= n_base; ++ci) {
    if (rc != PTHR_OK) break;
    if (ci == n_base && !try_overlap) break;
    pthr_schedule cand = ci < n_base ? cands[ci] : best;
    if (ci == n_base) {
      cand.overlap_reservoir = 1;
      ctx->sch = cand;
      if ((rc = ctx->make_side()) != PTHR_OK) break;
    }
    if (no_alloc) cand.graph_window = 0;
    ctx->sch = cand;
    hipError_t e = hipMemcpyAsync(d_scratch, real, ctx->lay.total, hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) {
      rc = ctx->hip_fail(e, "autotune copy");
      break;
    }
    ctx->d_state = static_cast<unsigned char*>(d_scratch);
    ctx->t = t_saved;
    float ms = 0.f;
    // one untimed EMCS first (caches, clocks), then two timed stretches of
    // n_emcs EMCS; the faster one counts (a single stretch varies with the
    // clocks and with work on other streams)
    rc = pthr_run(ctx, 1, nullptr, stream);
    for (int rep = 0; rep < 2 && rc == PTHR_OK; ++rep) {
      float rep_ms = 0.f;
      rc = timed(&rep_ms);
      if (rc == PTHR_OK && (rep == 0 || rep_ms < ms)) ms = rep_ms;
    }
    if (rc == PTHR_OK) {
      cand.graph_window = saved.graph_window;
      ctx->tune.push_back({cand, static_cast<double>(ms) / n_emcs});
      if (ms < best_t) {
        best_t = ms;
        best = cand;
      }
    }
    ctx->d_state = real;
  }
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  ctx->d_state = real;
  ctx->t = t_saved;
  ctx->e_current = e_saved;
  ctx->sch = rc == PTHR_OK ? best : saved;
  if (best_ms) *best_ms = best_t / n_emcs;
  return rc;
}
}  // namespace

extern "C" {

int pthr_autotune(pthr_ctx* ctx, void* d_scratch, int n_emcs, double* best_ms, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (int rc = ctx->need_ready()) return rc;
  if (!d_scratch || n_emcs < 1) return ctx->fail(PTHR_EINVAL, "need a scratch buffer and n_emcs >= 1");
  if (ctx->m_pt || ctx->m_er) return ctx->fail(PTHR_ESTATE, "an EMCS is in progress");
  return autotune_impl(ctx, d_scratch, n_emcs, best_ms, stream, false);
}

int pthr_autotune_results(const pthr_ctx* ctx, pthr_schedule* schedules, double* ms_per_emcs, int capacity) {
  if (!ctx) return PTHR_EINVAL;
  const int n = static_cast<int>(ctx->tune.size());
  for (int i = 0; i < n && i < capacity; ++i) {
    if (schedules) schedules[i] = ctx->tune[i].first;
    if (ms_per_emcs) ms_per_emcs[i] = ctx->tune[i].second;
  }
  return n;
}

int pthr_autotune_noalloc(pthr_ctx* ctx, int n_emcs, double* best_ms, void* stream) {
  if (!ctx) return PTHR_EINVAL;
  ctx->err.clear();
  if (int rc = ctx->need_ready()) return rc;
  if (n_emcs < 1) return ctx->fail(PTHR_EINVAL, "n_emcs must be >= 1");
  if (ctx->m_pt || ctx->m_er) return ctx->fail(PTHR_ESTATE, "an EMCS is in progress");
  if (ctx->lay.total > pthr::kScratchBytes)
    return ctx->fail(PTHR_EINVAL, "state buffer of %zu bytes exceeds the %zu-byte static workspace (use pthr_autotune)",
                     ctx->lay.total, pthr::kScratchBytes);
  if (int rc = ctx->prepare()) return rc;  // the workspace address of the current device
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return ctx->fail(PTHR_EHIP, "get device");
  void* ws = device_scratch()[dev];
  return autotune_impl(ctx, ws, n_emcs, best_ms, stream, true);
}

}  // extern "C"

// ------------------------------------------------------------------ groups
// Contexts advanced together: each context's EMCS chain runs on a side stream
// of its own, forked from and joined back into the caller's stream, so the
// chains of different lattices share the GPU.  Windows of EMCS are captured
// once into a single graph with one parallel branch per context.
// Hardware queues HIP gives a process (GPU_MAX_HW_QUEUES, 4 by default).
static int hw_queues() {
  const char* v = std::getenv("GPU_MAX_HW_QUEUES");
  const int n = v ? std::atoi(v) : 0;
  return n >= 1 && n <= 32 ? n : 4;
}

struct pthr_group {
  std::vector<pthr_ctx*> ctx;
  std::vector<int> lane;          // stream of each context
  std::vector<hipStream_t> side;  // one per lane
  std::vector<hipEvent_t> join;
  hipEvent_t fork = nullptr;
  hipStream_t cap_stream = nullptr;
  hipGraphExec_t gexec = nullptr;
  int g_window = 0;
  std::vector<void*> g_obs;
  std::vector<unsigned char*> g_state;
  std::vector<pthr_schedule> g_sch;
  std::string err;

  ~pthr_group() {
    drop_graph();
    for (hipStream_t st : side)
      if (st) (void)hipStreamDestroy(st);
    for (hipEvent_t ev : join)
      if (ev) (void)hipEventDestroy(ev);
    if (fork) (void)hipEventDestroy(fork);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
  }
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    gexec = nullptr;
    g_window = 0;
  }
  int fail(int code, const char* fmt, ...) {
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    err = buf;
    return code;
  }
  // n EMCS of every context, the contexts of a lane one after the other on
  // its stream, forked from `from` and joined back into it.
  int chains(int n, void* const* d_obs, hipStream_t from) {
    hipError_t e = hipEventRecord(fork, from);
    if (e != hipSuccess) return fail(PTHR_EHIP, "fork: %s", hipGetErrorString(e));
    for (size_t s = 0; s < side.size(); ++s) {
      if ((e = hipStreamWaitEvent(side[s], fork, 0)) != hipSuccess)
        return fail(PTHR_EHIP, "fork wait: %s", hipGetErrorString(e));
      for (size_t i = 0; i < ctx.size(); ++i) {
        if (lane[i] != static_cast<int>(s)) continue;
        for (int w = 0; w < n; ++w)
          if (int rc = ctx[i]->emcs(d_obs ? d_obs[i] : nullptr, side[s], true))
            return fail(rc, "context %zu: %s", i, ctx[i]->err.c_str());
      }
      if ((e = hipEventRecord(join[s], side[s])) != hipSuccess ||
          (e = hipStreamWaitEvent(from, join[s], 0)) != hipSuccess)
        return fail(PTHR_EHIP, "join: %s", hipGetErrorString(e));
    }
    return PTHR_OK;
  }
  bool graph_current(int window, void* const* d_obs) const {
    if (!gexec || g_window != window) return false;
    for (size_t i = 0; i < ctx.size(); ++i)
      if (g_obs[i] != (d_obs ? d_obs[i] : nullptr) || g_state[i] != ctx[i]->d_state ||
          std::memcmp(&g_sch[i], &ctx[i]->sch, sizeof(pthr_schedule)) != 0)
        return false;
    return true;
  }
  int graph(int window, void* const* d_obs) {
    if (graph_current(window, d_obs)) return PTHR_OK;
    drop_graph();
    hipError_t e = hipSuccess;
    if (!cap_stream) e = hipStreamCreateWithFlags(&cap_stream, hipStreamNonBlocking);
    if (e != hipSuccess) return fail(PTHR_EHIP, "capture stream: %s", hipGetErrorString(e));
    if ((e = hipStreamBeginCapture(cap_stream, hipStreamCaptureModeThreadLocal)) != hipSuccess)
      return fail(PTHR_EHIP, "begin capture: %s", hipGetErrorString(e));
    const int rc = chains(window, d_obs, cap_stream);
    hipGraph_t gr = nullptr;
    e = hipStreamEndCapture(cap_stream, &gr);
    if (rc != PTHR_OK) {
      if (gr) (void)hipGraphDestroy(gr);
      return rc;
    }
    if (e != hipSuccess) return fail(PTHR_EHIP, "end capture: %s", hipGetErrorString(e));
    e = hipGraphInstantiate(&gexec, gr, nullptr, nullptr, 0);
    (void)hipGraphDestroy(gr);
    if (e != hipSuccess) {
      gexec = nullptr;
      return fail(PTHR_EHIP, "graph instantiation: %s", hipGetErrorString(e));
    }
    g_window = window;
    g_obs.assign(ctx.size(), nullptr);
    g_state.resize(ctx.size());
    g_sch.resize(ctx.size());
    for (size_t i = 0; i < ctx.size(); ++i) {
      g_obs[i] = d_obs ? d_obs[i] : nullptr;
      g_state[i] = ctx[i]->d_state;
      g_sch[i] = ctx[i]->sch;
    }
    return PTHR_OK;
  }
};

extern "C" {

int pthr_group_create(pthr_ctx* const* ctxs, int n_ctx, pthr_group** out) {
  if (!out) {
    g_create_error = "out must not be NULL";
    return PTHR_EINVAL;
  }
  *out = nullptr;
  if (!ctxs || n_ctx < 1 || n_ctx > kMaxGroup) {
    g_create_error = "need 1 to 64 contexts";
    return PTHR_EINVAL;
  }
  for (int i = 0; i < n_ctx; ++i) {
    if (!ctxs[i]) {
      g_create_error = "context pointers must not be NULL";
      return PTHR_EINVAL;
    }
    for (int j = 0; j < i; ++j)
      if (ctxs[j] == ctxs[i]) {
        g_create_error = "a context appears twice";
        return PTHR_EINVAL;
      }
  }
  pthr_group* grp = new pthr_group();
  grp->ctx.assign(ctxs, ctxs + n_ctx);
  // lanes: at most one stream per hardware queue; contexts by decreasing
  // load, each to the lane with the smallest load so far
  const int n_lanes = std::min(n_ctx, hw_queues());
  std::vector<double> load(n_lanes, 0.0), work(n_ctx);
  std::vector<int> order(n_ctx);
  for (int i = 0; i < n_ctx; ++i) {
    const pthr_params& p = ctxs[i]->p;
    const double V = static_cast<double>(p.L) * p.L * p.L;
    work[i] = p.n_samples * V *
              (double(p.n_replicas) * p.n_temps * p.sweeps_per_emcs +
               double(p.n_replicas) * p.n_reservoir * p.er_sweeps_per_emcs);
    order[i] = i;
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  grp->lane.assign(n_ctx, 0);
  for (int i : order) {
    const int s = static_cast<int>(std::min_element(load.begin(), load.end()) - load.begin());
    grp->lane[i] = s;
    load[s] += work[i];
  }
  grp->side.assign(n_lanes, nullptr);
  grp->join.assign(n_lanes, nullptr);
  hipError_t e = hipEventCreateWithFlags(&grp->fork, hipEventDisableTiming);
  for (int s = 0; s < n_lanes && e == hipSuccess; ++s) {
    e = hipStreamCreateWithFlags(&grp->side[s], hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreateWithFlags(&grp->join[s], hipEventDisableTiming);
  }
  if (e != hipSuccess) {
    g_create_error = std::string("stream or event creation: ") + hipGetErrorString(e);
    delete grp;
    return PTHR_EHIP;
  }
  g_create_error.clear();
  *out = grp;
  return PTHR_OK;
}

int pthr_group_destroy(pthr_group* grp) {
  delete grp;
  return PTHR_OK;
}

const char* pthr_group_last_error(const pthr_group* grp) { return grp ? grp->err.c_str() : "null group"; }

int pthr_group_run(pthr_group* grp, int64_t n_emcs, void* const* d_obs, int graph_window, void* stream) {
  if (!grp) return PTHR_EINVAL;
  grp->err.clear();
  if (n_emcs < 0) return grp->fail(PTHR_EINVAL, "n_emcs must be >= 0");
  if (graph_window < 0 || graph_window > 4096) return grp->fail(PTHR_EINVAL, "graph_window must be in [0, 4096]");
  for (size_t i = 0; i < grp->ctx.size(); ++i) {
    pthr_ctx* c = grp->ctx[i];
    c->err.clear();
    if (!c->ready) return grp->fail(PTHR_ESTATE, "context %zu: state buffer not initialised", i);
    if (c->m_pt || c->m_er) return grp->fail(PTHR_ESTATE, "context %zu: an EMCS is in progress", i);
    if (c->t + n_emcs > 0xFFFFFFFFll) return grp->fail(PTHR_ESTATE, "context %zu: EMCS counter would pass 2^32", i);
    if (c->overlapping())
      return grp->fail(PTHR_EUNSUPPORTED, "context %zu: overlap_reservoir is not supported in groups", i);
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int64_t done = 0;
  if (graph_window > 0 && n_emcs >= graph_window) {
    if (int rc = grp->graph(graph_window, d_obs)) return rc;
    for (; done + graph_window <= n_emcs; done += graph_window) {
      hipError_t e = hipGraphLaunch(grp->gexec, s);
      if (e != hipSuccess) return grp->fail(PTHR_EHIP, "graph launch: %s", hipGetErrorString(e));
      for (pthr_ctx* c : grp->ctx) {
        c->t += graph_window;
        c->e_current = true;
      }
    }
  }
  // the remainder as plain launches, in chunks that fit chains()' int count
  while (done < n_emcs) {
    const int rest = static_cast<int>(std::min<int64_t>(n_emcs - done, int64_t(1) << 30));
    if (int rc = grp->chains(rest, d_obs, s)) return rc;
    for (pthr_ctx* c : grp->ctx) {
      c->t += rest;
      c->e_current = true;
    }
    done += rest;
  }
  return PTHR_OK;
}

}  // extern "C"
