// C ABI of the CPRA hot path: plan, workspace layout, kernel dispatch.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <numeric>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/cpra.h"
#include "host_geom.hpp"
#include "impl.hpp"

using namespace cpra;

static_assert(sizeof(cpra::Coupling) == sizeof(cpra_host::Coupling), "coupling record layout");
static_assert(sizeof(cpra::Tap) == sizeof(cpra_host::Tap), "tap record layout");

using namespace cpra_impl;

namespace {

constexpr int kErrSlots = 64;       // iterations per error-history chunk
constexpr int kStageAngles = 8;     // host-pointer submits are staged this many angles at a time
constexpr size_t kAlign = 256;

size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Fixed device-resident scratch of cpra_refine_volume_noalloc (every GPU the library runs on holds
// its own copy until the process ends).  Host code never uses the array's name as an address: its
// device address is looked up once per device at plan creation (scratch_init) and kept in
// g_scratch.  Every call on one GPU shares the array.
constexpr size_t kScratchBytes = 40ull << 20;
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
char* g_scratch[kMaxDevices] = {};

// row-pass mode of a real-space update rule (episode estimates use mode 2)
int mode_of(int32_t algo) { return algo == CPRA_HIO ? 1 : algo == CPRA_RAAR ? 4 : 2; }

thread_local std::string g_create_error;
// cpra_iterate_batch shares launches between plans of one size class when N <= this
// (cpra_set_batch_fusion; 0: never, the default: on uneven batches the plans' own launches
// interleaved over their streams measured faster than shared launches)
int g_fuse_max_n = 0;

// autotuned choices per shape (N, Np, real type, amplitude type, guesses), applied to new plans
struct TuneKey {
  int N, Np, real, amp, R;
  bool operator==(const TuneKey& o) const {
    return N == o.N && Np == o.Np && real == o.real && amp == o.amp && R == o.R;
  }
};
std::mutex g_tune_mu;
std::vector<std::pair<TuneKey, cpra_tuning>> g_tune;


bool size_supported(int N) {
  return N == 64 || N == 128 || N == 192 || N == 256 || N == 384 || N == 512 || N == 1024;
}

int col_tiles(int N) {
  switch (N) {
    case 64: return ColGeom<64>::TILES;
    case 128: return ColGeom<128>::TILES;
    case 192: return ColGeom<192>::TILES;
    case 256: return ColGeom<256>::TILES;
    case 384: return ColGeom<384>::TILES;
    case 512: return ColGeom<512>::TILES;
    default: return ColGeom<1024>::TILES;
  }
}

// z-planes per step-D chunk: divides N and is a multiple of the gather's planes per thread
int stepd_chunk(int N) { return N >= 384 ? 32 : N; }

size_t mask_words_per_row(int N) {
  switch (N) {
    case 64: return RowGeom<64>::T * RowGeom<64>::MW;
    case 128: return RowGeom<128>::T * RowGeom<128>::MW;
    case 192: return RowGeom<192>::T * RowGeom<192>::MW;
    case 256: return RowGeom<256>::T * RowGeom<256>::MW;
    case 384: return RowGeom<384>::T * RowGeom<384>::MW;
    case 512: return RowGeom<512>::T * RowGeom<512>::MW;
    default: return RowGeom<1024>::T * RowGeom<1024>::MW;
  }
}

int tau_count(int N) {
  switch (N) {
    case 64: return RowGeom<64>::T;
    case 128: return RowGeom<128>::T;
    case 192: return RowGeom<192>::T;
    case 256: return RowGeom<256>::T;
    case 384: return RowGeom<384>::T;
    case 512: return RowGeom<512>::T;
    default: return RowGeom<1024>::T;
  }
}

int bit_to_t(int N, int tau, int b) {
  switch (N) {
    case 64: return mask_bit_t<64>(tau, b);
    case 128: return mask_bit_t<128>(tau, b);
    case 192: return mask_bit_t<192>(tau, b);
    case 256: return mask_bit_t<256>(tau, b);
    case 384: return mask_bit_t<384>(tau, b);
    case 512: return mask_bit_t<512>(tau, b);
    default: return mask_bit_t<1024>(tau, b);
  }
}

cpra_status validate(const cpra_params* p, std::string& msg) {
  if (!p) { msg = "params is NULL"; return CPRA_ERR_ARG; }
  if (p->struct_size != sizeof(cpra_params)) { msg = "params.struct_size mismatch"; return CPRA_ERR_ARG; }
  if (!size_supported(p->N)) { msg = "N must be 64, 128, 192, 256, 384, 512 or 1024"; return CPRA_ERR_UNSUPPORTED; }
  if (p->Np < 1) { msg = "Np must be >= 1"; return CPRA_ERR_ARG; }
  if (p->n_taps != 0) {
    if (p->n_taps < 3 || p->n_taps % 2 == 0 || !p->taps) { msg = "n_taps must be 0 or an odd number >= 3 with taps set"; return CPRA_ERR_ARG; }
    if (p->n_taps > p->Np) { msg = "2K+1 taps need Np >= 2K+1"; return CPRA_ERR_ARG; }
    double ts = 0.0;
    for (int i = 0; i < p->n_taps; ++i) {
      if (!(p->taps[i] >= 0.0) || !std::isfinite(p->taps[i])) { msg = "taps must be finite and >= 0"; return CPRA_ERR_ARG; }
      ts += p->taps[i];
    }
    if (std::fabs(ts - 1.0) > 1e-12) { msg = "taps must sum to 1"; return CPRA_ERR_ARG; }
    if (!(p->taps[p->n_taps / 2] > 0.0)) { msg = "the centre tap must be > 0"; return CPRA_ERR_ARG; }
  }
  if (p->insertion != CPRA_INSERT_NEAREST && p->insertion != CPRA_INSERT_BILINEAR) {
    msg = "bad insertion"; return CPRA_ERR_ARG;
  }
  if (p->n_guess < 0 || (int64_t)p->Np * std::max(1, p->n_guess) > (1 << 24)) {
    msg = "n_guess must be >= 0 (0 = one) with n_guess * Np <= 2^24"; return CPRA_ERR_ARG;
  }
  if (p->n_ei < 1) { msg = "n_ei must be >= 1"; return CPRA_ERR_ARG; }
  if (p->wrap != CPRA_WRAP_MIRROR && p->wrap != CPRA_WRAP_PLAIN) { msg = "bad wrap"; return CPRA_ERR_ARG; }
  if (p->real_type != CPRA_REAL_F32 && p->real_type != CPRA_REAL_F64) { msg = "bad real_type"; return CPRA_ERR_ARG; }
  if (p->amp_type != CPRA_AMP_F32 && p->amp_type != CPRA_AMP_F16) { msg = "bad amp_type"; return CPRA_ERR_ARG; }
  if (p->amp_type == CPRA_AMP_F16 && p->real_type != CPRA_REAL_F32) {
    msg = "FP16 amplitudes need an F32 plan"; return CPRA_ERR_UNSUPPORTED;
  }
  double s = 0;
  for (int i = 0; i < 3; ++i) {
    if (!(p->alpha[i] >= 0.0) || !std::isfinite(p->alpha[i])) { msg = "alpha must be finite and >= 0"; return CPRA_ERR_ARG; }
    s += p->alpha[i];
  }
  if (std::fabs(s - 1.0) > 1e-12) { msg = "alpha must sum to 1"; return CPRA_ERR_ARG; }
  if (p->alpha[1] <= 0.0) { msg = "alpha_0 must be > 0"; return CPRA_ERR_ARG; }
  if (p->theta) {
    for (int i = 0; i < p->Np; ++i)
      if (!std::isfinite(p->theta[i])) { msg = "theta must be finite"; return CPRA_ERR_ARG; }
  }
  return CPRA_OK;
}

Layout layout_of(const cpra_params* p) {
  const size_t N = p->N, Np = p->Np, H = N / 2;
  const size_t S = Np * (size_t)std::max(1, p->n_guess);   // slots: guess r, angle n at r * Np + n
  const size_t rs = p->real_type == CPRA_REAL_F64 ? 8 : 4;
  const size_t cs = 2 * rs;
  const size_t aps = p->real_type == CPRA_REAL_F64 ? 16 : (p->amp_type == CPRA_AMP_F16 ? 4 : 8);
  Layout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
  L.P = take(S * N * H * cs);
  L.Pmid = take(S * N * H * cs);
  L.g0 = take(S * N * N * rs);
  L.g1 = take(S * N * N * rs);
  L.A2 = take(Np * N * H * aps);
  L.ampscale = take(Np * rs);
  L.maskw = take(Np * N * mask_words_per_row(p->N) * 4);
  L.den = take(Np * 8);
  L.tw = take((3 * N + 3 * H) * cs);   // twiddle tables (kernels.hpp, TwLayout)
  L.coup = take(S * sizeof(cpra::Coupling));
  L.alist = take(S * 4);
  L.iota = take(S * 4);                                            // 0 .. S-1
  L.errpart = take((size_t)kErrSlots * S * col_tiles(p->N) * 8);
  L.errhist = take((size_t)kErrSlots * S * 8);
  L.flags = take(256);
  L.stage_I = take((size_t)kStageAngles * N * N * 4);
  L.stage_S = take((size_t)kStageAngles * N * N);
  L.csr_ptr = take((N * N + 1) * 4);
  L.csr_cell = take(N * N * sizeof(cpra::CellRec));
  const size_t ents = Np * N * (p->insertion == CPRA_INSERT_BILINEAR ? 4 : 1);   // at most
  L.csr_heavy = take((ents / (cpra::kStepdHeavy + 1) + 1) * sizeof(cpra::CellRec));
  L.csr_ent = take(ents * 4);
  L.csr_w = take(p->insertion == CPRA_INSERT_BILINEAR ? ents * rs : 0);
  L.cnt_inv = take(N * N * rs);
  L.zc = stepd_chunk(p->N);
  L.plane = take((size_t)L.zc * N * N * cs);
  L.stage_T = take((size_t)L.zc * Np * H * cs);   // step D: a chunk's rows of every angle, plane-major
  L.prep_part = take(Np * cpra::kPrepBlocks * 12);
  L.mtab = take(S * 3 * 8 + S * 4 * 4 + (S / Np) * 64 + 256);   // step C tables
  L.swk = take((N + 1) * rs);                                      // shrinkwrap window taps
  L.ctab = take(p->n_taps > 3 ? S * p->n_taps * sizeof(cpra::Tap) : 0);   // Eq. 4, 2K+1 taps
  L.Pc = take(p->n_taps > 3 ? S * N * H * cs : 0);                         // their coupled spectra
  L.total = o;
  return L;
}

}  // namespace

static __device__ __align__(256) char scratch[kScratchBytes];

namespace {

// Look up this device's address of `scratch` (the current device must be the plan's); once per
// device.  Returns the HIP error of the lookup.
hipError_t scratch_init(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[dev]) return hipSuccess;
  void* ptr = nullptr;
  const hipError_t e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e == hipSuccess) g_scratch[dev] = reinterpret_cast<char*>(ptr);
  return e;
}

char* scratch_of(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  return g_scratch[dev];
}

}  // namespace

namespace {

cpra_status fail(cpra_plan_t pl, cpra_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  if (pl) {
    pl->err = buf;
    if (st == CPRA_ERR_DEVICE) pl->poisoned = true;
  } else {
    g_create_error = buf;
  }
  return st;
}

#define HIPCHK(pl, expr)                                                                   \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(pl, CPRA_ERR_DEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

#define LAUNCHCHK(pl)                                                                      \
  do {                                                                                     \
    hipError_t e_ = hipGetLastError();                                                     \
    if (e_ != hipSuccess) return fail(pl, CPRA_ERR_DEVICE, "kernel launch: %s", hipGetErrorString(e_)); \
  } while (0)


Ops ops_of(const cpra_params& p) {
  switch (p.N) {
    case 64: return ops_for_size<64>(p);
    case 128: return ops_for_size<128>(p);
    case 192: return ops_for_size<192>(p);
    case 256: return ops_for_size<256>(p);
    case 384: return ops_for_size<384>(p);
    case 512: return ops_for_size<512>(p);
    default: return ops_for_size<1024>(p);
  }
}

cpra_status upload_tables(cpra_plan_t pl) {
  const int Np = pl->p.Np, R = pl->R;
  // one ring per guess: the table of the Np angles, offset to each guess's slots
  std::vector<cpra_host::Coupling> one;
  cpra_host::coupling_table(Np, pl->present.data(), pl->p.alpha, pl->p.wrap == CPRA_WRAP_MIRROR, one);
  // an absent neighbour has weight 0; point it at the angle itself so that no unset plane is read
  for (int n = 0; n < Np; ++n) {
    if (one[n].wl == 0.0) { one[n].left = n; one[n].mirror_left = 0; }
    if (one[n].wr == 0.0) { one[n].right = n; one[n].mirror_right = 0; }
  }
  pl->coup_h.resize((size_t)R * Np);
  pl->alist_h.clear();
  for (int r = 0; r < R; ++r)
    for (int n = 0; n < Np; ++n) {
      cpra_host::Coupling c = one[n];
      c.left += r * Np;
      c.right += r * Np;
      pl->coup_h[(size_t)r * Np + n] = c;
      if (pl->present[n]) pl->alist_h.push_back(r * Np + n);
    }
  // the device tables are copied from the plan's pinned staging buffer, without synchronising the
  // stream: the copies are ordered behind the launches that read the previous tables, and the
  // staging slot is rewritten only after its previous upload, kTabSlots uploads back, has completed
  const int slot = pl->tab_next;
  pl->tab_next = (slot + 1) % cpra_plan_s::kTabSlots;
  if (pl->tab_pending[slot]) {
    HIPCHK(pl, hipEventSynchronize(pl->ev_tab[slot]));
    pl->tab_pending[slot] = false;
  }
  char* hb = reinterpret_cast<char*>(pl->h_tab) + (size_t)slot * pl->tab_bytes;
  std::memcpy(hb, pl->coup_h.data(), pl->coup_h.size() * sizeof(cpra::Coupling));
  HIPCHK(pl, hipMemcpyAsync(pl->ws + pl->L.coup, hb, pl->coup_h.size() * sizeof(cpra::Coupling),
                            hipMemcpyHostToDevice, pl->stream));
  hb += align_up(pl->coup_h.size() * sizeof(cpra::Coupling));
  if (pl->K > 1) {   // Eq. 4 with 2K+1 taps: one table per guess ring
    std::vector<cpra_host::Tap> t1;
    cpra_host::tap_table(Np, pl->present.data(), pl->taps.data(), pl->K, pl->p.wrap == CPRA_WRAP_MIRROR, t1);
    const int nt = 2 * pl->K + 1;
    pl->tap_h.resize((size_t)R * Np * nt);
    for (int r = 0; r < R; ++r)
      for (size_t i = 0; i < (size_t)Np * nt; ++i) {
        cpra_host::Tap t = t1[i];
        t.nb += r * Np;
        pl->tap_h[(size_t)r * Np * nt + i] = t;
      }
    std::memcpy(hb, pl->tap_h.data(), pl->tap_h.size() * sizeof(cpra::Tap));
    HIPCHK(pl, hipMemcpyAsync(pl->ws + pl->L.ctab, hb, pl->tap_h.size() * sizeof(cpra::Tap), hipMemcpyHostToDevice,
                              pl->stream));
    hb += align_up(pl->tap_h.size() * sizeof(cpra::Tap));
  }
  if (!pl->alist_h.empty()) {
    std::memcpy(hb, pl->alist_h.data(), pl->alist_h.size() * 4);
    HIPCHK(pl, hipMemcpyAsync(pl->ws + pl->L.alist, hb, pl->alist_h.size() * 4, hipMemcpyHostToDevice, pl->stream));
  }
  HIPCHK(pl, hipEventRecord(pl->ev_tab[slot], pl->stream));
  pl->tab_pending[slot] = true;
  pl->tables_dirty = false;
  pl->table_version += 1;
  return CPRA_OK;
}

}  // namespace

namespace cpra_impl {
namespace {
std::mutex g_pin_mu;
std::multimap<size_t, void*> g_pin_free;   // size class -> idle pinned buffer
size_t pin_class(size_t bytes) {
  size_t c = size_t(4) << 10;
  while (c < bytes) c <<= 1;
  return c;
}
}  // namespace

void* pinned_take(size_t bytes) {
  const size_t c = pin_class(bytes);
  {
    std::lock_guard<std::mutex> lk(g_pin_mu);
    auto it = g_pin_free.find(c);
    if (it != g_pin_free.end()) {
      void* p = it->second;
      g_pin_free.erase(it);
      return p;
    }
  }
  void* p = nullptr;
  return hipHostMalloc(&p, c, hipHostMallocDefault) == hipSuccess ? p : nullptr;
}

void pinned_give(void* p, size_t bytes) {
  if (!p) return;
  std::lock_guard<std::mutex> lk(g_pin_mu);
  g_pin_free.emplace(pin_class(bytes), p);
}
}  // namespace cpra_impl

extern "C" {

cpra_status cpra_workspace_size(const cpra_params* params, size_t* bytes) {
  std::string msg;
  cpra_status st = validate(params, msg);
  if (st != CPRA_OK) return fail(nullptr, st, "%s", msg.c_str());
  if (!bytes) return fail(nullptr, CPRA_ERR_ARG, "bytes is NULL");
  *bytes = layout_of(params).total;
  return CPRA_OK;
}

cpra_status cpra_plan(const cpra_params* params, void* workspace, size_t workspace_bytes, void* hip_stream,
                      cpra_plan_t* out) {
  std::string msg;
  cpra_status st = validate(params, msg);
  if (st != CPRA_OK) return fail(nullptr, st, "%s", msg.c_str());
  if (!out) return fail(nullptr, CPRA_ERR_ARG, "out is NULL");
  if (!workspace || (reinterpret_cast<uintptr_t>(workspace) % kAlign) != 0)
    return fail(nullptr, CPRA_ERR_ARG, "workspace must be non-NULL and 256-byte aligned");
  Layout L = layout_of(params);
  if (workspace_bytes < L.total)
    return fail(nullptr, CPRA_ERR_OOM, "workspace has %zu bytes, plan needs %zu", workspace_bytes, L.total);
  cpra_plan_t pl = new (std::nothrow) cpra_plan_s();
  if (!pl) return fail(nullptr, CPRA_ERR_OOM, "host allocation failed");
  pl->p = *params;
  pl->R = std::max(1, params->n_guess);
  pl->p.n_guess = pl->R;
  if (params->n_taps == 3) {               // three taps: the fused coupling with alpha
    for (int i = 0; i < 3; ++i) pl->p.alpha[i] = params->taps[i];
  } else if (params->n_taps > 3) {
    pl->taps.assign(params->taps, params->taps + params->n_taps);
    pl->K = params->n_taps / 2;
  }
  pl->p.taps = nullptr;
  pl->theta.resize(params->Np);
  for (int n = 0; n < params->Np; ++n)
    pl->theta[n] = params->theta ? params->theta[n] : cpra_host::default_theta(n, params->Np);
  pl->p.theta = nullptr;
  pl->L = L;
  pl->ws = reinterpret_cast<char*>(workspace);
  pl->stream = reinterpret_cast<hipStream_t>(hip_stream);
  pl->pid = (int)getpid();
  pl->landed.assign(params->Np, 0);
  pl->present.assign(params->Np, 0);
  pl->ntiles = col_tiles(params->N);
  hipError_t e = hipGetDevice(&pl->device);
  if (e == hipSuccess) e = scratch_init(pl->device);
  if (e != hipSuccess) {
    g_create_error = std::string("plan setup (device scratch): ") + hipGetErrorString(e);
    delete pl;
    return CPRA_ERR_DEVICE;
  }
  // pinned staging of the tables (coupling records, taps, slot list) and of the data-check flag
  const size_t S = (size_t)params->Np * pl->R;
  const size_t tab_bytes = align_up(S * sizeof(cpra::Coupling)) +
                           align_up(pl->K > 1 ? S * (2 * pl->K + 1) * sizeof(cpra::Tap) : 0) + S * 4;
  pl->tab_bytes = align_up(tab_bytes);
  pl->h_tab = pinned_take(pl->tab_bytes * cpra_plan_s::kTabSlots);
  pl->h_flag = static_cast<int32_t*>(pinned_take(256));
  if (!pl->h_tab || !pl->h_flag) e = hipErrorOutOfMemory;
  for (int i = 0; i < cpra_plan_s::kTabSlots && e == hipSuccess; ++i)
    e = hipEventCreateWithFlags(&pl->ev_tab[i], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&pl->ev_flag, hipEventDisableTiming);
  std::vector<int32_t> iota(S);
  std::iota(iota.begin(), iota.end(), 0);
  if (e == hipSuccess) e = hipMemcpyAsync(pl->ws + L.iota, iota.data(), S * 4, hipMemcpyHostToDevice, pl->stream);
  Ops ops = ops_of(pl->p);
  if (e == hipSuccess) {
    ops.twiddles(pl);
    e = hipGetLastError();
  }
  if (e == hipSuccess) e = hipMemsetAsync(pl->ws + L.flags, 0, 256, pl->stream);
  // angles not submitted yet read back as zero objects
  if (e == hipSuccess) e = hipMemsetAsync(pl->ws + L.g0, 0, L.A2 - L.g0, pl->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(pl->stream);
  if (e != hipSuccess) {
    g_create_error = std::string("plan setup: ") + hipGetErrorString(e);
    delete pl;
    return CPRA_ERR_DEVICE;
  }
  {
    // a shape tuned in this process starts with the tuned choices
    const TuneKey key{params->N, params->Np, params->real_type, params->amp_type, pl->R};
    std::lock_guard<std::mutex> lk(g_tune_mu);
    for (const auto& kv : g_tune)
      if (kv.first == key) {
        pl->row_alt = kv.second.row_tile != 0;
        pl->chunk = kv.second.chunk;
        pl->use_graphs = kv.second.graphs != 0;
      }
  }
  *out = pl;
  return CPRA_OK;
}

cpra_status cpra_plan_create(const cpra_params* params, void* workspace, size_t workspace_bytes, void* hip_stream,
                             cpra_plan_t* out) {
  return cpra_plan(params, workspace, workspace_bytes, hip_stream, out);
}

// Step-D tables: the integer cell map of the Fourier-slice insertion (built on the host in FP64),
// the bilinear weights, and the inverse count (or weight sum) per cell, packed into one pinned
// image: row pointers, cell records, entries, weights, inverse counts, heavy-cell records, each
// 256-byte aligned.  The image depends only on N, Np, the angles, the insertion and the precision,
// so a process keeps the images of up to kStepdImages shapes and later plans of a shape upload the same image (scans of a
// serving mix repeat a few shapes).  Built at the first step-D call rather than at plan creation,
// so that this host work overlaps the iterations already queued on the stream; the uploads come
// from pinned memory, so they are ordered on the stream before step D's kernels without the host
// waiting for the iterations ahead of them.
namespace {
struct StepdImage {
  int N = 0, Np = 0;
  bool bil = false, f64 = false;
  std::vector<double> theta;
  void* host = nullptr;        // pinned
  size_t bytes = 0;
  size_t piece[6] = {};        // bytes of each piece, in image order
  int n_heavy = 0;
};
constexpr size_t kStepdImages = 16;
std::mutex g_img_mu;
std::vector<std::shared_ptr<const StepdImage>> g_img;

std::shared_ptr<StepdImage> build_stepd_image(const cpra_params& p, const std::vector<double>& theta) {
  auto img = std::make_shared<StepdImage>();
  img->N = p.N;
  img->Np = p.Np;
  img->bil = p.insertion == CPRA_INSERT_BILINEAR;
  img->f64 = p.real_type == CPRA_REAL_F64;
  img->theta = theta;
  std::vector<int32_t> rp, ent;
  std::vector<double> wts;
  if (img->bil) cpra_host::insertion_csr_bilinear(p.N, p.Np, theta.data(), rp, ent, wts);
  else cpra_host::insertion_csr(p.N, p.Np, theta.data(), rp, ent);
  const size_t NN = (size_t)p.N * p.N;
  std::vector<float> wf(wts.begin(), wts.end());
  std::vector<double> inv_d(NN);
  std::vector<float> inv_f(NN);
  for (size_t c = 0; c < NN; ++c) {
    double tot = 0.0;   // entry count, or the sum of the bilinear weights (in entry order)
    for (int i = rp[c]; i < rp[c + 1]; ++i) tot += img->bil ? wts[i] : 1.0;
    inv_d[c] = tot > 0.0 ? 1.0 / tot : 0.0;
    inv_f[c] = (float)inv_d[c];
  }
  // the cell records of step D's gather: first entry, entry range, inverse count as FP32 bits; cells
  // with more than kStepdHeavy entries go to the heavy list (record: first = the cell index) and are
  // marked first = -2 in the gather's table
  std::vector<cpra::CellRec> cell(NN), heavy;
  for (size_t c = 0; c < NN; ++c) {
    cpra::CellRec& r = cell[c];
    r.begin = rp[c];
    r.end = rp[c + 1];
    r.first = rp[c] < rp[c + 1] ? ent[rp[c]] : -1;
    std::memcpy(&r.inv_bits, &inv_f[c], 4);
    if (r.end - r.begin > cpra::kStepdHeavy) {
      heavy.push_back(cpra::CellRec{(int)c, r.begin, r.end, r.inv_bits});
      r.first = -2;
    }
  }
  img->n_heavy = (int)heavy.size();
  const void* src[6] = {rp.data(), cell.data(), ent.data(),
                        img->f64 ? (const void*)wts.data() : (const void*)wf.data(),
                        img->f64 ? (const void*)inv_d.data() : (const void*)inv_f.data(), heavy.data()};
  img->piece[0] = rp.size() * 4;
  img->piece[1] = NN * sizeof(cpra::CellRec);
  img->piece[2] = ent.size() * 4;
  img->piece[3] = img->bil ? wts.size() * (img->f64 ? 8 : 4) : 0;
  img->piece[4] = NN * (img->f64 ? 8 : 4);
  img->piece[5] = heavy.size() * sizeof(cpra::CellRec);
  for (size_t b : img->piece) img->bytes += align_up(b);
  img->host = pinned_take(img->bytes);
  if (!img->host) return nullptr;
  char* hb = static_cast<char*>(img->host);
  for (int i = 0; i < 6; ++i) {
    if (img->piece[i]) std::memcpy(hb, src[i], img->piece[i]);
    hb += align_up(img->piece[i]);
  }
  return img;
}
}  // namespace

static cpra_status ensure_stepd_tables(cpra_plan_t pl) {
  if (pl->stepd_ready) return CPRA_OK;
  const cpra_params& p = pl->p;
  const bool bil = p.insertion == CPRA_INSERT_BILINEAR;
  const bool f64 = p.real_type == CPRA_REAL_F64;
  std::shared_ptr<const StepdImage> img;
  {
    std::lock_guard<std::mutex> lk(g_img_mu);
    for (const auto& m : g_img)
      if (m->N == p.N && m->Np == p.Np && m->bil == bil && m->f64 == f64 && m->theta == pl->theta) img = m;
  }
  if (!img) {
    std::shared_ptr<StepdImage> built = build_stepd_image(p, pl->theta);
    if (!built) return fail(pl, CPRA_ERR_DEVICE, "step D: pinned staging of the insertion tables failed");
    std::lock_guard<std::mutex> lk(g_img_mu);
    if (g_img.size() < kStepdImages) {
      g_img.push_back(built);          // kept for the process's lifetime
    } else {
      pl->h_stepd = built->host;       // not cached: the plan returns the buffer when it is destroyed
      pl->stepd_bytes = built->bytes;
    }
    img = built;
  }
  const Layout& L = pl->L;
  if (img->piece[5] > L.csr_ent - L.csr_heavy)   // cannot happen: each heavy cell holds > kStepdHeavy entries
    return fail(pl, CPRA_ERR_DEVICE, "step D: %d heavy cells exceed their table", img->n_heavy);
  const size_t dst[6] = {L.csr_ptr, L.csr_cell, L.csr_ent, L.csr_w, L.cnt_inv, L.csr_heavy};
  HIPCHK(pl, hipEventCreateWithFlags(&pl->ev_stepd, hipEventDisableTiming));
  const char* hb = static_cast<const char*>(img->host);
  for (int i = 0; i < 6; ++i) {
    if (img->piece[i])
      HIPCHK(pl, hipMemcpyAsync(pl->ws + dst[i], hb, img->piece[i], hipMemcpyHostToDevice, pl->stream));
    hb += align_up(img->piece[i]);
  }
  pl->n_heavy = img->n_heavy;
  HIPCHK(pl, hipEventRecord(pl->ev_stepd, pl->stream));
  pl->stepd_ready = true;
  return CPRA_OK;
}

// An asynchronous submit's data check: once its flag copy has landed, a NaN or Inf poisons the plan.
static cpra_status check_data(cpra_plan_t pl) {
  if (!pl->flag_pending) return CPRA_OK;
  const hipError_t q = hipEventQuery(pl->ev_flag);
  if (q == hipErrorNotReady) return CPRA_OK;
  if (q != hipSuccess) return fail(pl, CPRA_ERR_DEVICE, "data check: %s", hipGetErrorString(q));
  pl->flag_pending = false;
  if (*pl->h_flag & 1) {
    pl->poisoned = true;
    return fail(pl, CPRA_ERR_DATA, "the intensity of an asynchronously submitted angle contains NaN or Inf");
  }
  return CPRA_OK;
}

cpra_status cpra_submit_angles(cpra_plan_t pl, int32_t first, int32_t count, const float* intensity,
                               const uint8_t* support, int32_t ptr_kind) {
  if (!pl) return fail(nullptr, CPRA_ERR_ARG, "plan is NULL");
  if (pl->poisoned) return fail(pl, CPRA_ERR_STATE, "plan is poisoned by an earlier device error");
  if (count < 1 || first < 0 || first + count > pl->p.Np)
    return fail(pl, CPRA_ERR_ARG, "angles [%d, %d) outside [0, %d)", first, first + count, pl->p.Np);
  if (!intensity || !support) return fail(pl, CPRA_ERR_ARG, "intensity/support is NULL");
  if (ptr_kind != CPRA_PTR_HOST && ptr_kind != CPRA_PTR_DEVICE && ptr_kind != CPRA_PTR_DEVICE_ASYNC)
    return fail(pl, CPRA_ERR_ARG, "bad ptr_kind");
  for (int i = 0; i < count; ++i)
    if (pl->landed[first + i]) return fail(pl, CPRA_ERR_STATE, "angle %d was already submitted", first + i);
  {
    const cpra_status st = check_data(pl);
    if (st != CPRA_OK) return st;
  }
  const int N = pl->p.N;
  const size_t NN = (size_t)N * N;
  const bool async = ptr_kind == CPRA_PTR_DEVICE_ASYNC;
  Ops ops = ops_of(pl->p);
  // the synchronous forms report this call's data check; the asynchronous form keeps the flag,
  // which then covers every asynchronous submit since the last synchronous one
  if (!async) HIPCHK(pl, hipMemsetAsync(pl->ws + pl->L.flags, 0, 4, pl->stream));
  // slots to initialise: every guess's copy of each submitted angle, grouped per staging chunk
  const int R = pl->R, Np = pl->p.Np;
  // host inputs are staged through the workspace a few angles at a time;
  // device inputs go out in one launch of each kernel
  const int chunk = ptr_kind == CPRA_PTR_HOST ? kStageAngles : count;
  bool used_alist = false;
  for (int c0 = 0; c0 < count; c0 += chunk) {
    const int cn = std::min(chunk, count - c0);
    const float* dI;
    const uint8_t* dS;
    if (ptr_kind == CPRA_PTR_HOST) {
      HIPCHK(pl, hipMemcpyAsync(pl->ws + pl->L.stage_I, intensity + c0 * NN, cn * NN * 4, hipMemcpyHostToDevice, pl->stream));
      HIPCHK(pl, hipMemcpyAsync(pl->ws + pl->L.stage_S, support + c0 * NN, cn * NN, hipMemcpyHostToDevice, pl->stream));
      dI = at<float>(pl, pl->L.stage_I);
      dS = at<uint8_t>(pl, pl->L.stage_S);
    } else {
      dI = intensity + c0 * NN;
      dS = support + c0 * NN;
    }
    ops.prep(pl, dI, dS, first + c0, cn);
    LAUNCHCHK(pl);
    // initial objects of every guess go into the buffer that holds the current iterate; with one
    // guess the slots are consecutive and listed by the plan's fixed identity list
    if (R == 1) {
      ops.init(pl, at<int>(pl, pl->L.iota) + first + c0, cn, pl->cur);
      LAUNCHCHK(pl);
      if (ptr_kind == CPRA_PTR_HOST) HIPCHK(pl, hipStreamSynchronize(pl->stream));   // the staging buffers
    } else {
      std::vector<int32_t> ids;
      for (int r = 0; r < R; ++r)
        for (int i = 0; i < cn; ++i) ids.push_back(r * Np + first + c0 + i);
      HIPCHK(pl, hipMemcpyAsync(pl->ws + pl->L.alist, ids.data(), ids.size() * 4, hipMemcpyHostToDevice, pl->stream));
      ops.init(pl, at<int>(pl, pl->L.alist), (int)ids.size(), pl->cur);
      LAUNCHCHK(pl);
      HIPCHK(pl, hipStreamSynchronize(pl->stream));   // ids is rebuilt for the next chunk
      used_alist = true;
    }
  }
  if (async) {
    // the flag travels to pinned host memory behind this submit's work; check_data reads it
    HIPCHK(pl, hipMemcpyAsync(pl->h_flag, pl->ws + pl->L.flags, 4, hipMemcpyDeviceToHost, pl->stream));
    HIPCHK(pl, hipEventRecord(pl->ev_flag, pl->stream));
    pl->flag_pending = true;
  } else {
    int flag = 0;
    HIPCHK(pl, hipMemcpyAsync(&flag, pl->ws + pl->L.flags, 4, hipMemcpyDeviceToHost, pl->stream));
    HIPCHK(pl, hipStreamSynchronize(pl->stream));
    if (used_alist) pl->tables_dirty = true;   // alist was used as scratch
    if (flag & 1) {
      HIPCHK(pl, hipMemsetAsync(pl->ws + pl->L.flags, 0, 4, pl->stream));
      return fail(pl, CPRA_ERR_DATA, "intensity contains NaN or Inf");
    }
  }
  for (int i = 0; i < count; ++i) pl->landed[first + i] = 1;
  if (pl->k % pl->p.n_ei == 0 && pl->present != pl->landed) {
    pl->present = pl->landed;
    pl->tables_dirty = true;
  }
  return CPRA_OK;
}

// one iteration of the listed slots; a boundary couples (Eq. 4) on the way in: fused into the
// passes for three taps, or as a pass of its own into the Pc planes for 2K+1 > 3 taps (so the
// column pass reads them and writes Pmid, two distinct planes)
static void do_step(cpra_plan_t pl, const Ops& ops, const int* al, int nact, bool boundary, bool inplace,
                    int mode, double beta, double* ep) {
  if (boundary && pl->K > 1) {
    const int gout = inplace ? pl->cur : (pl->cur ^ 1);
    ops.couple_taps(pl, al, nact, pl->cur, gout);
    ops.step(pl, al, nact, false, false, mode, beta, ep, pl->ws + pl->L.Pc, gout);
  } else {
    ops.step(pl, al, nact, boundary, inplace, mode, beta, ep, nullptr, -1);
  }
}

// episode bookkeeping before an iteration: the angle set changes only at a boundary
static cpra_status refresh_tables(cpra_plan_t pl) {
  if ((pl->k % pl->p.n_ei) == 0 && pl->present != pl->landed) {
    pl->present = pl->landed;
    pl->tables_dirty = true;
  }
  return pl->tables_dirty ? upload_tables(pl) : CPRA_OK;
}

// m iterations after an episode's boundary, the first of them at position j0 (>= 1) of the
// episode.  Between boundaries the slots do not interact, so the order is chunk-major: each
// chunk of pl->chunk listed slots runs all m iterations before the next chunk starts, which keeps
// a chunk's planes in the last-level cache from one pass to the next.  Same arithmetic as m
// iterations over all slots.
static void run_inner(cpra_plan_t pl, const Ops& ops, int32_t algo, double beta, int j0, int m) {
  const int nact = (int)pl->alist_h.size();
  const int ch = pl->chunk > 0 && pl->chunk < nact ? pl->chunk : nact;
  const int* al = at<int>(pl, pl->L.alist);
  for (int c0 = 0; c0 < nact; c0 += ch) {
    const int cn = nact - c0 < ch ? nact - c0 : ch;
    for (int i = 0; i < m; ++i) {
      const int mode = (j0 + i + 1) % pl->p.n_ei == 0 ? 2 : mode_of(algo);
      do_step(pl, ops, al + c0, cn, false, false, mode, beta, nullptr);
    }
  }
}

// the rest of the current episode, at most n iterations, from a position j0 >= 1
static cpra_status episode_rest(cpra_plan_t pl, const Ops& ops, int32_t algo, double beta, int32_t& n) {
  cpra_status st = refresh_tables(pl);
  if (st != CPRA_OK) return st;
  const int j0 = (int)(pl->k % pl->p.n_ei);
  const int m = pl->p.n_ei - j0 < n ? pl->p.n_ei - j0 : n;
  run_inner(pl, ops, algo, beta, j0, m);
  LAUNCHCHK(pl);
  pl->k += m;
  n -= m;
  return CPRA_OK;
}

// one iteration of one plan with no error history: episode bookkeeping, then the two passes
static cpra_status step_once(cpra_plan_t pl, const Ops& ops, int32_t algo, double beta) {
  const bool boundary = (pl->k % pl->p.n_ei) == 0;
  cpra_status st = refresh_tables(pl);
  if (st != CPRA_OK) return st;
  const int nact = (int)pl->alist_h.size();
  const bool estimate = ((pl->k + 1) % pl->p.n_ei) == 0;
  const int mode = estimate ? 2 : mode_of(algo);
  do_step(pl, ops, at<int>(pl, pl->L.alist), nact, boundary, false, mode, beta, nullptr);
  LAUNCHCHK(pl);
  if (boundary) pl->cur ^= 1;
  pl->k += 1;
  return CPRA_OK;
}

// Capture one episode (n_ei iterations from a boundary, starting with buffer `parity` current)
// into pl->gexec[parity].  Kernels only: no copies or fills are recorded.  The capture runs on a
// private stream; the graph is launched on the plan's stream.
static cpra_status capture_episode(cpra_plan_t pl, const Ops& ops, int32_t algo, double beta, int parity) {
  if (!pl->cap_stream) HIPCHK(pl, hipStreamCreateWithFlags(&pl->cap_stream, hipStreamNonBlocking));
  const hipStream_t keep_stream = pl->stream;
  const bool keep_timing = pl->timing;
  const int keep_cur = pl->cur;
  pl->stream = pl->cap_stream;
  pl->timing = false;
  pl->cur = parity;
  hipError_t e = hipStreamBeginCapture(pl->cap_stream, hipStreamCaptureModeThreadLocal);
  hipGraph_t g = nullptr;
  if (e == hipSuccess) {
    const int nact = (int)pl->alist_h.size();
    do_step(pl, ops, at<int>(pl, pl->L.alist), nact, true, false, pl->p.n_ei == 1 ? 2 : mode_of(algo), beta,
            nullptr);
    pl->cur ^= 1;
    if (pl->p.n_ei > 1) run_inner(pl, ops, algo, beta, 1, pl->p.n_ei - 1);
    e = hipStreamEndCapture(pl->cap_stream, &g);
  }
  pl->stream = keep_stream;
  pl->timing = keep_timing;
  pl->cur = keep_cur;
  if (e != hipSuccess) return fail(pl, CPRA_ERR_DEVICE, "episode capture: %s", hipGetErrorString(e));
  e = hipGraphInstantiate(&pl->gexec[parity], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return fail(pl, CPRA_ERR_DEVICE, "graph instantiate: %s", hipGetErrorString(e));
  return CPRA_OK;
}

// One whole episode from a boundary (k mod n_ei == 0) through the captured graph of the current
// parity; same arithmetic as n_ei calls of step_once.
static cpra_status graph_episode(cpra_plan_t pl, const Ops& ops, int32_t algo, double beta) {
  cpra_status st0 = refresh_tables(pl);
  if (st0 != CPRA_OK) return st0;
  if (pl->g_algo != algo || pl->g_beta != beta || pl->g_version != pl->table_version) {
    pl->drop_graphs();
    pl->g_algo = algo;
    pl->g_beta = beta;
    pl->g_version = pl->table_version;
  }
  if (!pl->gexec[pl->cur]) {
    cpra_status st = capture_episode(pl, ops, algo, beta, pl->cur);
    if (st != CPRA_OK) return st;
  }
  HIPCHK(pl, hipGraphLaunch(pl->gexec[pl->cur], pl->stream));
  pl->cur ^= 1;
  pl->k += pl->p.n_ei;
  return CPRA_OK;
}

// advance one plan without error history by a boundary iteration, by the rest of an episode, or
// by a whole episode through its graph, taking at most n iterations
static cpra_status advance(cpra_plan_t pl, const Ops& ops, int32_t algo, double beta, int32_t& n) {
  if (pl->k % pl->p.n_ei != 0) return episode_rest(pl, ops, algo, beta, n);
  if (pl->use_graphs && n >= pl->p.n_ei) {
    n -= pl->p.n_ei;
    return graph_episode(pl, ops, algo, beta);
  }
  n -= 1;
  return step_once(pl, ops, algo, beta);
}

cpra_status cpra_set_tuning(cpra_plan_t pl, const cpra_tuning* t) {
  if (!pl) return fail(nullptr, CPRA_ERR_ARG, "plan is NULL");
  if (!t) return fail(pl, CPRA_ERR_ARG, "tuning is NULL");
  if (t->row_tile != 0 && t->row_tile != 1) return fail(pl, CPRA_ERR_ARG, "row_tile must be 0 or 1");
  if (t->chunk < 0) return fail(pl, CPRA_ERR_ARG, "chunk must be >= 0");
  pl->row_alt = t->row_tile != 0;
  pl->chunk = t->chunk;
  pl->use_graphs = t->graphs != 0;
  pl->drop_graphs();   // captured episodes hold the previous launch shapes
  return CPRA_OK;
}

constexpr double kTuneMargin = 0.02;

cpra_status cpra_autotune(const cpra_params* params, void* workspace, size_t workspace_bytes, void* hip_stream,
                          int32_t n_iter, cpra_tuning* best) {
  if (!best) return fail(nullptr, CPRA_ERR_ARG, "best is NULL");
  if (n_iter < 1) return fail(nullptr, CPRA_ERR_ARG, "n_iter must be >= 1");
  cpra_plan_t pl = nullptr;
  cpra_status st = cpra_plan(params, workspace, workspace_bytes, hip_stream, &pl);
  if (st != CPRA_OK) return st;
  struct Guard {
    cpra_plan_t p;
    ~Guard() { delete p; }
  } guard{pl};
  pl->row_alt = false;
  pl->chunk = 0;
  pl->use_graphs = false;
  // a synthetic scan, staged through the plan's own buffers a few angles at a time
  const int Np = pl->p.Np;
  Ops ops = ops_of(pl->p);
  for (int c0 = 0; c0 < Np; c0 += kStageAngles) {
    const int cn = std::min(kStageAngles, Np - c0);
    ops.synth(pl, c0, cn, 0x5eedULL);
    LAUNCHCHK(pl);
    st = cpra_submit_angles(pl, c0, cn, at<float>(pl, pl->L.stage_I), at<uint8_t>(pl, pl->L.stage_S),
                            CPRA_PTR_DEVICE);
    if (st != CPRA_OK) return st;
  }
  // whole episodes, so that every candidate (graphs included) runs the same iterations
  const int ne = pl->p.n_ei;
  const int iters = (n_iter + ne - 1) / ne * ne;
  st = cpra_iterate(pl, ne, CPRA_HIO, 0.9, nullptr);
  if (st != CPRA_OK) return st;
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(pl, hipEventCreate(&e0));
  HIPCHK(pl, hipEventCreate(&e1));
  struct EvGuard {
    hipEvent_t a, b;
    ~EvGuard() {
      (void)hipEventDestroy(a);
      (void)hipEventDestroy(b);
    }
  } evg{e0, e1};
  const int S = (int)((size_t)Np * pl->R);
  std::vector<int> chunks = {0};
  for (int d : {2, 4})
    if (S / d >= 16) chunks.push_back((S + d - 1) / d);
  cpra_tuning top{}, dflt{};
  top.ms_per_iteration = -1.0;
  for (int rt = 0; rt < 2; ++rt)
    for (int ch : chunks)
      for (int gr = 0; gr < 2; ++gr) {
        const cpra_tuning cand{rt, ch, gr, 0.0};
        st = cpra_set_tuning(pl, &cand);
        if (st != CPRA_OK) return st;
        st = cpra_iterate(pl, ne, CPRA_HIO, 0.9, nullptr);   // warm (and capture a graph)
        if (st != CPRA_OK) return st;
        HIPCHK(pl, hipEventRecord(e0, pl->stream));
        st = cpra_iterate(pl, iters, CPRA_HIO, 0.9, nullptr);
        if (st != CPRA_OK) return st;
        HIPCHK(pl, hipEventRecord(e1, pl->stream));
        HIPCHK(pl, hipEventSynchronize(e1));
        float ms = 0.f;
        HIPCHK(pl, hipEventElapsedTime(&ms, e0, e1));
        const double per = (double)ms / iters;
        if (rt == 0 && ch == 0 && gr == 0) {
          dflt = cand;
          dflt.ms_per_iteration = per;
        }
        if (top.ms_per_iteration < 0.0 || per < top.ms_per_iteration) {
          top = cand;
          top.ms_per_iteration = per;
        }
      }
  // a choice within kTuneMargin of the default's time is noise: keep the default
  if (top.ms_per_iteration > dflt.ms_per_iteration * (1.0 - kTuneMargin)) top = dflt;
  *best = top;
  const TuneKey key{params->N, params->Np, params->real_type, params->amp_type, pl->R};
  std::lock_guard<std::mutex> lk(g_tune_mu);
  for (auto& kv : g_tune)
    if (kv.first == key) {
      kv.second = top;
      return CPRA_OK;
    }
  g_tune.push_back({key, top});
  return CPRA_OK;
}

// Several plans of one size and precision advanced together, one launch per pass per iteration
// (per kFuseMax plans and per kind of iteration: boundary or not, estimate or not), on the stream
// of the first plan.  That stream is ordered after every plan's stream first, the plans' own work
// (table uploads) goes to it meanwhile, and every plan's stream is ordered after it at the end.
static cpra_status fused_batch(std::vector<cpra_plan_t>& pls, const Ops& ops, int32_t n_iter, int32_t algo,
                               double beta) {
  const hipStream_t bs = pls[0]->stream;
  std::vector<hipStream_t> own(pls.size());
  for (size_t i = 0; i < pls.size(); ++i) {
    cpra_plan_t pl = pls[i];
    own[i] = pl->stream;
    if (pl->stream != bs) {
      if (!pl->ev_batch) HIPCHK(pl, hipEventCreateWithFlags(&pl->ev_batch, hipEventDisableTiming));
      HIPCHK(pl, hipEventRecord(pl->ev_batch, pl->stream));
      HIPCHK(pl, hipStreamWaitEvent(bs, pl->ev_batch, 0));
    }
    pl->stream = bs;
  }
  cpra_status st = CPRA_OK;
  std::vector<cpra_plan_t> grp;
  for (int32_t it = 0; it < n_iter && st == CPRA_OK; ++it) {
    for (cpra_plan_t pl : pls) {
      st = refresh_tables(pl);
      if (st != CPRA_OK) break;
    }
    if (st != CPRA_OK) break;
    // the kinds of iteration present: (boundary, mode); usually one
    for (int kind = 0; kind < 4; ++kind) {
      grp.clear();
      for (cpra_plan_t pl : pls) {
        const bool boundary = (pl->k % pl->p.n_ei) == 0;
        const bool estimate = ((pl->k + 1) % pl->p.n_ei) == 0;
        if ((boundary ? 1 : 0) + (estimate ? 2 : 0) == kind) grp.push_back(pl);
      }
      if (grp.empty()) continue;
      ops.fused_step(grp.data(), (int)grp.size(), (kind & 1) != 0, (kind & 2) ? 2 : mode_of(algo), beta, bs);
      const hipError_t e = hipGetLastError();
      if (e != hipSuccess) {
        st = fail(grp[0], CPRA_ERR_DEVICE, "fused launch: %s", hipGetErrorString(e));
        break;
      }
    }
    for (cpra_plan_t pl : pls) {
      if (pl->k % pl->p.n_ei == 0) pl->cur ^= 1;
      pl->k += 1;
    }
  }
  for (size_t i = 0; i < pls.size(); ++i) {
    cpra_plan_t pl = pls[i];
    pl->stream = own[i];
    if (own[i] != bs) {
      if (hipEventRecord(pl->ev_batch, bs) != hipSuccess || hipStreamWaitEvent(own[i], pl->ev_batch, 0) != hipSuccess)
        st = fail(pl, CPRA_ERR_DEVICE, "batch stream ordering");
    }
  }
  return st;
}

cpra_status cpra_set_batch_fusion(int32_t max_n) {
  if (max_n < 0) return fail(nullptr, CPRA_ERR_ARG, "max_n must be >= 0");
  g_fuse_max_n = max_n;
  return CPRA_OK;
}

cpra_status cpra_get_batch_fusion(int32_t* max_n) {
  if (!max_n) return fail(nullptr, CPRA_ERR_ARG, "max_n is NULL");
  *max_n = g_fuse_max_n;
  return CPRA_OK;
}

cpra_status cpra_iterate_batch(cpra_plan_t* plans, int32_t count, int32_t n_iter, int32_t algo, double beta) {
  if (!plans) return fail(nullptr, CPRA_ERR_ARG, "plans is NULL");
  if (count < 0) return fail(nullptr, CPRA_ERR_ARG, "count < 0");
  for (int i = 0; i < count; ++i) {
    cpra_plan_t pl = plans[i];
    if (!pl) return fail(nullptr, CPRA_ERR_ARG, "plans[%d] is NULL", i);
    for (int j = 0; j < i; ++j)
      if (plans[j] == pl) return fail(pl, CPRA_ERR_ARG, "plan %d repeated at %d", j, i);
    if (pl->poisoned) return fail(pl, CPRA_ERR_STATE, "plan is poisoned by an earlier device error");
    if (n_iter < 0) return fail(pl, CPRA_ERR_ARG, "n_iter < 0");
    if (algo != CPRA_HIO && algo != CPRA_ER && algo != CPRA_RAAR) return fail(pl, CPRA_ERR_ARG, "bad algo");
    if (!std::isfinite(beta)) return fail(pl, CPRA_ERR_ARG, "beta must be finite");
    bool any = false;
    for (int n = 0; n < pl->p.Np; ++n) any = any || pl->landed[n];
    if (!any) return fail(pl, CPRA_ERR_STATE, "no angle has been submitted");
    const cpra_status st = check_data(pl);
    if (st != CPRA_OK) return st;
  }
  cpra_status worst = CPRA_OK;
  if (n_iter == 0) return worst;
  // size classes (N, real type, amplitude type) of two or more plans with three-tap coupling and
  // launch-by-launch episodes go through fused launches; every other plan advances on its own
  std::vector<std::vector<cpra_plan_t>> classes;
  std::vector<cpra_plan_t> single;
  for (int i = 0; i < count; ++i) {
    cpra_plan_t pl = plans[i];
    if (pl->p.N > g_fuse_max_n || pl->K > 1 || pl->use_graphs || pl->chunk > 0) {
      single.push_back(pl);
      continue;
    }
    bool placed = false;
    for (auto& c : classes)
      if (c[0]->p.N == pl->p.N && c[0]->p.real_type == pl->p.real_type && c[0]->p.amp_type == pl->p.amp_type) {
        c.push_back(pl);
        placed = true;
        break;
      }
    if (!placed) classes.push_back({pl});
  }
  for (auto& c : classes) {
    if (c.size() == 1) {
      single.push_back(c[0]);
      continue;
    }
    const cpra_status st = fused_batch(c, ops_of(c[0]->p), n_iter, algo, beta);
    if (st != CPRA_OK) worst = st;
  }
  std::vector<Ops> ops(single.size());
  std::vector<int32_t> left(single.size(), n_iter);
  for (size_t i = 0; i < single.size(); ++i) ops[i] = ops_of(single[i]->p);
  // round robin: each round advances every plan by its boundary iteration, by the rest of its
  // episode, or by a whole episode when the plan replays captured episodes
  for (bool more = !single.empty(); more;) {
    more = false;
    for (size_t i = 0; i < single.size(); ++i) {
      if (left[i] <= 0 || single[i]->poisoned) continue;
      const cpra_status st = advance(single[i], ops[i], algo, beta, left[i]);
      if (st != CPRA_OK) worst = st;
      more = more || left[i] > 0;
    }
  }
  return worst;
}

cpra_status cpra_iterate(cpra_plan_t pl, int32_t n_iter, int32_t algo, double beta, double* err_out) {
  if (!pl) return fail(nullptr, CPRA_ERR_ARG, "plan is NULL");
  if (pl->poisoned) return fail(pl, CPRA_ERR_STATE, "plan is poisoned by an earlier device error");
  if (n_iter < 0) return fail(pl, CPRA_ERR_ARG, "n_iter < 0");
  if (algo != CPRA_HIO && algo != CPRA_ER && algo != CPRA_RAAR) return fail(pl, CPRA_ERR_ARG, "bad algo");
  if (!std::isfinite(beta)) return fail(pl, CPRA_ERR_ARG, "beta must be finite");
  {
    const cpra_status st = check_data(pl);
    if (st != CPRA_OK) return st;
  }
  const int Np = pl->p.Np;
  {
    bool any = false;
    for (int n = 0; n < Np; ++n) any = any || pl->landed[n];
    if (!any) return fail(pl, CPRA_ERR_STATE, "no angle has been submitted");
  }
  Ops ops = ops_of(pl->p);
  if (!err_out) {
    int32_t left = n_iter;
    while (left > 0) {
      const cpra_status st = advance(pl, ops, algo, beta, left);
      if (st != CPRA_OK) return st;
    }
    return CPRA_OK;
  }
  const size_t Sl = (size_t)Np * pl->R;
  if (err_out)
    for (size_t i = 0; i < (size_t)n_iter * Sl; ++i) err_out[i] = NAN;
  int slot = 0, slot_base = 0;
  // reduce the pending error slots with the angle list they were computed with
  auto flush = [&]() -> cpra_status {
    if (!err_out || slot == 0) return CPRA_OK;
    const int nact = (int)pl->alist_h.size();
    const int tot = slot * nact;
    k_err_reduce<<<(tot + 255) / 256, 256, 0, pl->stream>>>(at<double>(pl, pl->L.errpart), at<double>(pl, pl->L.den),
                                                            at<int>(pl, pl->L.alist), nact, pl->ntiles, slot,
                                                            pl->p.Np, at<double>(pl, pl->L.errhist));
    LAUNCHCHK(pl);
    pl->errhist_h.resize(tot);
    HIPCHK(pl, hipMemcpyAsync(pl->errhist_h.data(), pl->ws + pl->L.errhist, tot * 8, hipMemcpyDeviceToHost, pl->stream));
    HIPCHK(pl, hipStreamSynchronize(pl->stream));
    for (int s = 0; s < slot; ++s)
      for (int ai = 0; ai < nact; ++ai)
        err_out[(size_t)(slot_base + s) * Sl + pl->alist_h[ai]] = pl->errhist_h[(size_t)s * nact + ai];
    slot_base += slot;
    slot = 0;
    return CPRA_OK;
  };
  for (int it = 0; it < n_iter; ++it) {
    const bool boundary = (pl->k % pl->p.n_ei) == 0;
    if (boundary && pl->present != pl->landed) {
      pl->present = pl->landed;
      pl->tables_dirty = true;
    }
    if (pl->tables_dirty) {
      cpra_status st = flush();
      if (st != CPRA_OK) return st;
      st = upload_tables(pl);
      if (st != CPRA_OK) return st;
    }
    const int nact = (int)pl->alist_h.size();
    const bool estimate = ((pl->k + 1) % pl->p.n_ei) == 0;
    const int mode = estimate ? 2 : mode_of(algo);
    double* ep = err_out ? at<double>(pl, pl->L.errpart) + (size_t)slot * nact * pl->ntiles : nullptr;
    do_step(pl, ops, at<int>(pl, pl->L.alist), nact, boundary, false, mode, beta, ep);
    LAUNCHCHK(pl);
    if (boundary) pl->cur ^= 1;
    pl->k += 1;
    if (err_out) {
      ++slot;
      if (slot == kErrSlots || it == n_iter - 1) {
        cpra_status st = flush();
        if (st != CPRA_OK) return st;
      }
    }
  }
  return CPRA_OK;
}

namespace {

// slots of angle i in every guess at alist + i * R (the order of the consecutive sweep)
cpra_status upload_sweep_lists(cpra_plan_t pl) {
  const int Np = pl->p.Np, R = pl->R;
  std::vector<int32_t> v((size_t)Np * R);
  for (int i = 0; i < Np; ++i)
    for (int r = 0; r < R; ++r) v[(size_t)i * R + r] = r * Np + i;
  HIPCHK(pl, hipMemcpyAsync(pl->ws + pl->L.alist, v.data(), v.size() * 4, hipMemcpyHostToDevice, pl->stream));
  HIPCHK(pl, hipStreamSynchronize(pl->stream));
  pl->tables_dirty = true;   // cpra_iterate rebuilds its own list
  return CPRA_OK;
}

// n_it iterations of the R listed slots (one angle of every guess), in place; with `couple` the
// first iteration starts from Eq. 4 over the neighbours' current objects; the last writes the
// estimate.  err (R x n_it, row per slot) receives E_F when non-NULL.
cpra_status run_po(cpra_plan_t pl, const Ops& ops, const int* d_list, int n_it, bool couple, int algo,
                   double beta, double* err) {
  const int R = pl->R;
  double* errpart = at<double>(pl, pl->L.errpart);
  std::vector<double> hist;
  for (int it = 0; it < n_it; ++it) {
    const int mode = it == n_it - 1 ? 2 : mode_of(algo);
    double* ep = err ? errpart + (size_t)(it % kErrSlots) * R * pl->ntiles : nullptr;
    do_step(pl, ops, d_list, R, couple && it == 0, true, mode, beta, ep);
    LAUNCHCHK(pl);
    if (err && (it % kErrSlots == kErrSlots - 1 || it == n_it - 1)) {
      const int ns = it % kErrSlots + 1;
      k_err_reduce<<<(ns * R + 255) / 256, 256, 0, pl->stream>>>(errpart, at<double>(pl, pl->L.den), d_list, R,
                                                                  pl->ntiles, ns, pl->p.Np,
                                                                  at<double>(pl, pl->L.errhist));
      LAUNCHCHK(pl);
      hist.resize((size_t)ns * R);
      HIPCHK(pl, hipMemcpyAsync(hist.data(), pl->ws + pl->L.errhist, hist.size() * 8, hipMemcpyDeviceToHost,
                                pl->stream));
      HIPCHK(pl, hipStreamSynchronize(pl->stream));
      for (int q = 0; q < ns; ++q)
        for (int r = 0; r < R; ++r) err[(size_t)r * n_it + (it - ns + 1 + q)] = hist[(size_t)q * R + r];
    }
  }
  return CPRA_OK;
}

cpra_status check_algo(cpra_plan_t pl, int32_t algo, double beta) {
  if (algo != CPRA_HIO && algo != CPRA_ER && algo != CPRA_RAAR) return fail(pl, CPRA_ERR_ARG, "bad algo");
  if (!std::isfinite(beta)) return fail(pl, CPRA_ERR_ARG, "beta must be finite");
  return CPRA_OK;
}

bool all_landed(cpra_plan_t pl) {
  return std::all_of(pl->landed.begin(), pl->landed.end(), [](uint8_t v) { return v != 0; });
}

}  // namespace

cpra_status cpra_prereconstruct(cpra_plan_t pl, int32_t n_iter, int32_t algo, double beta, double* err_out) {
  if (!pl) return fail(nullptr, CPRA_ERR_ARG, "plan is NULL");
  if (pl->poisoned) return fail(pl, CPRA_ERR_STATE, "plan is poisoned by an earlier device error");
  if (n_iter < 1) return fail(pl, CPRA_ERR_ARG, "n_iter < 1");
  cpra_status st = check_algo(pl, algo, beta);
  if (st != CPRA_OK) return st;
  if (!pl->landed[0]) return fail(pl, CPRA_ERR_STATE, "angle 0 has not been submitted");
  Ops ops = ops_of(pl->p);
  st = upload_sweep_lists(pl);
  if (st != CPRA_OK) return st;
  std::vector<double> e(err_out ? (size_t)pl->R * n_iter : 0);
  st = run_po(pl, ops, at<int>(pl, pl->L.alist), n_iter, false, algo, beta, err_out ? e.data() : nullptr);
  if (st != CPRA_OK) return st;
  if (err_out) std::copy(e.begin(), e.end(), err_out);
  return CPRA_OK;
}

cpra_status cpra_sweep(cpra_plan_t pl, int32_t n_episodes, int32_t algo, double beta, double* err_out) {
  if (!pl) return fail(nullptr, CPRA_ERR_ARG, "plan is NULL");
  if (pl->poisoned) return fail(pl, CPRA_ERR_STATE, "plan is poisoned by an earlier device error");
  if (n_episodes < 0) return fail(pl, CPRA_ERR_ARG, "n_episodes < 0");
  cpra_status st = check_algo(pl, algo, beta);
  if (st != CPRA_OK) return st;
  if (!all_landed(pl)) return fail(pl, CPRA_ERR_STATE, "the consecutive sweep needs every angle submitted");
  if (pl->k % pl->p.n_ei != 0)
    return fail(pl, CPRA_ERR_STATE, "the sweep starts at an episode boundary (k=%lld)", (long long)pl->k);
  const int Np = pl->p.Np, R = pl->R, ne = pl->p.n_ei;
  Ops ops = ops_of(pl->p);
  pl->present = pl->landed;
  st = upload_tables(pl);   // the full ring of every guess
  if (st != CPRA_OK) return st;
  st = upload_sweep_lists(pl);
  if (st != CPRA_OK) return st;
  std::vector<double> e(err_out ? (size_t)R * ne : 0);
  for (int m = 0; m < n_episodes; ++m)
    for (int i = 0; i < Np; ++i) {
      st = run_po(pl, ops, at<int>(pl, pl->L.alist) + (size_t)i * R, ne, true, algo, beta,
                  err_out ? e.data() : nullptr);
      if (st != CPRA_OK) return st;
      if (err_out)
        for (int r = 0; r < R; ++r)
          for (int it = 0; it < ne; ++it)
            err_out[(((size_t)m * R + r) * Np + i) * ne + it] = e[(size_t)r * ne + it];
    }
  pl->k += (int64_t)n_episodes * ne;
  return CPRA_OK;
}

cpra_status cpra_merge(cpra_plan_t pl, int32_t n_best, int32_t* kept, int32_t* inverted) {
  if (!pl) return fail(nullptr, CPRA_ERR_ARG, "plan is NULL");
  if (pl->poisoned) return fail(pl, CPRA_ERR_STATE, "plan is poisoned by an earlier device error");
  const int Np = pl->p.Np, R = pl->R, N = pl->p.N;
  if (n_best < 1 || n_best > R) return fail(pl, CPRA_ERR_ARG, "n_best must be in [1, %d]", R);
  if (!all_landed(pl)) return fail(pl, CPRA_ERR_STATE, "the merge needs every angle submitted");
  if (pl->k % pl->p.n_ei != 0)
    return fail(pl, CPRA_ERR_STATE, "the merge needs an episode end (k=%lld)", (long long)pl->k);
  const size_t S = (size_t)R * Np;
  const int K = n_best;
  Ops ops = ops_of(pl->p);
  // device tables in the step-C region
  char* mt = pl->ws + pl->L.mtab;
  double* d_mom = reinterpret_cast<double*>(mt);
  int* d_shift = reinterpret_cast<int*>(mt + S * 3 * 8);
  int* d_list = d_shift + S * 2;
  double* d_twin = reinterpret_cast<double*>(mt + S * 3 * 8 + S * 4 * 4);
  int* d_small = reinterpret_cast<int*>(d_twin + 2 * R);   // keep (R), inverted (R), twin slots (R), twin shifts (2R)
  // 1. episode error of every guess: pooled E_F of its current objects
  std::vector<int32_t> all(S);
  std::iota(all.begin(), all.end(), 0);
  HIPCHK(pl, hipMemcpyAsync(d_list, all.data(), S * 4, hipMemcpyHostToDevice, pl->stream));
  ops.colerr(pl, d_list, (int)S, at<double>(pl, pl->L.errpart));
  LAUNCHCHK(pl);
  k_err_reduce<<<(unsigned)((S + 255) / 256), 256, 0, pl->stream>>>(at<double>(pl, pl->L.errpart),
                                                                      at<double>(pl, pl->L.den), d_list, (int)S,
                                                                      pl->ntiles, 1, Np, at<double>(pl, pl->L.errhist));
  LAUNCHCHK(pl);
  std::vector<double> e(S), den(Np);
  HIPCHK(pl, hipMemcpyAsync(e.data(), pl->ws + pl->L.errhist, S * 8, hipMemcpyDeviceToHost, pl->stream));
  HIPCHK(pl, hipMemcpyAsync(den.data(), pl->ws + pl->L.den, Np * 8, hipMemcpyDeviceToHost, pl->stream));
  HIPCHK(pl, hipStreamSynchronize(pl->stream));
  double dsum = 0.0;
  for (int n = 0; n < Np; ++n) dsum += den[n];
  std::vector<double> E(R);
  for (int r = 0; r < R; ++r) {
    double num = 0.0;
    for (int n = 0; n < Np; ++n) num += e[(size_t)r * Np + n] * e[(size_t)r * Np + n] * den[n];
    E[r] = dsum > 0.0 ? std::sqrt(num / dsum) : std::sqrt(num);
  }
  // 2. the n_best guesses of lowest error, in rank order (ties keep guess order)
  std::vector<int32_t> order(R);
  std::iota(order.begin(), order.end(), 0);
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return E[a] < E[b]; });
  std::vector<int32_t> keep(order.begin(), order.begin() + K);
  // 3. mass centres of the kept POs -> integer shifts floor(-c + 1/2)
  std::vector<int32_t> list((size_t)K * Np);
  for (int j = 0; j < K; ++j)
    for (int n = 0; n < Np; ++n) list[(size_t)j * Np + n] = keep[j] * Np + n;
  HIPCHK(pl, hipMemcpyAsync(d_list, list.data(), list.size() * 4, hipMemcpyHostToDevice, pl->stream));
  ops.moments(pl, d_list, K * Np, d_mom);
  LAUNCHCHK(pl);
  std::vector<double> mom((size_t)K * Np * 3);
  HIPCHK(pl, hipMemcpyAsync(mom.data(), d_mom, mom.size() * 8, hipMemcpyDeviceToHost, pl->stream));
  HIPCHK(pl, hipStreamSynchronize(pl->stream));
  std::vector<int32_t> shift((size_t)K * Np * 2);
  for (size_t q = 0; q < (size_t)K * Np; ++q) {
    const double m0 = mom[3 * q];
    const double cz = m0 != 0.0 ? mom[3 * q + 1] / m0 : 0.0, ct = m0 != 0.0 ? mom[3 * q + 2] / m0 : 0.0;
    shift[2 * q] = (int32_t)std::floor(-cz + 0.5);
    shift[2 * q + 1] = (int32_t)std::floor(-ct + 0.5);
  }
  // 4. twin test of every other kept guess against the best one, on PO 0
  std::vector<int32_t> inv(K, 0);
  if (K > 1) {
    std::vector<int32_t> tsl(K), tsh(2 * K);
    for (int j = 0; j < K; ++j) {
      tsl[j] = keep[j] * Np;
      tsh[2 * j] = shift[(size_t)2 * j * Np];
      tsh[2 * j + 1] = shift[(size_t)2 * j * Np + 1];
    }
    HIPCHK(pl, hipMemcpyAsync(d_small + 2 * R, tsl.data(), K * 4, hipMemcpyHostToDevice, pl->stream));
    HIPCHK(pl, hipMemcpyAsync(d_small + 3 * R, tsh.data(), 2 * K * 4, hipMemcpyHostToDevice, pl->stream));
    ops.twin(pl, d_small + 2 * R, d_small + 3 * R, K, d_twin);
    LAUNCHCHK(pl);
    std::vector<double> tw(2 * K);
    HIPCHK(pl, hipMemcpyAsync(tw.data(), d_twin, 2 * K * 8, hipMemcpyDeviceToHost, pl->stream));
    HIPCHK(pl, hipStreamSynchronize(pl->stream));
    for (int j = 1; j < K; ++j) inv[j] = tw[2 * j + 1] < tw[2 * j] ? 1 : 0;
  }
  // 5. average into guess 0's slots (through the Pmid scratch) and rebuild their row spectra
  HIPCHK(pl, hipMemcpyAsync(d_small, keep.data(), K * 4, hipMemcpyHostToDevice, pl->stream));
  HIPCHK(pl, hipMemcpyAsync(d_small + R, inv.data(), K * 4, hipMemcpyHostToDevice, pl->stream));
  HIPCHK(pl, hipMemcpyAsync(d_shift, shift.data(), shift.size() * 4, hipMemcpyHostToDevice, pl->stream));
  ops.merge_avg(pl, K, d_small, d_small + R, d_shift, pl->ws + pl->L.Pmid);
  LAUNCHCHK(pl);
  const size_t rs = pl->p.real_type == CPRA_REAL_F64 ? 8 : 4;
  HIPCHK(pl, hipMemcpyAsync(pl->ws + (pl->cur ? pl->L.g1 : pl->L.g0), pl->ws + pl->L.Pmid, (size_t)Np * N * N * rs,
                            hipMemcpyDeviceToDevice, pl->stream));
  HIPCHK(pl, hipMemcpyAsync(d_list, all.data(), (size_t)Np * 4, hipMemcpyHostToDevice, pl->stream));
  ops.reload(pl, d_list, Np, pl->cur);
  LAUNCHCHK(pl);
  HIPCHK(pl, hipStreamSynchronize(pl->stream));
  pl->tables_dirty = true;
  if (kept) std::copy(keep.begin(), keep.end(), kept);
  if (inverted) std::copy(inv.begin(), inv.end(), inverted);
  return CPRA_OK;
}

cpra_status cpra_shrinkwrap(cpra_plan_t pl, double sigma, double threshold) {
  if (!pl) return fail(nullptr, CPRA_ERR_ARG, "plan is NULL");
  if (pl->poisoned) return fail(pl, CPRA_ERR_STATE, "plan is poisoned by an earlier device error");
  const int N = pl->p.N, Np = pl->p.Np;
  if (!(sigma > 0.0) || !(4.0 * sigma <= N / 2 - 1))
    return fail(pl, CPRA_ERR_ARG, "sigma must be > 0 with ceil(4 sigma) < N/2");
  if (!(threshold > 0.0 && threshold <= 1.0)) return fail(pl, CPRA_ERR_ARG, "threshold must be in (0, 1]");
  if (pl->R != 1) return fail(pl, CPRA_ERR_UNSUPPORTED, "shrinkwrap needs a one-guess plan (supports are per angle)");
  if (pl->k % pl->p.n_ei != 0)
    return fail(pl, CPRA_ERR_STATE, "shrinkwrap needs an episode end (k=%lld)", (long long)pl->k);
  std::vector<int32_t> ids;
  for (int n = 0; n < Np; ++n)
    if (pl->present[n]) ids.push_back(n);
  if (ids.empty()) return fail(pl, CPRA_ERR_STATE, "no angle is present");
  // window taps exp(-d^2 / 2 sigma^2), d = -W..W, W = ceil(4 sigma), normalised in FP64
  const int W = (int)std::ceil(4.0 * sigma);
  std::vector<double> k(2 * W + 1);
  double ks = 0.0;
  for (int d = -W; d <= W; ++d) ks += (k[d + W] = std::exp(-(double)d * d / (2.0 * sigma * sigma)));
  for (double& v : k) v /= ks;
  std::vector<float> kf(k.begin(), k.end());
  const bool f64 = pl->p.real_type == CPRA_REAL_F64;
  HIPCHK(pl, hipMemcpyAsync(pl->ws + pl->L.swk, f64 ? (const void*)k.data() : (const void*)kf.data(),
                            k.size() * (f64 ? 8 : 4), hipMemcpyHostToDevice, pl->stream));
  HIPCHK(pl, hipMemcpyAsync(pl->ws + pl->L.alist, ids.data(), ids.size() * 4, hipMemcpyHostToDevice, pl->stream));
  Ops ops = ops_of(pl->p);
  ops.shrinkwrap(pl, at<int>(pl, pl->L.alist), (int)ids.size(), W, threshold);
  LAUNCHCHK(pl);
  HIPCHK(pl, hipStreamSynchronize(pl->stream));   // host vectors go out of scope
  pl->tables_dirty = true;                         // alist was used as scratch
  return CPRA_OK;
}

namespace {

struct RefineLayout {
  size_t qh, cb, s3, pmax, win, sc, list, total;
};

RefineLayout refine_layout(const cpra_params* p) {
  const size_t N = p->N, Np = p->Np, N3 = N * N * N;
  const size_t rs = p->real_type == CPRA_REAL_F64 ? 8 : 4;
  RefineLayout L{};
  size_t o = 0;
  auto take = [&](size_t bytes) { size_t at = o; o = align_up(o + bytes); return at; };
  L.qh = take(N3 * 2 * rs);
  L.cb = take(N3 * 2 * rs);
  L.s3 = take(N3);
  L.pmax = take((N * N / 8 + 1) * 8);
  L.win = take((N + 1) * rs);
  L.sc = take(Np * 16);
  L.list = take((Np + N) * 4);
  L.total = o;
  return L;
}

}  // namespace

cpra_status cpra_refine_workspace_size(const cpra_params* params, size_t* bytes) {
  std::string msg;
  cpra_status st = validate(params, msg);
  if (st != CPRA_OK) return fail(nullptr, st, "%s", msg.c_str());
  if (!bytes) return fail(nullptr, CPRA_ERR_ARG, "bytes is NULL");
  *bytes = refine_layout(params).total;
  return CPRA_OK;
}

// the refinement on the scratch buffer `work` of work_bytes (the caller's, or the fixed device array)
static cpra_status refine_run(cpra_plan_t pl, int32_t n_iter, int32_t shrink_every, double sigma, double threshold,
                              void* work, size_t work_bytes, void* d_volume) {
  if (!pl) return fail(nullptr, CPRA_ERR_ARG, "plan is NULL");
  if (pl->poisoned) return fail(pl, CPRA_ERR_STATE, "plan is poisoned by an earlier device error");
  if (!d_volume) return fail(pl, CPRA_ERR_ARG, "d_volume is NULL");
  if (n_iter < 0 || shrink_every < 0) return fail(pl, CPRA_ERR_ARG, "n_iter and shrink_every must be >= 0");
  const int N = pl->p.N, Np = pl->p.Np;
  if (shrink_every > 0) {
    if (!(sigma > 0.0) || !(4.0 * sigma <= N / 2 - 1))
      return fail(pl, CPRA_ERR_ARG, "sigma must be > 0 with ceil(4 sigma) < N/2");
    if (!(threshold > 0.0 && threshold <= 1.0)) return fail(pl, CPRA_ERR_ARG, "threshold must be in (0, 1]");
  }
  const RefineLayout RL = refine_layout(&pl->p);
  if (!work || (reinterpret_cast<uintptr_t>(work) % kAlign) != 0)
    return fail(pl, CPRA_ERR_ARG, "work must be non-NULL and 256-byte aligned");
  if (work_bytes < RL.total)
    return fail(pl, CPRA_ERR_OOM, "refinement workspace has %zu bytes, needs %zu", work_bytes, RL.total);
  if (pl->k == 0 || pl->k % pl->p.n_ei != 0)
    return fail(pl, CPRA_ERR_STATE, "the refinement starts from step D at an episode end (k=%lld)", (long long)pl->k);
  {
    cpra_status st = ensure_stepd_tables(pl);
    if (st != CPRA_OK) return st;
  }
  char* w = reinterpret_cast<char*>(work);
  // present data angles and their (sin, cos); then 0 .. N-1 (the planes as slots for the blur)
  std::vector<int32_t> list;
  std::vector<double> sc;
  for (int n = 0; n < Np; ++n)
    if (pl->present[n]) {
      list.push_back(n);
      sc.push_back(std::sin(pl->theta[n]));
      sc.push_back(std::cos(pl->theta[n]));
    }
  if (list.empty()) return fail(pl, CPRA_ERR_STATE, "no angle is present");
  const int count = (int)list.size();
  for (int z = 0; z < N; ++z) list.push_back(z);
  int W = 0;
  std::vector<double> k;
  if (shrink_every > 0) {
    W = (int)std::ceil(4.0 * sigma);
    k.resize(2 * W + 1);
    double ks = 0.0;
    for (int d = -W; d <= W; ++d) ks += (k[d + W] = std::exp(-(double)d * d / (2.0 * sigma * sigma)));
    for (double& v : k) v /= ks;
  }
  std::vector<float> kf(k.begin(), k.end());
  const bool f64 = pl->p.real_type == CPRA_REAL_F64;
  HIPCHK(pl, hipMemcpyAsync(w + RL.list, list.data(), list.size() * 4, hipMemcpyHostToDevice, pl->stream));
  HIPCHK(pl, hipMemcpyAsync(w + RL.sc, sc.data(), sc.size() * 8, hipMemcpyHostToDevice, pl->stream));
  if (!k.empty())
    HIPCHK(pl, hipMemcpyAsync(w + RL.win, f64 ? (const void*)k.data() : (const void*)kf.data(),
                              k.size() * (f64 ? 8 : 4), hipMemcpyHostToDevice, pl->stream));
  Ops ops = ops_of(pl->p);
  ops.assemble(pl, d_volume);   // step D: the starting volume
  LAUNCHCHK(pl);
  RefineArgs a{};
  a.vol = d_volume;
  a.qh = w + RL.qh;
  a.cb = w + RL.cb;
  a.s3 = reinterpret_cast<uint8_t*>(w + RL.s3);
  a.pmax = reinterpret_cast<double*>(w + RL.pmax);
  a.win = w + RL.win;
  a.sc = reinterpret_cast<const double*>(w + RL.sc);
  a.list = reinterpret_cast<const int*>(w + RL.list);
  a.count = count;
  a.n_iter = n_iter;
  a.shrink_every = shrink_every;
  a.W = W;
  a.threshold = threshold;
  ops.refine(pl, a);
  LAUNCHCHK(pl);
  HIPCHK(pl, hipStreamSynchronize(pl->stream));   // host tables go out of scope
  return CPRA_OK;
}

cpra_status cpra_refine_volume(cpra_plan_t pl, int32_t n_iter, int32_t shrink_every, double sigma, double threshold,
                               void* work, size_t work_bytes, void* d_volume) {
  return refine_run(pl, n_iter, shrink_every, sigma, threshold, work, work_bytes, d_volume);
}

cpra_status cpra_refine_volume_noalloc(cpra_plan_t pl, int32_t n_iter, int32_t shrink_every, double sigma,
                                       double threshold, void* d_volume) {
  if (!pl) return fail(nullptr, CPRA_ERR_ARG, "plan is NULL");
  const size_t need = refine_layout(&pl->p).total;
  if (need > kScratchBytes)
    return fail(pl, CPRA_ERR_UNSUPPORTED,
                "the fixed refinement scratch holds %zu bytes; N=%d with this real type needs %zu "
                "(use cpra_refine_volume with a caller workspace)", kScratchBytes, pl->p.N, need);
  char* w = scratch_of(pl->device);
  if (!w) return fail(pl, CPRA_ERR_STATE, "no scratch address for device %d", pl->device);
  return refine_run(pl, n_iter, shrink_every, sigma, threshold, w, kScratchBytes, d_volume);
}

cpra_status cpra_read_support(cpra_plan_t pl, uint8_t* out) {
  if (!pl) return fail(nullptr, CPRA_ERR_ARG, "plan is NULL");
  if (pl->poisoned) return fail(pl, CPRA_ERR_STATE, "plan is poisoned by an earlier device error");
  if (!out) return fail(pl, CPRA_ERR_ARG, "out is NULL");
  const int N = pl->p.N, Np = pl->p.Np;
  const size_t wpr = mask_words_per_row(N);          // words per row, in the row pass's thread order
  std::vector<uint32_t> w((size_t)Np * N * wpr);
  HIPCHK(pl, hipMemcpyAsync(w.data(), pl->ws + pl->L.maskw, w.size() * 4, hipMemcpyDeviceToHost, pl->stream));
  HIPCHK(pl, hipStreamSynchronize(pl->stream));
  const int mw = (int)(wpr / tau_count(N));
  std::fill(out, out + (size_t)Np * N * N, (uint8_t)0);
  for (int n = 0; n < Np; ++n)
    for (int z = 0; z < N; ++z)
      for (size_t r = 0; r < wpr; ++r) {
        const uint32_t word = w[((size_t)n * N + z) * wpr + r];
        const int tau = (int)r / mw, wd = (int)r % mw;
        for (int b = 0; b < 32; ++b) {
          const int t = bit_to_t(N, tau, wd * 32 + b);
          if (t >= 0 && ((word >> b) & 1u)) out[((size_t)n * N + z) * N + t] = 1;
        }
      }
  return CPRA_OK;
}

cpra_status cpra_load_objects(cpra_plan_t pl, const void* objects, int32_t ptr_kind) {
  if (!pl) return fail(nullptr, CPRA_ERR_ARG, "plan is NULL");
  if (pl->poisoned) return fail(pl, CPRA_ERR_STATE, "plan is poisoned by an earlier device error");
  if (!objects) return fail(pl, CPRA_ERR_ARG, "objects is NULL");
  if (ptr_kind != CPRA_PTR_HOST && ptr_kind != CPRA_PTR_DEVICE) return fail(pl, CPRA_ERR_ARG, "bad ptr_kind");
  const int Np = pl->p.Np;
  std::vector<int32_t> ids;
  for (int r = 0; r < pl->R; ++r)
    for (int n = 0; n < Np; ++n)
      if (pl->landed[n]) ids.push_back(r * Np + n);
  if (ids.empty()) return fail(pl, CPRA_ERR_STATE, "no angle has been submitted");
  const size_t plane = (size_t)pl->p.N * pl->p.N * (pl->p.real_type == CPRA_REAL_F64 ? 8 : 4);
  char* dst = pl->ws + (pl->cur ? pl->L.g1 : pl->L.g0);
  const hipMemcpyKind kind = ptr_kind == CPRA_PTR_HOST ? hipMemcpyHostToDevice : hipMemcpyDeviceToDevice;
  for (int32_t n : ids)
    HIPCHK(pl, hipMemcpyAsync(dst + n * plane, static_cast<const char*>(objects) + n * plane, plane, kind, pl->stream));
  HIPCHK(pl, hipMemcpyAsync(pl->ws + pl->L.alist, ids.data(), ids.size() * 4, hipMemcpyHostToDevice, pl->stream));
  Ops ops = ops_of(pl->p);
  ops.reload(pl, at<int>(pl, pl->L.alist), (int)ids.size(), pl->cur);
  LAUNCHCHK(pl);
  HIPCHK(pl, hipStreamSynchronize(pl->stream));   // ids is a host temporary; host inputs must be consumed
  pl->tables_dirty = true;                         // alist was used as scratch
  return CPRA_OK;
}

cpra_status cpra_read_objects(cpra_plan_t pl, void* out, int32_t ptr_kind) {
  if (!pl) return fail(nullptr, CPRA_ERR_ARG, "plan is NULL");
  if (pl->poisoned) return fail(pl, CPRA_ERR_STATE, "plan is poisoned by an earlier device error");
  if (!out) return fail(pl, CPRA_ERR_ARG, "out is NULL");
  if (ptr_kind != CPRA_PTR_HOST && ptr_kind != CPRA_PTR_DEVICE) return fail(pl, CPRA_ERR_ARG, "bad ptr_kind");
  {
    const cpra_status st = check_data(pl);
    if (st != CPRA_OK) return st;
  }
  const size_t bytes = (size_t)pl->R * pl->p.Np * pl->p.N * pl->p.N * (pl->p.real_type == CPRA_REAL_F64 ? 8 : 4);
  const char* src = pl->ws + (pl->cur ? pl->L.g1 : pl->L.g0);
  HIPCHK(pl, hipMemcpyAsync(out, src, bytes, ptr_kind == CPRA_PTR_HOST ? hipMemcpyDeviceToHost : hipMemcpyDeviceToDevice,
                            pl->stream));
  if (ptr_kind == CPRA_PTR_HOST) HIPCHK(pl, hipStreamSynchronize(pl->stream));
  return CPRA_OK;
}

cpra_status cpra_assemble_volume(cpra_plan_t pl, void* d_volume) {
  if (!pl) return fail(nullptr, CPRA_ERR_ARG, "plan is NULL");
  if (pl->poisoned) return fail(pl, CPRA_ERR_STATE, "plan is poisoned by an earlier device error");
  if (!d_volume) return fail(pl, CPRA_ERR_ARG, "d_volume is NULL");
  if (pl->k == 0 || pl->k % pl->p.n_ei != 0)
    return fail(pl, CPRA_ERR_STATE, "step D needs an episode end (k=%lld, n_ei=%d)", (long long)pl->k, pl->p.n_ei);
  cpra_status st = check_data(pl);
  if (st != CPRA_OK) return st;
  st = ensure_stepd_tables(pl);
  if (st != CPRA_OK) return st;
  Ops ops = ops_of(pl->p);
  ops.assemble(pl, d_volume);
  LAUNCHCHK(pl);
  return CPRA_OK;
}

cpra_status cpra_destroy(cpra_plan_t pl) {
  delete pl;
  return CPRA_OK;
}

const char* cpra_last_error(cpra_plan_t pl) { return pl ? pl->err.c_str() : g_create_error.c_str(); }

cpra_status cpra_iteration_count(cpra_plan_t pl, int64_t* k) {
  if (!pl || !k) return CPRA_ERR_ARG;
  *k = pl->k;
  return CPRA_OK;
}

cpra_status cpra_set_graphs(cpra_plan_t pl, int32_t enable) {
  if (!pl) return fail(nullptr, CPRA_ERR_ARG, "plan is NULL");
  pl->use_graphs = enable != 0;
  if (!pl->use_graphs) pl->drop_graphs();
  return CPRA_OK;
}

cpra_status cpra_set_chunk(cpra_plan_t pl, int32_t slots) {
  if (!pl) return fail(nullptr, CPRA_ERR_ARG, "plan is NULL");
  if (slots < 0) return fail(pl, CPRA_ERR_ARG, "slots < 0");
  pl->chunk = slots;
  pl->drop_graphs();
  return CPRA_OK;
}

cpra_status cpra_set_kernel_timing(cpra_plan_t pl, int32_t enable) {
  if (!pl) return fail(nullptr, CPRA_ERR_ARG, "plan is NULL");
  pl->timing = enable != 0;
  pl->ev_used = 0;
  return CPRA_OK;
}

cpra_status cpra_kernel_timing(cpra_plan_t pl, double* col_ms, int64_t* col_launches, double* row_ms,
                               int64_t* row_launches) {
  if (!pl || !col_ms || !col_launches || !row_ms || !row_launches) return fail(pl, CPRA_ERR_ARG, "NULL argument");
  if (pl->poisoned) return fail(pl, CPRA_ERR_STATE, "plan is poisoned by an earlier device error");
  HIPCHK(pl, hipStreamSynchronize(pl->stream));
  double c = 0.0, r = 0.0;
  const size_t trip = pl->ev_used / 3;
  for (size_t i = 0; i < trip; ++i) {
    float a = 0.f, b = 0.f;
    HIPCHK(pl, hipEventElapsedTime(&a, pl->evpool[3 * i], pl->evpool[3 * i + 1]));
    HIPCHK(pl, hipEventElapsedTime(&b, pl->evpool[3 * i + 1], pl->evpool[3 * i + 2]));
    c += a;
    r += b;
  }
  *col_ms = c;
  *row_ms = r;
  *col_launches = (int64_t)trip;
  *row_launches = (int64_t)trip;
  pl->ev_used = 0;
  return CPRA_OK;
}

cpra_status cpra_slice_cells(int32_t N, int32_t Np, const double* theta, int32_t* kx_out, int32_t* ky_out) {
  if (N < 2 || (N % 2) != 0 || Np < 1 || !kx_out || !ky_out) return fail(nullptr, CPRA_ERR_ARG, "bad arguments");
  cpra_host::slice_cells(N, Np, theta, kx_out, ky_out);
  return CPRA_OK;
}

cpra_status cpra_coupling_table(const cpra_params* params, const uint8_t* present, int32_t* left, int32_t* right,
                                double* w, uint8_t* mirror) {
  std::string msg;
  cpra_status st = validate(params, msg);
  if (st != CPRA_OK) return fail(nullptr, st, "%s", msg.c_str());
  if (!left || !right || !w || !mirror) return fail(nullptr, CPRA_ERR_ARG, "output is NULL");
  std::vector<cpra_host::Coupling> t;
  cpra_host::coupling_table(params->Np, present, params->alpha, params->wrap == CPRA_WRAP_MIRROR, t);
  for (int n = 0; n < params->Np; ++n) {
    left[n] = t[n].left;
    right[n] = t[n].right;
    w[3 * n] = t[n].wl;
    w[3 * n + 1] = t[n].w0;
    w[3 * n + 2] = t[n].wr;
    mirror[2 * n] = (uint8_t)t[n].mirror_left;
    mirror[2 * n + 1] = (uint8_t)t[n].mirror_right;
  }
  return CPRA_OK;
}

}  // extern "C"
