// C ABI of the channel RK3 hot path: context, workspace layout, sub-step driver.
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <algorithm>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/chn.h"
#include "kernels.hpp"

namespace {

using chn::FftPlan;

// Semi-implicit low-storage RK3 of Spalart, Moser & Rogers (1991), which the
// paper cites without printing the values.
const double kAlpha[3] = {29.0 / 96.0, -3.0 / 40.0, 1.0 / 6.0};
const double kBeta[3] = {37.0 / 160.0, 5.0 / 24.0, 1.0 / 6.0};
const double kGamma[3] = {8.0 / 15.0, 5.0 / 12.0, 3.0 / 4.0};
const double kZeta[3] = {0.0, -17.0 / 60.0, -5.0 / 12.0};

std::string g_create_error;

// A sub-step whose CFL number dt max(|u1|/dx + |u2|/dy_j + |u3|/dz) is above
// this (or not finite) leaves the state untouched and the call returns
// CHN_EUNSTABLE.
constexpr double kCflLimit = 2.0;

// chn_create refuses a mesh on which cond_1(A1) or cond_1(A2 with Dirichlet
// end rows) exceeds this.
constexpr double kCondMax = 1e6;

constexpr int kMaxQ = 4096;  // largest q1, q3 of the filter stage's output grid

bool smooth23(int n) {
  if (n < 1) return false;
  while (n % 2 == 0) n /= 2;
  while (n % 3 == 0) n /= 3;
  return n == 1;
}

struct Carver {
  size_t off = 0;
  char* base = nullptr;
  void* take(size_t bytes) {
    off = (off + 255) & ~(size_t)255;
    void* p = base ? base + off : nullptr;
    off += bytes;
    return p;
  }
};

}  // namespace

struct chn_ctx {
  chn_config cfg{};
  std::vector<double> y;
  hipStream_t stream = nullptr;
  int n1 = 0, n2 = 0, n3 = 0, n1h = 0, M = 0, p1 = 0, p3 = 0;
  double nu = 0.0;
  bool mixed = false, have_state = false, phase_valid = false;
  chn_status sticky = CHN_OK;
  std::string err;
  size_t ws_bytes = 0;
  // state
  double *v = nullptr, *chi = nullptr, *om2 = nullptr, *nchi_old = nullptr, *nom_old = nullptr;
  double *U1 = nullptr, *U3 = nullptr, *nu_old = nullptr, *nw_old = nullptr;
  // phase buffers (element type = fft precision)
  void* ph[6] = {};
  void* H[3] = {};
  void* inter = nullptr;
  size_t inter_bytes = 0;
  double* S[8] = {};
  double* SU[8] = {};
  double* junk = nullptr;  // one lane-indexed row that absorbs history writes nobody reads
  double* rowsum = nullptr;
  double* rowcfl = nullptr;
  // homogeneous solutions and Helmholtz factor tables of the three sub-steps
  // for the time step htab_dt, and the Poisson factor table (SU[4..7]).  The
  // tables of sub-steps 1 and 2 share S[3], S[4], S[6], S[7] with the filter
  // stage and chn_get_fields, which reset htab_dt.
  double* hc[3] = {};
  double* hw[3] = {};
  double* hm[3] = {};
  double* hu[3][4] = {};
  double htab_dt = 0.0;  // 0: not computed
  // tables
  double *A1, *B1, *A2, *B2, *L1d, *U1d, *L1u, *U1u, *L2d, *U2d, *clo, *chi_w, *quad, *inv_dy;
  void *tw1 = nullptr, *tw3 = nullptr;
  double2 *tw1d = nullptr, *tw3d = nullptr, *twq = nullptr;  // float64 tables (filter stage)
  std::vector<double> twq_host;
  double2* twf = nullptr;  // filter-grid tables (filter stage) of the plans twf_p1, twf_p3
  std::vector<double> twf_host;
  FftPlan twf_p1{}, twf_p3{}, twf_pz{};
  FftPlan plan1{}, plan3{};
  double *mean_scr = nullptr, *mean_out = nullptr, *info_dev = nullptr;
  unsigned* guard = nullptr;  // instability guard, four words (common.hpp)
  // per-phase times of the last step of chn_step_rk3 when info is requested
  bool phase_rec = false;
  std::vector<double> hA1, hB1, hA2, hB2, hquad;
  chn::PencilGeom geom{};
  chn::PlaneDims dims{};
  int lds_max = 65536;  // bytes of LDS one workgroup may use on this device
  // plane-phase schedule (chn_set_plan / chn_autotune)
  int xrows = 2;        // x-pass rows per workgroup (2, or 1 for long rows)
  int zK = 1;           // lines per z-pass workgroup
  int ychunk = 1;       // planes per plane-phase launch
  int ffix = 0;         // compile-time radix schedules where available
  int zpipe = 0;        // pipelined z passes (next field's loads during this field's transform)
  int radix = 0;        // radix sets: bit 0 composite radices for plan1 (x), bit 1 for plan3 (z)
  bool in_ensemble = false;  // a channel of an ensemble: keeps the radix sets its batched tables were built with
  int ychunk_max = 1;   // planes the intermediate holds
  bool planes_only = false;
  // per-kernel timing (chn_timing_enable): events bracketing every launch
  bool timing = false;
  struct Timed { int kind; hipEvent_t a, b; };
  std::vector<Timed> timed;
  std::vector<Timed> phase_timed;
  std::vector<hipEvent_t> pool;
  size_t pool_used = 0;
  // one RK3 step (three sub-steps) captured as a graph and replayed, for
  // the time step and schedule of graph_key
  bool use_graph = true;
  hipStream_t cap = nullptr;  // capture stream (the caller's may be the null stream)
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<double> graph_key;
  void drop_graph() {
    if (gexec) (void)hipGraphExecDestroy(gexec);
    if (graph) (void)hipGraphDestroy(graph);
    gexec = nullptr;
    graph = nullptr;
    graph_key.clear();
  }
  ~chn_ctx() {
    drop_graph();
    if (cap) (void)hipStreamDestroy(cap);
    for (hipEvent_t e : pool) (void)hipEventDestroy(e);
  }
};

namespace {

size_t layout(const chn_config* c, char* base, chn_ctx* x) {
  const int n1h = c->n1 / 2, n2 = c->n2, n3 = c->n3;
  const int p1 = 3 * c->n1 / 2, p3 = 3 * c->n3 / 2;
  const size_t M = (size_t)n1h * n3, NP = (size_t)n2 * M;
  const size_t te = c->precision == CHN_MIXED ? 8 : 16;
  // a planes_only context keeps no state, phase or pencil buffers
  const bool po = c->planes_only != 0;
  const size_t CB = po ? 0 : 16 * NP;
  const size_t NPb = po ? 0 : NP;
  const int ych = po ? c->plane_chunk : n2;
  Carver cv;
  cv.base = base;
  auto D = [&](size_t n) { return reinterpret_cast<double*>(cv.take(n * sizeof(double))); };
  double* v = reinterpret_cast<double*>(cv.take(CB));
  double* chi = reinterpret_cast<double*>(cv.take(CB));
  double* om2 = reinterpret_cast<double*>(cv.take(CB));
  double* nco = reinterpret_cast<double*>(cv.take(CB));
  double* noo = reinterpret_cast<double*>(cv.take(CB));
  double* U1 = D(n2);
  double* U3 = D(n2);
  double* nuo = D(n2);
  double* nwo = D(n2);
  void* ph[6];
  for (int f = 0; f < 6; ++f) ph[f] = cv.take(te * NPb);
  void* H[3];
  for (int f = 0; f < 3; ++f) H[f] = cv.take(te * NPb);
  const size_t ib = te * 6 * (size_t)ych * p3 * n1h;
  void* inter = cv.take(ib);
  // (the pencil kernel keeps its scratch rows per wave: every lane of its
  // last workgroup, up to 256 beyond M, has its own column)
  const size_t SB = po ? 0 : CB + 16 * (size_t)n2 * 256;
  double* S[8];
  for (int k = 0; k < 8; ++k) S[k] = reinterpret_cast<double*>(cv.take(SB));
  double* SU[8];
  for (int k = 0; k < 8; ++k) SU[k] = D(NPb);
  double* junk = D(po ? 0 : 2 * M);
  double* hc[3];
  double* hw[3];
  double* hm[3];
  for (int k = 0; k < 3; ++k) {
    hc[k] = reinterpret_cast<double*>(cv.take(CB));
    hw[k] = reinterpret_cast<double*>(cv.take(CB));
    hm[k] = D(po ? 0 : 4 * M);
  }
  double* rowsum = D(2 * (size_t)n2 * p3);
  double* rowcfl = D((size_t)n2 * p3);
  double* tabs = D((size_t)n2 * (4 * 7 + 3 * 3 + 3 * 4 + 4));
  void* tw1 = cv.take(te * (size_t)p1);
  void* tw3 = cv.take(te * (size_t)p3);
  void* tw1d = cv.take(16 * (size_t)p1);
  void* tw3d = cv.take(16 * (size_t)p3);
  void* twq = cv.take(16 * (size_t)kMaxQ * 2);
  void* twf = cv.take(16 * (size_t)kMaxQ * 3);
  double* mean_scr = D(3 * (size_t)n2 * 5 + 4 * (size_t)n2);
  double* mean_out = D(8);
  double* info = D(8);
  unsigned* guard = reinterpret_cast<unsigned*>(cv.take(4 * sizeof(unsigned)));
  if (x) {
    x->v = v; x->chi = chi; x->om2 = om2; x->nchi_old = nco; x->nom_old = noo;
    x->U1 = U1; x->U3 = U3; x->nu_old = nuo; x->nw_old = nwo;
    for (int f = 0; f < 6; ++f) x->ph[f] = ph[f];
    for (int f = 0; f < 3; ++f) x->H[f] = H[f];
    x->inter = inter;
    x->inter_bytes = ib;
    for (int k = 0; k < 8; ++k) { x->S[k] = S[k]; x->SU[k] = SU[k]; }
    x->junk = junk;
    // Helmholtz factor tables, NP doubles each: sub-step 0 in SU[0..3], 1 and
    // 2 in the halves of S[3], S[4] and S[6], S[7] (2 NP doubles each)
    for (int k = 0; k < 4; ++k) {
      x->hu[0][k] = SU[k];
      x->hu[1][k] = S[3 + k / 2] + (k % 2) * NPb;
      x->hu[2][k] = S[6 + k / 2] + (k % 2) * NPb;
    }
    x->rowsum = rowsum; x->rowcfl = rowcfl;
    for (int k = 0; k < 3; ++k) { x->hc[k] = hc[k]; x->hw[k] = hw[k]; x->hm[k] = hm[k]; }
    double* t = tabs;
    x->A1 = t; t += 7 * n2; x->B1 = t; t += 7 * n2; x->A2 = t; t += 7 * n2; x->B2 = t; t += 7 * n2;
    x->L1d = t; t += 3 * n2; x->L1u = t; t += 3 * n2; x->L2d = t; t += 3 * n2;
    x->U1d = t; t += 4 * n2; x->U1u = t; t += 4 * n2; x->U2d = t; t += 4 * n2;
    x->clo = t; t += n2; x->chi_w = t; t += n2; x->quad = t; t += n2; x->inv_dy = t; t += n2;
    x->tw1 = tw1; x->tw3 = tw3;
    x->tw1d = reinterpret_cast<double2*>(tw1d);
    x->tw3d = reinterpret_cast<double2*>(tw3d);
    x->twq = reinterpret_cast<double2*>(twq);
    x->twf = reinterpret_cast<double2*>(twf);
    x->mean_scr = mean_scr; x->mean_out = mean_out; x->info_dev = info;
    x->guard = guard;
  }
  return cv.off + 256;
}

const char* validate(const chn_config* c) {
  if (!c) return "config is NULL";
  if (c->n1 < 4 || c->n3 < 4 || (c->n1 % 2) || (c->n3 % 4)) return "n1 must be even and >= 4, n3 a multiple of 4";
  if (!smooth23(3 * c->n1 / 2) || !smooth23(3 * c->n3 / 2)) return "3*n1/2 and 3*n3/2 must factor into 2s and 3s";
  if (c->n2 < 9 || c->n2 > 2048) return "n2 must be in [9, 2048]";
  if (!(c->lx > 0) || !(c->lz > 0) || !(c->re_b > 0)) return "lx, lz and re_b must be positive";
  if (c->precision != CHN_FP64 && c->precision != CHN_MIXED) return "unknown precision";
  if (c->plane_chunk < 0 || c->plane_chunk > c->n2) return "plane_chunk must be in [0, n2]";
  if (c->planes_only && c->plane_chunk < 1) return "a planes_only context needs plane_chunk >= 1";
  const int p1 = 3 * c->n1 / 2, p3 = 3 * c->n3 / 2;
  const int maxv = c->precision == CHN_MIXED ? 48 : 24;
  const int vb = c->precision == CHN_MIXED ? 8 : 16;
  if (!chn::xpass_two_rows(p1, vb) && chn::xrow_threads(p1, vb) == 0) return "3*n1/2 too large for the x-pass kernel";
  if (p3 > maxv * 256) return "3*n3/2 too large for the z-pass kernels";
  if (c->y) {
    if (c->y[0] != -1.0 || c->y[c->n2 - 1] != 1.0) return "y must start at -1 and end at 1";
    for (int j = 1; j < c->n2; ++j)
      if (!(c->y[j] > c->y[j - 1])) return "y must be strictly ascending";
  }
  return nullptr;
}

chn_status fail(chn_ctx* x, chn_status s, const std::string& m) {
  if (x) {
    x->err = m;
    if (s == CHN_EDEVICE) x->sticky = CHN_EDEVICE;
  } else {
    g_create_error = m;
  }
  return s;
}

#define HIPCHK(ctx, call)                                                              \
  do {                                                                                 \
    hipError_t e_ = (call);                                                            \
    if (e_ != hipSuccess)                                                              \
      return fail((ctx), CHN_EDEVICE, std::string(#call ": ") + hipGetErrorString(e_)); \
  } while (0)

hipEvent_t pool_event(chn_ctx* x) {
  if (x->pool_used == x->pool.size()) {
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    x->pool.push_back(e);
  }
  return x->pool[x->pool_used++];
}

// Runs one kernel launch; with timing on, brackets it with events on the context's stream.
template <typename F> hipError_t timed(chn_ctx* x, int kind, F&& launch) {
  if (!x->timing && !x->phase_rec) return launch();
  hipEvent_t a = pool_event(x), b = pool_event(x);
  if (!a || !b) return hipErrorOutOfMemory;
  hipError_t e = hipEventRecord(a, x->stream);
  if (e == hipSuccess) e = launch();
  if (e == hipSuccess) e = hipEventRecord(b, x->stream);
  if (e == hipSuccess && x->timing) x->timed.push_back({kind, a, b});
  if (e == hipSuccess && x->phase_rec) x->phase_timed.push_back({kind, a, b});
  return e;
}

template <typename T> struct Ty;
template <> struct Ty<double> { using c = double2; };
template <> struct Ty<float> { using c = float2; };


// LDS line stride (complex elements) of the plane kernels for lines of p
// points: one slot skipped after every 8 elements (bank spreading).
int plane_lds_stride(int p) { return p + p / 8 + 1; }

// Largest number of z lines one workgroup can transform (staging registers and LDS).
int z_lines_max(const chn_ctx* x) {
  const int maxv = x->mixed ? 48 : 24;
  const int cb = x->mixed ? 8 : 16;
  int K = maxv * 256 / x->p3;
  const int byl = x->lds_max / (plane_lds_stride(x->p3) * cb);
  if (K > byl) K = byl;
  if (K > x->n1h) K = x->n1h;
  return K;
}
// Default schedule, from the autotuner's choices on 384 x 193 x 384 and on
// the 8192 x 6144 planes: z-pass workgroups of about 2304 (float) or 1152
// (double) points, but at least 1024 of them per launch (small grids); two x
// rows when six lines fit; compile-time radix schedules where they exist.
bool plan_fits(const chn_ctx* x, int xrows, int zK, int ych);
void default_plan(chn_ctx* x) {
  x->ychunk = x->planes_only || x->cfg.plane_chunk > 0 ? x->cfg.plane_chunk : x->n2;
  int K = std::max(1, (x->mixed ? 2304 : 1152) / x->p3);
  K = std::min(K, std::max(1, (int)((size_t)x->ychunk * x->n1h / 1024)));
  x->zK = std::max(1, std::min(K, z_lines_max(x)));
  x->xrows = plan_fits(x, 2, x->zK, x->ychunk) ? 2 : 1;
  x->ffix = 1;
}
bool plan_fits(const chn_ctx* x, int xrows, int zK, int ych) {
  const int cb = x->mixed ? 8 : 16;
  if (ych < 1 || ych > x->ychunk_max) return false;
  if (zK < 1 || zK > z_lines_max(x) || chn::z_staging(x->plan3, zK, cb) == 0) return false;
  if (xrows == 2 || xrows == 4 || xrows == 8)
    return chn::staging_for(x->plan1, 3 * xrows, cb) > 0 &&
           (size_t)3 * xrows * plane_lds_stride(x->p1) * cb <= (size_t)x->lds_max;
  if (xrows == 1) return chn::xrow_fits(x->plan1, cb) && (size_t)x->p1 * cb <= (size_t)x->lds_max;
  return false;
}

// Rebuild plan1, plan3 and their twiddle tables for the radix sets rs
// (bit 0: x transforms composite, bit 1: z transforms composite).
chn_status set_radix(chn_ctx* x, int rs) {
  if (rs == x->radix) return CHN_OK;
  if (x->in_ensemble) return fail(x, CHN_EUNSUPPORTED, "the channels of an ensemble keep the radix sets of their batched tables");
  FftPlan p1{}, p3{};
  std::vector<double> t1, t3;
  const int r1 = (rs & 1) ? chn::host::kRadixComposite : chn::host::kRadixClassic;
  const int r3 = (rs & 2) ? chn::host::kRadixComposite : chn::host::kRadixClassic;
  if (!chn::host::fft_plan(x->p1, &p1, &t1, r1) || !chn::host::fft_plan(x->p3, &p3, &t3, r3))
    return fail(x, CHN_EINVAL, "FFT length not supported by this radix set");
  HIPCHK(x, hipStreamSynchronize(x->stream));
  if (x->mixed) {
    std::vector<float> g1(t1.begin(), t1.end()), g3(t3.begin(), t3.end());
    HIPCHK(x, hipMemcpy(x->tw1, g1.data(), g1.size() * 4, hipMemcpyHostToDevice));
    HIPCHK(x, hipMemcpy(x->tw3, g3.data(), g3.size() * 4, hipMemcpyHostToDevice));
  } else {
    HIPCHK(x, hipMemcpy(x->tw1, t1.data(), t1.size() * 8, hipMemcpyHostToDevice));
    HIPCHK(x, hipMemcpy(x->tw3, t3.data(), t3.size() * 8, hipMemcpyHostToDevice));
  }
  HIPCHK(x, hipMemcpy(x->tw1d, t1.data(), t1.size() * 8, hipMemcpyHostToDevice));
  HIPCHK(x, hipMemcpy(x->tw3d, t3.data(), t3.size() * 8, hipMemcpyHostToDevice));
  x->plan1 = p1;
  x->plan3 = p3;
  x->radix = rs;
  return CHN_OK;
}
template <typename T> int z_lines(const chn_ctx* x) { return x->zK; }

// guard: the context's instability guard inside the time step, else nullptr;
// inter: the transform intermediate (nullptr: the context's own)
template <typename T, typename TO>
void plane_args(chn_ctx* x, const void* const* in, bool omega2_given, void* const* out, chn::ZinvArgs<T>& za,
                chn::XpassArgs<T>& xa, chn::ZfwdArgs<T, TO>& fa, unsigned* guard = nullptr,
                void* inter = nullptr) {
  using C = typename Ty<T>::c;
  if (!inter) inter = x->inter;
  const int K = z_lines<T>(x);
  za = {};
  for (int f = 0; f < 6; ++f) za.in[f] = reinterpret_cast<const C*>(in[f]);
  if (!omega2_given) za.in[4] = nullptr;
  za.out = reinterpret_cast<C*>(inter);
  za.tw = reinterpret_cast<const C*>(x->tw3);
  za.plan = x->plan3;
  za.d = x->dims;
  za.K = K;
  za.lstride = plane_lds_stride(x->p3);
  za.nfields = 6;
  za.nslot = 6;
  za.y0 = 0;
  za.ny = x->n2;
  za.fixed = x->ffix;
  za.pipe = x->zpipe;
  za.guard = guard;
  xa = {};
  xa.buf = reinterpret_cast<C*>(inter);
  xa.tw = reinterpret_cast<const C*>(x->tw1);
  xa.plan = x->plan1;
  xa.d = x->dims;
  xa.lstride = plane_lds_stride(x->p1);
  xa.rowsum = x->rowsum;
  xa.rowcfl = x->rowcfl;
  xa.inv_dx = x->n1 / x->cfg.lx;
  xa.inv_dz = x->n3 / x->cfg.lz;
  xa.inv_dy = x->inv_dy;
  xa.rows = x->xrows;
  xa.y0 = 0;
  xa.ny = x->n2;
  xa.fixed = x->ffix;
  xa.guard = guard;
  fa = {};
  fa.buf = reinterpret_cast<const C*>(inter);
  for (int f = 0; f < 3; ++f) fa.out[f] = reinterpret_cast<typename Ty<TO>::c*>(out[f]);
  fa.tw = reinterpret_cast<const C*>(x->tw3);
  fa.plan = x->plan3;
  fa.d = x->dims;
  fa.K = K;
  fa.lstride = plane_lds_stride(x->p3);
  fa.scale = 1.0 / ((double)x->p1 * x->p3);
  fa.y0 = 0;
  fa.ny = x->n2;
  fa.fixed = x->ffix;
  fa.pipe = x->zpipe;
}

// plane phase: ph (6 slots) -> H (3 slots) through the intermediate
// inter, chunk: an intermediate other than the context's, holding chunk planes
template <typename T, typename TO>
chn_status plane_phase(chn_ctx* x, const void* const* in, bool omega2_given, void* const* out,
                       unsigned* guard = nullptr, void* inter = nullptr, int chunk = 0) {
  chn::ZinvArgs<T> za;
  chn::XpassArgs<T> xa;
  chn::ZfwdArgs<T, TO> fa;
  plane_args<T, TO>(x, in, omega2_given, out, za, xa, fa, guard, inter);
  const int ych = chunk > 0 ? chunk : x->ychunk;
  // chunks of planes: the intermediate holds the chunk from its plane 0
  for (int y0 = 0; y0 < x->n2; y0 += ych) {
    za.y0 = xa.y0 = fa.y0 = y0;
    za.ny = xa.ny = fa.ny = std::min(ych, x->n2 - y0);
    HIPCHK(x, timed(x, CHN_K_ZINV, [&] { return chn::launch_zinv<T>(za, x->stream); }));
    HIPCHK(x, timed(x, CHN_K_XPASS, [&] { return chn::launch_xpass<T>(xa, x->stream); }));
    HIPCHK(x, timed(x, CHN_K_ZFWD, [&] { return chn::launch_zfwd<T, TO>(fa, x->stream); }));
  }
  return CHN_OK;
}

// omega = false: u1, u2, u3 only (out[3], out[4] untouched)
template <typename TP> chn_status recover(chn_ctx* x, TP* const* out, bool omega = true) {
  chn::RecoverArgs<TP> ra{};
  ra.omega = omega ? 1 : 0;
  ra.g = x->geom;
  ra.v = x->v;
  ra.om2 = x->om2;
  ra.U1 = x->U1;
  ra.U3 = x->U3;
  for (int f = 0; f < 5; ++f) ra.out[f] = out[f];
  ra.S0 = x->S[0];
  ra.S1 = x->S[1];
  ra.S2 = x->S[2];
  HIPCHK(x, timed(x, CHN_K_RECOVER, [&] { return chn::launch_recover<TP>(ra, x->stream); }));
  return CHN_OK;
}

template <typename T> T* const* phase_ptrs(chn_ctx* x, T** po) {
  po[0] = reinterpret_cast<T*>(x->ph[0]);
  po[1] = reinterpret_cast<T*>(x->ph[1]);
  po[2] = reinterpret_cast<T*>(x->ph[2]);
  po[3] = reinterpret_cast<T*>(x->ph[3]);
  po[4] = reinterpret_cast<T*>(x->ph[5]);
  return po;
}

template <typename T> void advance_args(chn_ctx* x, int s, double dt, chn::AdvanceArgs<T, T>& aa);

// Homogeneous solutions for the time step dt (recomputed when dt changes).
chn_status homog_tables(chn_ctx* x, double dt, hipStream_t st) {
  if (x->htab_dt == dt) return CHN_OK;
  chn::HomogArgs h{};
  h.g = x->geom;
  h.nu = x->nu;
  h.dt = dt;
  for (int k = 0; k < 3; ++k) {
    h.be[k] = kBeta[k];
    h.hc[k] = x->hc[k];
    h.hw[k] = x->hw[k];
    h.hm[k] = x->hm[k];
  }
  h.S0 = x->S[0];
  h.S1 = x->S[1];
  h.T = x->S[2];
  // four [n2][M] factor-row arrays for the transposed solves, in the plane
  // intermediate (free between plane phases; it holds 9 n2 M doubles or more)
  const size_t NP = (size_t)x->n2 * x->M;
  if (x->inter_bytes < 4 * NP * sizeof(double)) return fail(x, CHN_EUNSUPPORTED, "intermediate too small for k_homog");
  for (int k = 0; k < 4; ++k) h.Q[k] = reinterpret_cast<double*>(x->inter) + k * NP;
  for (int k = 0; k < 8; ++k) h.SU[k] = x->SU[k];
  for (int s = 0; s < 3; ++s)
    for (int k = 0; k < 4; ++k) h.hu[s][k] = x->hu[s][k];
  HIPCHK(x, chn::launch_homog(h, st));
  x->htab_dt = dt;
  return CHN_OK;
}

template <typename T> chn_status substep(chn_ctx* x, int s, double dt) {
  T* po[5];
  phase_ptrs<T>(x, po);
  // 1. velocities and vorticities of the state (after set_state or chn_nonlinear;
  //    otherwise the previous sub-step's advance kernel already wrote them)
  if (!x->phase_valid) {
    chn_status st = recover<T>(x, po);
    if (st != CHN_OK) return st;
    x->phase_valid = true;
  }
  // 2. dealiased u x omega (the x pass also gathers the CFL number for the guard)
  chn_status st = plane_phase<T, T>(x, x->ph, false, x->H, x->guard);
  if (st != CHN_OK) return st;
  // 3. pencils + mean modes + next sub-step's velocities and vorticities
  if (chn_status hs = homog_tables(x, dt, x->stream)) return hs;
  chn::AdvanceArgs<T, T> aa;
  advance_args<T>(x, s, dt, aa);
  HIPCHK(x, timed(x, CHN_K_ADVANCE, [&] { return chn::launch_advance<T, T>(aa, x->stream); }));
  return CHN_OK;
}

template <typename T> void advance_args(chn_ctx* x, int s, double dt, chn::AdvanceArgs<T, T>& aa) {
  T* po[5];
  phase_ptrs<T>(x, po);
  aa = {};
  aa.g = x->geom;
  for (int f = 0; f < 5; ++f) aa.ph[f] = po[f];
  for (int f = 0; f < 3; ++f) aa.H[f] = reinterpret_cast<const T*>(x->H[f]);
  aa.v = x->v; aa.chi = x->chi; aa.om2 = x->om2;
  // histories: sub-step s reads the previous one's N with weight zeta_s; the
  // last sub-step's N is read next by sub-step 0 of the next step, with
  // weight zeta_0.  A zero weight needs no data: the reads then stay on one
  // (finite) row, the writes go to the junk row.
  const size_t st = 2 * (size_t)x->M;
  aa.nchi_rd = x->nchi_old; aa.nom_rd = x->nom_old;
  aa.hist_rs = kZeta[s] == 0.0 ? 0 : st;
  const bool dead = s == 2 && kZeta[0] == 0.0;
  aa.nchi_wr = dead ? x->junk : x->nchi_old;
  aa.nom_wr = dead ? x->junk : x->nom_old;
  aa.hist_ws = dead ? 0 : st;
  for (int k = 0; k < 8; ++k) aa.S[k] = x->S[k];
  for (int k = 0; k < 4; ++k) {
    aa.SU[k] = x->hu[s][k];
    aa.SU[4 + k] = x->SU[4 + k];
  }
  aa.U1 = x->U1; aa.U3 = x->U3; aa.nu_old = x->nu_old; aa.nw_old = x->nw_old;
  aa.rowsum = x->rowsum;
  aa.p3 = x->p3;
  aa.inv_p1p3 = 1.0 / ((double)x->p1 * x->p3);
  aa.mean_scr = x->mean_scr;
  aa.mean_out = x->mean_out;
  aa.mass_flux = x->cfg.mass_flux;
  aa.dt = dt; aa.nu = x->nu;
  aa.al = kAlpha[s]; aa.be = kBeta[s]; aa.ga = kGamma[s]; aa.ze = kZeta[s];
  aa.hc = x->hc[s];
  aa.hw = x->hw[s];
  aa.hm = x->hm[s];
  aa.guard = x->guard;
  aa.cfl_limit = kCflLimit;
  aa.substep = s;
}

// Divergence of the phase velocities (the step record), raised into *maxbits.
template <typename T> chn_status divergence(chn_ctx* x, unsigned long long* maxbits) {
  T* po[5];
  phase_ptrs<T>(x, po);
  if (!x->phase_valid) {
    if (chn_status st = recover<T>(x, po)) return st;
    x->phase_valid = true;
  }
  chn::DivArgs<T> da{};
  da.g = x->geom;
  for (int f = 0; f < 3; ++f) da.u[f] = po[f];
  da.S0 = x->S[0];
  da.maxbits = maxbits;
  HIPCHK(x, chn::launch_div<T>(da, x->stream));
  return CHN_OK;
}

chn_status check(chn_ctx* x);
chn_status need_fields(chn_ctx* x);

// ---------------------------------------------------------------- static scratch
// The transform intermediate of chn_plane_products_static: a file-scope
// device array, one per GPU the library runs on, held until the process
// ends.  In host code its name is only a stand-in: its device address comes
// from hipGetSymbolAddress, taken once per device (with that device
// current) and kept in g_scratch_ptr; every launch uses that address.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
constexpr int kMaxDevices = 64;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
void* g_scratch_ptr[kMaxDevices] = {};
std::mutex g_scratch_mu;

chn_status static_scratch(chn_ctx* x, void** out) {
  int dev = -1;
  HIPCHK(x, hipGetDevice(&dev));
  if (dev < 0 || dev >= kMaxDevices) return fail(x, CHN_EUNSUPPORTED, "device index beyond the static scratch table");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    HIPCHK(x, hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(x, CHN_EDEVICE, "hipGetSymbolAddress returned no address for the static scratch");
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return CHN_OK;
}

// The filter stage transforms in float64 on both paths.  tau_ij is a small
// difference of F(u_i u_j) and F(u_i) F(u_j) (about 1e-2 to 1e-3 of either
// term on the 1536 x 385 x 1152 field), so the 1.6e-7 relative error of
// float32 transforms reaches 1e-4 in tau.  The mixed path stores the
// velocity coefficients in float32 (every term of tau then sees the same
// rounded data) and keeps the transforms and products in float64.
// With d_ens the same transforms run on the vorticity (omega1, omega2,
// omega3) instead of the velocity, and only the trace F(omega_i omega_i), the
// filtered enstrophy, is written (q1, q3, d_ubar, d_uubar, d_tau unused).
// Smallest 2,3-smooth size above 2 h + kc (h = highest stored wavenumber of
// the direction, kc = cut-off), at most p: a grid on which the retained modes
// of every product are exact.
int filter_grid(int h, int kc, int p) {
  for (int n = 2 * h + kc + 1; n < p; ++n)
    if (smooth23(n)) return n;
  return p;
}

// The low-storage stage (filter + products + stresses, or the filtered
// enstrophy when d_ens is given) from the phase-precision fields of the
// state.  Buffers: the z-inverse output in the plane intermediate, the x
// output in S[0..2], pp in the H buffers, the q-grid intermediate in the
// plane intermediate.  The state, the phase fields and the factor tables
// are left as they are.
chn_status filter_stage(chn_ctx* x, int kcx, int kcz, int q1, int q3, double* d_ubar, double* d_uubar,
                        double* d_tau, double* d_ens = nullptr) {
  using CT = double2;
  const bool ens = d_ens != nullptr;
  const int n2 = x->n2, n1h = x->n1h, n3 = x->n3;
  if (!ens && (!d_ubar || !d_uubar)) return fail(x, CHN_EINVAL, "NULL output pointer");
  if (kcx < 0 || kcz < 0 || kcx >= n1h || kcz >= n3 / 2) return fail(x, CHN_EINVAL, "need 0 <= kcx < n1/2, 0 <= kcz < n3/2");
  if (!ens && (q1 <= 2 * kcx || q3 <= 2 * kcz || (q1 % 2) || (q3 % 2) || !smooth23(q1) || !smooth23(q3) ||
               q1 > kMaxQ || q3 > kMaxQ))
    return fail(x, CHN_EINVAL, "q1, q3 must be even, 2,3-smooth, <= 4096 and exceed 2 kcx, 2 kcz");
  const int kc1 = kcx + 1, nz = 2 * kcz + 1;
  const size_t NP = (size_t)n2 * x->M;
  const int f1 = filter_grid(n1h - 1, kcx, x->p1), f3 = filter_grid(n3 / 2 - 1, kcz, x->p3);
  const int nout = ens ? 1 : 6;
  if (f1 > 12 * 256 || f3 > kMaxQ) return fail(x, CHN_EUNSUPPORTED, "plane too large for the filter x-pass");
  if ((size_t)3 * n2 * f3 * n1h * sizeof(CT) > x->inter_bytes)
    return fail(x, CHN_EUNSUPPORTED, "filter grid too large for the workspace");
  // S[0..2] are consecutive allocations, so their span holds 3 * 16 NP bytes
  if ((size_t)nout * n2 * f3 * kc1 * 16 > 3 * 16 * NP) return fail(x, CHN_EUNSUPPORTED, "kcx too large for the workspace");
  if (!ens && (size_t)6 * n2 * kc1 * nz * 16 > 3 * NP * (x->mixed ? 8 : 16))
    return fail(x, CHN_EUNSUPPORTED, "cut-off too large for the workspace");
  if (!ens && (size_t)9 * n2 * q3 * kc1 * 16 > x->inter_bytes) return fail(x, CHN_EUNSUPPORTED, "q grid too large for the workspace");
  const size_t lds_x = (size_t)(f1 + 1) * 16;  // one float64 line
  const size_t lds_t = (size_t)5 * (q1 + 1) * 16;
  auto lines = [&](int len, int cap) {
    int K = 24 * 256 / len;
    const int byl = x->lds_max / ((len + 1) * 16);
    if (K > byl) K = byl;
    if (K > 16) K = 16;
    if (K > cap) K = cap;
    return K < 1 ? 1 : K;
  };
  int Kf = lines(f3, kc1);
  const int Kq = ens ? 1 : lines(q3, kc1);
  if (lds_x > (size_t)x->lds_max || (size_t)(f3 + 1) * 16 > (size_t)x->lds_max || f3 > 24 * 256 ||
      (!ens && (lds_t > (size_t)x->lds_max || 5 * q1 > 24 * 256 || q3 > 24 * 256)))
    return fail(x, CHN_EUNSUPPORTED, "plane too large for the filter kernels' LDS tiles on this device");
  // z inverse: one line per workgroup, one field at a time (float64 lines:
  // the fewest registers give the most waves; measured on 1536x385x1152,
  // 20 -> 15 ms against two lines with the pipelined loads)
  const int zls = plane_lds_stride(f3);
  const int zK = 1;
  if ((size_t)zK * zls * sizeof(CT) > (size_t)x->lds_max) return fail(x, CHN_EUNSUPPORTED, "z lines exceed LDS");
  // FFT plans (float64 tables): the composite radix set where every launch's
  // staging holds it, else the classic one
  auto make_plan = [&](int n, FftPlan* pl, std::vector<double>* t, auto fits) {
    if (chn::host::fft_plan(n, pl, t, chn::host::kRadixComposite) && fits(*pl)) return true;
    return chn::host::fft_plan(n, pl, t, chn::host::kRadixClassic) && fits(*pl);
  };
  FftPlan pf1{}, pf3{}, pz3{};
  {
    std::vector<double> t1, t3;
    // the z forward takes the most lines per workgroup (at most Kf) the plan's staging holds
    const int kf_max = Kf;
    auto z_fits = [&](const FftPlan& p) {
      if (chn::z_staging(p, zK, 16) == 0) return false;
      for (Kf = kf_max; Kf >= 1; --Kf)
        if (chn::staging_fits(p, Kf, 256, 24)) return true;
      return false;
    };
    // the float64 z inverse keeps small radices: the composite form with
    // radices up to 16 needs staging registers that cost occupancy.  Radices
    // up to 6 are taken where they save passes over the classic set (1296 as
    // 6, 6, 6, 6 instead of 8, 2, 3, 3, 3, 3: the same eight staged values
    // per thread; on 1536x385x1152, filter + stresses 43.1 -> 42.3 ms,
    // filtered enstrophy 28.3 -> 27.0 ms), else the classic radices.
    auto fewer_passes_up_to6 = [](int n) {
      FftPlan a{}, b{};
      std::vector<double> t;
      return chn::host::fft_plan(n, &a, &t, chn::host::kRadixUpTo6) &&
             (!chn::host::fft_plan(n, &b, &t, chn::host::kRadixClassic) || a.npass < b.npass);
    };
    std::vector<double> tz;
    if (!make_plan(f1, &pf1, &t1, [&](const FftPlan& p) { return chn::staging_fits(p, 1, 256, 16); }) ||
        !make_plan(f3, &pf3, &t3, z_fits) ||
        !((fewer_passes_up_to6(f3) && chn::host::fft_plan(f3, &pz3, &tz, chn::host::kRadixUpTo6) &&
           chn::z_staging(pz3, zK, 16) > 0) ||
          (chn::host::fft_plan(f3, &pz3, &tz, chn::host::kRadixClassic) && chn::z_staging(pz3, zK, 16) > 0) ||
          (chn::host::fft_plan(f3, &pz3, &tz, chn::host::kRadixComposite) && chn::z_staging(pz3, zK, 16) > 0)))
      return fail(x, CHN_EUNSUPPORTED, "filter grid not supported by the transform kernels");
    if (std::memcmp(&x->twf_p1, &pf1, sizeof pf1) != 0 || std::memcmp(&x->twf_p3, &pf3, sizeof pf3) != 0 ||
        std::memcmp(&x->twf_pz, &pz3, sizeof pz3) != 0) {
      std::vector<double>& h = x->twf_host;  // [f1 | f3 z forward | f3 z inverse], kMaxQ entries each
      h.assign((size_t)6 * kMaxQ, 0.0);
      std::copy(t1.begin(), t1.end(), h.begin());
      std::copy(t3.begin(), t3.end(), h.begin() + 2 * kMaxQ);
      std::copy(tz.begin(), tz.end(), h.begin() + 4 * kMaxQ);
      HIPCHK(x, hipMemcpyAsync(x->twf, h.data(), h.size() * 8, hipMemcpyHostToDevice, x->stream));
      x->twf_p1 = pf1;
      x->twf_p3 = pf3;
      x->twf_pz = pz3;
    }
  }
  const double2* twf1 = x->twf;
  const double2* twf3 = x->twf + kMaxQ;
  const double2* twz3 = x->twf + 2 * kMaxQ;
  FftPlan pq1{}, pq3{};
  if (!ens) {
    std::vector<double> t1, t3;
    if (!make_plan(q1, &pq1, &t1, [&](const FftPlan& p) { return chn::staging_fits(p, 5, 256, 24); }) ||
        !make_plan(q3, &pq3, &t3, [&](const FftPlan& p) { return chn::staging_fits(p, Kq, 256, 24); }))
      return fail(x, CHN_EINVAL, "q grid not supported");
    x->twq_host.assign(t1.begin(), t1.end());
    x->twq_host.resize(2 * kMaxQ, 0.0);
    x->twq_host.insert(x->twq_host.end(), t3.begin(), t3.end());
    HIPCHK(x, hipMemcpyAsync(x->twq, x->twq_host.data(), x->twq_host.size() * 8, hipMemcpyHostToDevice, x->stream));
  }
  const double2* twq1 = x->twq;
  const double2* twq3 = x->twq + kMaxQ;
  // 1. the phase fields of the state: u1, u2, u3, omega1, omega3 (current
  //    after a step; recovered for a new state), float32 on the mixed path;
  //    omega2 is the float64 state itself
  void* po[5];
  if (x->mixed) {
    float* pf[5];
    phase_ptrs<float>(x, pf);
    if (!x->phase_valid) {
      if (chn_status st = recover<float>(x, pf)) return st;
      x->phase_valid = true;
    }
    for (int f = 0; f < 5; ++f) po[f] = pf[f];
  } else {
    double* pd[5];
    phase_ptrs<double>(x, pd);
    if (!x->phase_valid) {
      if (chn_status st = recover<double>(x, pd)) return st;
      x->phase_valid = true;
    }
    for (int f = 0; f < 5; ++f) po[f] = pd[f];
  }
  chn::FieldsIn fin{};
  const unsigned all32 = x->mixed ? 7u : 0u;
  if (ens) {
    fin.u[0] = po[3];
    fin.u[1] = x->om2;
    fin.u[2] = po[4];
    fin.f32 = all32 & 5u;
  } else {
    for (int f = 0; f < 3; ++f) fin.u[f] = po[f];
    fin.f32 = all32;
  }
  // 2. z inverse of the fluctuations onto f3 points
  chn::PlaneDims fd = x->dims;
  fd.p1 = f1;
  fd.p3 = f3;
  chn::ZinvArgs<double> za{};
  for (int f = 0; f < 3; ++f) za.in[f] = reinterpret_cast<const CT*>(fin.u[f]);
  za.in_f32 = fin.f32;
  za.out = reinterpret_cast<CT*>(x->inter);
  za.tw = twz3;
  za.plan = pz3;
  za.d = fd;
  za.lstride = zls;
  za.K = zK;
  za.nfields = 3;
  za.nslot = 3;
  za.zero_mean = 1;
  za.y0 = 0;
  za.ny = n2;
  za.pipe = 0;
  HIPCHK(x, timed(x, CHN_K_FILTER, [&] { return chn::launch_zinv<double>(za, x->stream); }));
  // 3. inverse in x, products, float64 forward in x
  chn::XfilterArgs<double> xa{};
  xa.buf = za.out;
  xa.out = reinterpret_cast<double2*>(x->S[0]);
  xa.plane_stride = (size_t)nout * f3 * kc1;
  xa.tw = twf1;
  xa.plan = pf1;
  xa.tw_d = twf1;
  xa.n1h = n1h;
  xa.n2 = n2;
  xa.f1 = f1;
  xa.f3 = f3;
  xa.lst = f1 + 1;
  xa.lsd = f1 + 1;
  xa.kcx = kcx;
  xa.trace = ens ? 1 : 0;
  HIPCHK(x, timed(x, CHN_K_FILTER, [&] { return chn::launch_xfilter<double>(xa, lds_x, x->stream); }));
  // 4. float64 forward in z, retained set, mean terms
  chn::ZfilterArgs fa{};
  fa.xout = xa.out;
  fa.plane_stride = xa.plane_stride;
  fa.u = fin;
  fa.pp = reinterpret_cast<double2*>(x->H[0]);
  fa.uubar = ens ? nullptr : reinterpret_cast<double2*>(d_uubar);
  fa.ubar = ens ? nullptr : reinterpret_cast<double2*>(d_ubar);
  fa.trace = ens ? reinterpret_cast<double2*>(d_ens) : nullptr;
  fa.trace_only = ens ? 1 : 0;
  fa.tw = twf3;
  fa.plan = pf3;
  fa.n1h = n1h;
  fa.n2 = n2;
  fa.n3 = n3;
  fa.f3 = f3;
  fa.kcx = kcx;
  fa.kcz = kcz;
  fa.K = Kf;
  fa.lstride = f3 + 1;
  fa.scale = 1.0 / ((double)f1 * f3);
  HIPCHK(x, timed(x, CHN_K_FILTER, [&] {
    return chn::launch_zfilter(fa, (size_t)Kf * (f3 + 1) * 16, x->stream);
  }));
  if (ens || !d_tau) return CHN_OK;
  // 5. q grid: inverse in z, then in x with tau = pp - ub ub
  chn::ZinvQArgs qa{};
  qa.pp = fa.pp;
  qa.u = fin;
  qa.out = reinterpret_cast<double2*>(x->inter);
  qa.tw = twq3;
  qa.plan = pq3;
  qa.n1h = n1h; qa.n2 = n2; qa.n3 = n3; qa.q3 = q3; qa.kcx = kcx; qa.kcz = kcz; qa.K = Kq;
  qa.lstride = q3 + 1;
  HIPCHK(x, timed(x, CHN_K_FILTER, [&] {
    return chn::launch_zinv_q(qa, (size_t)Kq * (q3 + 1) * 16, x->stream);
  }));
  chn::XtauArgs ta{};
  ta.in = qa.out;
  ta.tau = d_tau;
  ta.tw = twq1;
  ta.plan = pq1;
  ta.n2 = n2; ta.q1 = q1; ta.q3 = q3; ta.kcx = kcx;
  ta.lstride = q1 + 1;
  HIPCHK(x, timed(x, CHN_K_FILTER, [&] { return chn::launch_xtau(ta, lds_t, x->stream); }));
  return CHN_OK;
}

chn_status need_fields(chn_ctx* x) {
  return x->planes_only ? fail(x, CHN_EUNSUPPORTED, "not available on a planes_only context") : CHN_OK;
}

chn_status check(chn_ctx* x) {
  if (!x) return CHN_EINVAL;
  if (x->sticky != CHN_OK) return x->sticky;
  return CHN_OK;
}

}  // namespace


// ---------------------------------------------------------------- ensembles
struct chn_ens {
  int n = 0;
  bool mixed = false;
  hipStream_t user = nullptr, own = nullptr, own2 = nullptr;
  hipEvent_t ev_in = nullptr, ev_out = nullptr, ev_lag = nullptr, ev_join = nullptr;
  std::vector<chn_ctx*> ctx;
  std::string err;
  // device tables
  void* d_zinv = nullptr;
  void* d_xpass = nullptr;
  void* d_zfwd = nullptr;
  void* d_adv = nullptr;      // [3][n] advance argument blocks
  unsigned* d_guard = nullptr;  // [n][4] instability guards of the channels
  int4 *d_wz = nullptr, *d_wx = nullptr, *d_wa = nullptr;
  int nz = 0, nx = 0, na = 0;
  // two groups of channels (work-list items of group 0 first): the step
  // graph runs them on two branches, group 1 one plane phase behind, so one
  // group's pencil phase overlaps the other's plane phase
  int gz[2] = {0, 0}, gx[2] = {0, 0}, ga[2] = {0, 0};
  bool lag = true;  // group 1 starts after group 0's first plane phase
  int n2max = 0;     // largest wall-normal size (LDS tables of the pencil kernel)
  size_t lds_z = 0, lds_x = 0;
  int mz = 0, mx = 0;  // transform staging of the batched z and x passes
  int rz = 2;          // rows per batched x-pass workgroup
  int comp = 0;        // some channel's plans hold composite radices
  std::vector<char> h_adv;    // host copy of the advance blocks (dt dependent)
  std::vector<double> last_dt;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  ~chn_ens() {
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
    for (chn_ctx* c : ctx) delete c;
    if (ev_in) (void)hipEventDestroy(ev_in);
    if (ev_out) (void)hipEventDestroy(ev_out);
    if (ev_lag) (void)hipEventDestroy(ev_lag);
    if (ev_join) (void)hipEventDestroy(ev_join);
    if (own) (void)hipStreamDestroy(own);
    if (own2) (void)hipStreamDestroy(own2);
  }
};

namespace {

// Per-channel workspace sizes and the ensemble's own tables, 256-byte aligned.
struct EnsLayout {
  std::vector<size_t> off, bytes;
  size_t tables = 0, total = 0;
};

size_t arg_bytes(bool mixed) {
  return mixed ? sizeof(chn::ZinvArgs<float>) + sizeof(chn::XpassArgs<float>) + sizeof(chn::ZfwdArgs<float, float>) +
                     3 * sizeof(chn::AdvanceArgs<float, float>)
               : sizeof(chn::ZinvArgs<double>) + sizeof(chn::XpassArgs<double>) +
                     sizeof(chn::ZfwdArgs<double, double>) + 3 * sizeof(chn::AdvanceArgs<double, double>);
}

bool ens_layout(int n, const chn_config* cfgs, EnsLayout* L) {
  if (n < 1 || !cfgs) return false;
  size_t off = 0, items = 0;
  for (int i = 0; i < n; ++i) {
    if (validate(&cfgs[i])) return false;
    if (cfgs[i].precision != cfgs[0].precision || cfgs[i].stream != cfgs[0].stream) return false;
    // batched plane kernels use the two-row x-pass only
    if (!chn::xpass_two_rows(3 * cfgs[i].n1 / 2, cfgs[i].precision == CHN_MIXED ? 8 : 16)) return false;
    const size_t b = layout(&cfgs[i], nullptr, nullptr);
    off = (off + 255) & ~(size_t)255;
    L->off.push_back(off);
    L->bytes.push_back(b);
    off += b;
    const int n1h = cfgs[i].n1 / 2, p3 = 3 * cfgs[i].n3 / 2;
    const size_t M = (size_t)n1h * cfgs[i].n3;
    items += (size_t)cfgs[i].n2 * (n1h + p3) + (2 * M + 255) / 256 + 1;
  }
  off = (off + 255) & ~(size_t)255;
  L->tables = off;
  L->total = off + (size_t)n * arg_bytes(cfgs[0].precision == CHN_MIXED) + 256 * 5 + items * sizeof(int4) * 2 +
             16 * (size_t)n + 4096;
  return true;
}

template <typename T> chn_status ens_build(chn_ens* e, char* tables) {
  const int n = e->n;
  // composite radices in a direction where they take fewer passes (the
  // channels' short lines: 48 = 8 x 6, 72 = 9 x 8, 96 = 12 x 8)
  e->comp = 0;
  for (chn_ctx* c : e->ctx) {
    int rs = 0;
    for (int d = 0; d < 2; ++d) {
      FftPlan pc{}, pk{};
      std::vector<double> t;
      const int n = d == 0 ? c->p1 : c->p3;
      if (chn::host::fft_plan(n, &pc, &t, chn::host::kRadixComposite) &&
          chn::host::fft_plan(n, &pk, &t, chn::host::kRadixClassic) && pc.npass < pk.npass)
        rs |= 1 << d;
    }
    if (rs && set_radix(c, rs) != CHN_OK) {
      e->err = "channel radix set: " + c->err;
      return CHN_EDEVICE;
    }
    if (rs) e->comp = 1;
  }
  // larger channels first: a static longest-processing-time order
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::sort(order.begin(), order.end(), [&](int a, int b) {
    const chn_ctx *A = e->ctx[a], *B = e->ctx[b];
    return (size_t)A->n2 * A->M > (size_t)B->n2 * B->M;
  });
  std::vector<chn::ZinvArgs<T>> za(n);
  std::vector<chn::XpassArgs<T>> xa(n);
  std::vector<chn::ZfwdArgs<T, T>> fa(n);
  std::vector<int4> wz, wx, wa;
  const int cb = (int)sizeof(typename Ty<T>::c);
  // rows per x-pass workgroup: the most (8, 4, 2) whose transforms every
  // channel holds in the smallest staging size (short rows fill workgroups)
  e->rz = 2;
  for (int rz : {8, 4}) {
    bool ok = true;
    for (int i = 0; i < n && ok; ++i) {
      const int m = chn::staging_for(e->ctx[i]->plan1, 3 * rz, cb);
      ok = m > 0 && m <= (cb == 8 ? 16 : 8) &&
           (size_t)3 * rz * plane_lds_stride(e->ctx[i]->p1) * cb <= (size_t)e->ctx[i]->lds_max;
    }
    if (ok) {
      e->rz = rz;
      break;
    }
  }
  e->lds_z = e->lds_x = 0;
  e->mz = e->mx = 0;
  // device placement of the tables
  char* p = tables;
  auto take = [&](size_t bytes) {
    char* q = p;
    p += (bytes + 255) & ~(size_t)255;
    return q;
  };
  // the channels' guards side by side, so one copy reads them all
  e->d_guard = reinterpret_cast<unsigned*>(take(16 * (size_t)n));
  for (int i = 0; i < n; ++i) e->ctx[i]->guard = e->d_guard + 4 * i;
  for (int i = 0; i < n; ++i) {
    chn_ctx* x = e->ctx[i];
    // one launch covers every channel, so no channel needs a workgroup
    // floor of its own: up to 16 z lines per workgroup
    x->zK = std::max(1, std::min(16, z_lines_max(x)));
    plane_args<T, T>(x, x->ph, false, x->H, za[i], xa[i], fa[i], x->guard);
    xa[i].rows = e->rz;
    const int mz = chn::staging_for(x->plan3, za[i].K, cb);
    const int mx = chn::staging_for(x->plan1, 3 * e->rz, cb);
    if (!mz || !mx) {
      e->err = "channel " + std::to_string(i) + ": transform staging does not fit";
      return CHN_EINVAL;
    }
    e->mz = std::max(e->mz, mz);
    e->mx = std::max(e->mx, mx);
    e->lds_z = std::max(e->lds_z, (size_t)za[i].K * za[i].lstride * cb);
    e->lds_x = std::max(e->lds_x, (size_t)3 * e->rz * xa[i].lstride * cb);
  }
  // Two groups of channels.  The pencil phase of a channel takes as long as
  // its n2-row chains, whatever the number of channels beside it, so when
  // the wall-normal sizes differ, group 0 holds the channels with the
  // longest lines and both groups start together: the other group's shorter
  // pencil phases and plane phases fill the time.  With one n2 for all,
  // channels are dealt to the groups in turn and group 1 starts one plane
  // phase later, so each group's pencil phase runs beside the other's plane
  // phase.
  int n2max = 0, n2min = 1 << 30;
  for (chn_ctx* c : e->ctx) {
    n2max = std::max(n2max, c->n2);
    n2min = std::min(n2min, c->n2);
  }
  e->lag = n2max == n2min;
  e->n2max = n2max;
  std::vector<int> grp(n);
  for (int k = 0; k < n; ++k) grp[order[k]] = e->lag ? k % 2 : (e->ctx[order[k]]->n2 == n2max ? 0 : 1);
  for (int g = 0; g < 2; ++g) {
    const size_t z0 = wz.size(), x0 = wx.size(), a0 = wa.size();
    for (int k = 0; k < n; ++k) {
      const int c = order[k];
      if (grp[c] != g) continue;
      chn_ctx* x = e->ctx[c];
      const int nbz = (x->n1h + za[c].K - 1) / za[c].K;
      for (int y = 0; y < x->n2; ++y)
        for (int b = 0; b < nbz; ++b) wz.push_back(make_int4(c, b, y, 0));
      for (int y = 0; y < x->n2; ++y)
        for (int b = 0; b < (x->p3 + e->rz - 1) / e->rz; ++b) wx.push_back(make_int4(c, b, y, 0));
      const int nb = chn::advance_blocks(x->M);
      wa.push_back(make_int4(c, 0, 0, 1));  // mean-mode workgroup
      for (int b = 0; b < nb; ++b) wa.push_back(make_int4(c, b, 0, 0));
    }
    e->gz[g] = (int)(wz.size() - z0);
    e->gx[g] = (int)(wx.size() - x0);
    e->ga[g] = (int)(wa.size() - a0);
  }
  e->d_zinv = take(sizeof(za[0]) * n);
  e->d_xpass = take(sizeof(xa[0]) * n);
  e->d_zfwd = take(sizeof(fa[0]) * n);
  e->d_adv = take(sizeof(chn::AdvanceArgs<T, T>) * 3 * n);
  e->d_wz = reinterpret_cast<int4*>(take(sizeof(int4) * wz.size()));
  e->d_wx = reinterpret_cast<int4*>(take(sizeof(int4) * wx.size()));
  e->d_wa = reinterpret_cast<int4*>(take(sizeof(int4) * wa.size()));
  e->nz = (int)wz.size();
  e->nx = (int)wx.size();
  e->na = (int)wa.size();
  hipError_t r = hipMemcpyAsync(e->d_zinv, za.data(), sizeof(za[0]) * n, hipMemcpyHostToDevice, e->user);
  if (r == hipSuccess) r = hipMemcpyAsync(e->d_xpass, xa.data(), sizeof(xa[0]) * n, hipMemcpyHostToDevice, e->user);
  if (r == hipSuccess) r = hipMemcpyAsync(e->d_zfwd, fa.data(), sizeof(fa[0]) * n, hipMemcpyHostToDevice, e->user);
  if (r == hipSuccess) r = hipMemcpyAsync(e->d_wz, wz.data(), sizeof(int4) * wz.size(), hipMemcpyHostToDevice, e->user);
  if (r == hipSuccess) r = hipMemcpyAsync(e->d_wx, wx.data(), sizeof(int4) * wx.size(), hipMemcpyHostToDevice, e->user);
  if (r == hipSuccess) r = hipMemcpyAsync(e->d_wa, wa.data(), sizeof(int4) * wa.size(), hipMemcpyHostToDevice, e->user);
  if (r == hipSuccess) r = hipMemsetAsync(e->d_guard, 0, 16 * (size_t)n, e->user);
  if (r == hipSuccess) r = hipStreamSynchronize(e->user);
  if (r != hipSuccess) {
    e->err = std::string("uploading ensemble tables: ") + hipGetErrorString(r);
    return CHN_EDEVICE;
  }
  e->h_adv.resize(sizeof(chn::AdvanceArgs<T, T>) * 3 * n);
  return CHN_OK;
}

#define ENSCHK(e, call)                                                        \
  do {                                                                         \
    hipError_t r_ = (call);                                                    \
    if (r_ != hipSuccess) {                                                    \
      (e)->err = std::string(#call ": ") + hipGetErrorString(r_);              \
      return CHN_EDEVICE;                                                      \
    }                                                                          \
  } while (0)

template <typename T> chn_status ens_step(chn_ens* e, const double* dt, int nsteps) {
  const int n = e->n;
  for (int i = 0; i < n; ++i) {
    chn_ctx* x = e->ctx[i];
    if (chn_status s = check(x)) {
      e->err = "channel " + std::to_string(i) + ": " + x->err;
      return s;
    }
    if (!x->have_state) {
      e->err = "channel " + std::to_string(i) + " has no state";
      return CHN_ESTATE;
    }
    if (!(dt[i] > 0)) {
      e->err = "dt must be positive";
      return CHN_EINVAL;
    }
    if (!x->phase_valid) {  // velocities/vorticities of a new state
      T* po[5];
      phase_ptrs<T>(x, po);
      if (chn_status s = recover<T>(x, po)) {
        e->err = x->err;
        return s;
      }
      x->phase_valid = true;
    }
  }
  // homogeneous solutions for these step sizes (outside the graph, on the configured stream)
  for (int i = 0; i < n; ++i)
    if (chn_status hs = homog_tables(e->ctx[i], dt[i], e->user)) {
      e->err = "channel " + std::to_string(i) + ": " + e->ctx[i]->err;
      return hs;
    }
  // advance argument blocks for these step sizes (the graph reads them from device memory)
  if (e->last_dt.size() != (size_t)n || !std::equal(e->last_dt.begin(), e->last_dt.end(), dt)) {
    auto* h = reinterpret_cast<chn::AdvanceArgs<T, T>*>(e->h_adv.data());
    for (int s = 0; s < 3; ++s)
      for (int i = 0; i < n; ++i) advance_args<T>(e->ctx[i], s, dt[i], h[s * n + i]);
    ENSCHK(e, hipMemcpyAsync(e->d_adv, e->h_adv.data(), e->h_adv.size(), hipMemcpyHostToDevice, e->user));
    e->last_dt.assign(dt, dt + n);
  }
  ENSCHK(e, hipMemsetAsync(e->d_guard, 0, 16 * (size_t)n, e->user));
  ENSCHK(e, hipEventRecord(e->ev_in, e->user));
  ENSCHK(e, hipStreamWaitEvent(e->own, e->ev_in, 0));
  chn::BatchPlan<T> bp{};
  bp.zinv = reinterpret_cast<const chn::ZinvArgs<T>*>(e->d_zinv);
  bp.xpass = reinterpret_cast<const chn::XpassArgs<T>*>(e->d_xpass);
  bp.zfwd = reinterpret_cast<const chn::ZfwdArgs<T, T>*>(e->d_zfwd);
  bp.wz = e->d_wz;
  bp.wx = e->d_wx;
  bp.nz = e->nz;
  bp.nx = e->nx;
  bp.lds_z = e->lds_z;
  bp.lds_x = e->lds_x;
  bp.mz = e->mz;
  bp.mx = e->mx;
  bp.rz = e->rz;
  bp.comp = e->comp;
  const auto* adv = reinterpret_cast<const chn::AdvanceArgs<T, T>*>(e->d_adv);
  // group g's work lists: a contiguous range of each list
  chn::BatchPlan<T> bg[2] = {bp, bp};
  bg[0].nz = e->gz[0];
  bg[0].nx = e->gx[0];
  bg[1].wz = e->d_wz + e->gz[0];
  bg[1].wx = e->d_wx + e->gx[0];
  bg[1].nz = e->gz[1];
  bg[1].nx = e->gx[1];
  const int4* wag[2] = {e->d_wa, e->d_wa + e->ga[0]};
  // One RK3 step: group 0 on the ensemble's stream, group 1 on a second
  // branch (from the start, or after group 0's first plane phase).
  auto one_step = [&]() -> hipError_t {
    hipError_t r = hipSuccess;
    const bool two = e->gz[1] > 0;
    if (two && !e->lag) {
      r = hipEventRecord(e->ev_lag, e->own);
      if (r == hipSuccess) r = hipStreamWaitEvent(e->own2, e->ev_lag, 0);
    }
    for (int s = 0; s < 3 && r == hipSuccess; ++s) {
      r = chn::launch_plane_batch<T>(bg[0], e->own);
      if (r == hipSuccess && s == 0 && two && e->lag) r = hipEventRecord(e->ev_lag, e->own);
      if (r == hipSuccess && s == 0 && two && e->lag) r = hipStreamWaitEvent(e->own2, e->ev_lag, 0);
      if (r == hipSuccess) r = chn::launch_advance_batch<T>(adv + s * n, wag[0], e->ga[0], e->n2max, e->own);
    }
    for (int s = 0; s < 3 && r == hipSuccess && two; ++s) {
      r = chn::launch_plane_batch<T>(bg[1], e->own2);
      if (r == hipSuccess) r = chn::launch_advance_batch<T>(adv + s * n, wag[1], e->ga[1], e->n2max, e->own2);
    }
    if (r == hipSuccess && two) r = hipEventRecord(e->ev_join, e->own2);
    if (r == hipSuccess && two) r = hipStreamWaitEvent(e->own, e->ev_join, 0);
    return r;
  };
  if (!e->exec) {  // capture one RK3 step of the whole ensemble once
    ENSCHK(e, hipStreamBeginCapture(e->own, hipStreamCaptureModeThreadLocal));
    const hipError_t r = one_step();
    hipGraph_t g = nullptr;
    const hipError_t r2 = hipStreamEndCapture(e->own, &g);
    if (r != hipSuccess || r2 != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      e->err = std::string("capturing the ensemble step: ") + hipGetErrorString(r != hipSuccess ? r : r2);
      return CHN_EDEVICE;
    }
    e->graph = g;
    ENSCHK(e, hipGraphInstantiate(&e->exec, e->graph, nullptr, nullptr, 0));
  }
  for (int k = 0; k < nsteps; ++k) ENSCHK(e, hipGraphLaunch(e->exec, e->own));
  ENSCHK(e, hipEventRecord(e->ev_out, e->own));
  ENSCHK(e, hipStreamWaitEvent(e->user, e->ev_out, 0));
  std::vector<unsigned> gw(4 * (size_t)n);
  ENSCHK(e, hipMemcpyAsync(gw.data(), e->d_guard, 16 * (size_t)n, hipMemcpyDeviceToHost, e->user));
  ENSCHK(e, hipStreamSynchronize(e->user));
  for (int i = 0; i < n; ++i)
    if (gw[4 * i + 1]) {
      const unsigned c = gw[4 * i + 1] - 1;
      e->err = "channel " + std::to_string(i) + ": step " + std::to_string(c / 3) + ", sub-step " +
               std::to_string(c % 3) + ": CFL not finite or above the limit; that channel's state is as at the "
               "start of that sub-step";
      return CHN_EUNSTABLE;
    }
  return CHN_OK;
}

}  // namespace

extern "C" {

size_t chn_workspace_bytes(const chn_config* cfg) {
  if (validate(cfg)) return 0;
  return layout(cfg, nullptr, nullptr);
}

chn_status chn_create(const chn_config* cfg, void* d_ws, size_t ws_bytes, chn_ctx** out) {
  if (!out) return fail(nullptr, CHN_EINVAL, "out is NULL");
  *out = nullptr;
  if (const char* m = validate(cfg)) return fail(nullptr, CHN_EINVAL, m);
  const size_t need = layout(cfg, nullptr, nullptr);
  if (!d_ws || ws_bytes < need) return fail(nullptr, CHN_EINVAL, "workspace missing or smaller than chn_workspace_bytes");
  if (reinterpret_cast<uintptr_t>(d_ws) % 256) return fail(nullptr, CHN_EINVAL, "workspace must be 256-byte aligned");
  chn_ctx* x = new chn_ctx();
  x->cfg = *cfg;
  x->stream = reinterpret_cast<hipStream_t>(cfg->stream);
  x->n1 = cfg->n1; x->n2 = cfg->n2; x->n3 = cfg->n3;
  x->n1h = cfg->n1 / 2; x->M = x->n1h * x->n3;
  x->p1 = 3 * cfg->n1 / 2; x->p3 = 3 * cfg->n3 / 2;
  x->nu = 1.0 / cfg->re_b;
  x->mixed = cfg->precision == CHN_MIXED;
  x->planes_only = cfg->planes_only != 0;
  x->ychunk_max = x->planes_only ? cfg->plane_chunk : x->n2;
  x->ws_bytes = ws_bytes;
  layout(cfg, reinterpret_cast<char*>(d_ws), x);
  {
    int dev = 0, lds = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) == hipSuccess && lds > 0)
      x->lds_max = lds;
  }
  x->y.resize(x->n2);
  if (cfg->y) std::memcpy(x->y.data(), cfg->y, sizeof(double) * x->n2);
  else chn::host::default_mesh(x->n2, x->y.data());
  x->cfg.y = nullptr;
  const int n2 = x->n2;
  // The banded LUs are unpivoted; refuse meshes on which the compact
  // operators are close to singular (the maximum-order stencils degenerate
  // for some local stretchings, Appendix B).  A plane-phase context uses the
  // mesh for the CFL number only.
  if (!x->planes_only) {
    double c1 = INFINITY, c2 = INFINITY;
    const bool ok = chn::host::operator_conditioning(n2, x->y.data(), &c1, &c2);
    if (!ok || !(c1 <= kCondMax) || !(c2 <= kCondMax)) {
      char msg[200];
      std::snprintf(msg, sizeof(msg),
                    "compact operators ill-conditioned on this mesh: cond_1(A1) = %.3g, cond_1(A2 with Dirichlet "
                    "rows) = %.3g, bound %.0e (a milder wall stretching helps)", c1, c2, kCondMax);
      delete x;
      return fail(nullptr, CHN_EINVAL, msg);
    }
  }
  // tables
  x->hA1.resize(7 * n2); x->hB1.resize(7 * n2); x->hA2.resize(7 * n2); x->hB2.resize(7 * n2);
  x->hquad.resize(n2);
  std::vector<double> L1d(3 * n2), U1d(4 * n2), L1u(3 * n2), U1u(4 * n2), L2d(3 * n2), U2d(4 * n2);
  std::vector<double> clo(n2), chw(n2), idy(n2);
  bool ok = chn::host::compact_bands(n2, x->y.data(), 1, x->hA1.data(), x->hB1.data()) &&
            chn::host::compact_bands(n2, x->y.data(), 2, x->hA2.data(), x->hB2.data()) &&
            chn::host::band_lu(n2, x->hA1.data(), +1, L1d.data(), U1d.data()) &&
            chn::host::band_lu(n2, x->hA1.data(), -1, L1u.data(), U1u.data()) &&
            chn::host::band_lu(n2, x->hA2.data(), +1, L2d.data(), U2d.data()) &&
            chn::host::wall_rows(n2, x->hA1.data(), x->hB1.data(), clo.data(), chw.data());
  if (!ok && !x->planes_only) {  // a plane-phase context uses the mesh for the CFL only
    delete x;
    return fail(nullptr, CHN_EINVAL, "compact-difference system singular on this mesh");
  }
  chn::host::quadrature(n2, x->y.data(), x->hquad.data());
  for (int j = 0; j < n2; ++j) {
    const double lo = j > 0 ? x->y[j] - x->y[j - 1] : x->y[1] - x->y[0];
    const double hi = j < n2 - 1 ? x->y[j + 1] - x->y[j] : lo;
    idy[j] = 1.0 / (lo < hi ? lo : hi);
  }
  std::vector<double> tw1, tw3;
  if (!chn::host::fft_plan(x->p1, &x->plan1, &tw1) || !chn::host::fft_plan(x->p3, &x->plan3, &tw3)) {
    delete x;
    return fail(nullptr, CHN_EINVAL, "FFT length not supported");
  }
  default_plan(x);
  if (!plan_fits(x, x->xrows, x->zK, x->ychunk)) {
    delete x;
    return fail(nullptr, CHN_EINVAL, "plane too large for the x- or z-pass LDS tiles on this device");
  }
  auto up = [&](double* d, const std::vector<double>& h) {
    return hipMemcpyAsync(d, h.data(), h.size() * sizeof(double), hipMemcpyHostToDevice, x->stream);
  };
  hipError_t e = hipSuccess;
  std::vector<double> f1, f3;
  std::vector<float> g1, g3;
  if (e == hipSuccess) e = up(x->A1, x->hA1);
  if (e == hipSuccess) e = up(x->B1, x->hB1);
  if (e == hipSuccess) e = up(x->A2, x->hA2);
  if (e == hipSuccess) e = up(x->B2, x->hB2);
  if (e == hipSuccess) e = up(x->L1d, L1d);
  if (e == hipSuccess) e = up(x->U1d, U1d);
  if (e == hipSuccess) e = up(x->L1u, L1u);
  if (e == hipSuccess) e = up(x->U1u, U1u);
  if (e == hipSuccess) e = up(x->L2d, L2d);
  if (e == hipSuccess) e = up(x->U2d, U2d);
  if (e == hipSuccess) e = up(x->clo, clo);
  if (e == hipSuccess) e = up(x->chi_w, chw);
  if (e == hipSuccess) e = up(x->quad, x->hquad);
  if (e == hipSuccess) e = up(x->inv_dy, idy);
  if (x->mixed) {
    g1.assign(tw1.begin(), tw1.end());
    g3.assign(tw3.begin(), tw3.end());
    if (e == hipSuccess) e = hipMemcpyAsync(x->tw1, g1.data(), g1.size() * 4, hipMemcpyHostToDevice, x->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(x->tw3, g3.data(), g3.size() * 4, hipMemcpyHostToDevice, x->stream);
  } else {
    if (e == hipSuccess) e = hipMemcpyAsync(x->tw1, tw1.data(), tw1.size() * 8, hipMemcpyHostToDevice, x->stream);
    if (e == hipSuccess) e = hipMemcpyAsync(x->tw3, tw3.data(), tw3.size() * 8, hipMemcpyHostToDevice, x->stream);
  }
  if (e == hipSuccess) e = hipMemcpyAsync(x->tw1d, tw1.data(), tw1.size() * 8, hipMemcpyHostToDevice, x->stream);
  if (e == hipSuccess) e = hipMemcpyAsync(x->tw3d, tw3.data(), tw3.size() * 8, hipMemcpyHostToDevice, x->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(x->stream);
  if (e != hipSuccess) {
    delete x;
    return fail(nullptr, CHN_EDEVICE, std::string("uploading tables: ") + hipGetErrorString(e));
  }
  chn::PencilGeom& g = x->geom;
  g.n2 = n2; g.n3 = x->n3; g.n1h = x->n1h; g.M = x->M;
  g.ka = 2.0 * M_PI / cfg->lx; g.kb = 2.0 * M_PI / cfg->lz;
  g.A1 = x->A1; g.B1 = x->B1; g.A2 = x->A2; g.B2 = x->B2;
  g.L1d = x->L1d; g.U1d = x->U1d; g.L1u = x->L1u; g.U1u = x->U1u; g.L2d = x->L2d; g.U2d = x->U2d;
  g.clo = x->clo; g.chi = x->chi_w; g.quad = x->quad;
  chn::PlaneDims& d = x->dims;
  d.n1h = x->n1h; d.n2 = n2; d.n3 = x->n3; d.p1 = x->p1; d.p3 = x->p3; d.lx = cfg->lx; d.lz = cfg->lz;
  *out = x;
  return CHN_OK;
}

chn_status chn_destroy(chn_ctx* ctx) {
  delete ctx;
  return CHN_OK;
}

chn_status chn_set_state(chn_ctx* x, const double* d_v, const double* d_om2, const double* d_u1m,
                         const double* d_u3m) {
  if (chn_status s = check(x)) return s;
  if (chn_status s = need_fields(x)) return s;
  if (!d_v || !d_om2 || !d_u1m || !d_u3m) return fail(x, CHN_EINVAL, "NULL state pointer");
  chn::ChiArgs ca{};
  ca.g = x->geom;
  ca.vin = d_v;
  ca.omin = d_om2;
  ca.v = x->v;
  ca.om2 = x->om2;
  ca.chi = x->chi;
  ca.S0 = x->S[0];
  HIPCHK(x, chn::launch_chi_from_v(ca, x->stream));
  const size_t n2b = sizeof(double) * x->n2;
  HIPCHK(x, hipMemcpyAsync(x->U1, d_u1m, n2b, hipMemcpyDeviceToDevice, x->stream));
  HIPCHK(x, hipMemcpyAsync(x->U3, d_u3m, n2b, hipMemcpyDeviceToDevice, x->stream));
  const size_t CB = 16 * (size_t)x->n2 * x->M;
  HIPCHK(x, hipMemsetAsync(x->nchi_old, 0, CB, x->stream));
  HIPCHK(x, hipMemsetAsync(x->nom_old, 0, CB, x->stream));
  HIPCHK(x, hipMemsetAsync(x->nu_old, 0, n2b, x->stream));
  HIPCHK(x, hipMemsetAsync(x->nw_old, 0, n2b, x->stream));
  HIPCHK(x, hipMemsetAsync(x->guard, 0, 4 * sizeof(unsigned), x->stream));
  x->have_state = true;
  x->phase_valid = false;
  return CHN_OK;
}

namespace {
chn_status step_eager(chn_ctx* x, double dt) {
  for (int s = 0; s < 3; ++s)
    if (chn_status st = x->mixed ? substep<float>(x, s, dt) : substep<double>(x, s, dt)) return st;
  return CHN_OK;
}

// The graph of one step for dt and the current schedule, captured on the
// context's capture stream (kernel launches only: the tables of dt and the
// phase fields are current, so the step makes no other call).
chn_status step_graph(chn_ctx* x, double dt) {
  const std::vector<double> key = {dt, (double)x->xrows, (double)x->zK, (double)x->ychunk, (double)x->ffix,
                                   (double)x->zpipe, (double)x->radix};
  if (x->gexec && x->graph_key == key) return CHN_OK;
  x->drop_graph();
  if (!x->cap) HIPCHK(x, hipStreamCreate(&x->cap));
  hipStream_t user = x->stream;
  x->stream = x->cap;
  hipError_t e = hipStreamBeginCapture(x->cap, hipStreamCaptureModeThreadLocal);
  chn_status st = e == hipSuccess ? step_eager(x, dt) : CHN_OK;
  hipGraph_t g = nullptr;
  const hipError_t e2 = e == hipSuccess ? hipStreamEndCapture(x->cap, &g) : e;
  x->stream = user;
  if (st != CHN_OK) {
    if (g) (void)hipGraphDestroy(g);
    return st;
  }
  if (e2 != hipSuccess) return fail(x, CHN_EDEVICE, std::string("capturing the step: ") + hipGetErrorString(e2));
  x->graph = g;
  HIPCHK(x, hipGraphInstantiate(&x->gexec, g, nullptr, nullptr, 0));
  x->graph_key = key;
  return CHN_OK;
}
}  // namespace

chn_status chn_step_graph_enable(chn_ctx* x, int32_t enable) {
  if (chn_status s = check(x)) return s;
  x->use_graph = enable != 0;
  if (!x->use_graph) x->drop_graph();
  return CHN_OK;
}

chn_status chn_step_rk3(chn_ctx* x, double dt, int32_t nsteps, chn_step_info* info) {
  if (chn_status s = check(x)) return s;
  if (chn_status s = need_fields(x)) return s;
  if (!x->have_state) return fail(x, CHN_ESTATE, "chn_step_rk3 before chn_set_state");
  if (!(dt > 0) || nsteps < 0) return fail(x, CHN_EINVAL, "dt must be positive and nsteps >= 0");
  // the guard's CFL word, fail code and step count start from zero
  HIPCHK(x, hipMemsetAsync(x->guard, 0, 4 * sizeof(unsigned), x->stream));
  const size_t pool_mark = x->pool_used;
  // steps replayed from the graph: those after the tables of dt and the
  // phase fields are current, before the last step when info asks for its
  // per-phase times; never while per-kernel events are recorded
  const bool graph_ok = x->use_graph && !x->timing;
  for (int k = 0; k < nsteps; ++k) {
    const bool last_rec = info && k == nsteps - 1;
    if (last_rec) {  // per-phase times of the last step
      x->phase_rec = true;
      x->phase_timed.clear();
    }
    chn_status st = CHN_OK;
    if (graph_ok && !last_rec && x->phase_valid && x->htab_dt == dt) {
      st = step_graph(x, dt);
      if (st == CHN_OK) HIPCHK(x, hipGraphLaunch(x->gexec, x->stream));
    } else {
      st = step_eager(x, dt);
    }
    if (st != CHN_OK) {
      x->phase_rec = false;
      return st;
    }
  }
  x->phase_rec = false;
  if (info) {
    double* div = x->info_dev + 6;
    HIPCHK(x, hipMemsetAsync(div, 0, sizeof(double), x->stream));
    const chn_status ds = x->mixed ? divergence<float>(x, reinterpret_cast<unsigned long long*>(div))
                                   : divergence<double>(x, reinterpret_cast<unsigned long long*>(div));
    if (ds != CHN_OK) return ds;
    chn::InfoArgs ia{};
    ia.g = x->geom;
    ia.rowcfl = x->rowcfl;
    ia.p3 = x->p3;
    ia.U1 = x->U1;
    ia.dt = dt;
    ia.nu = x->nu;
    ia.out = x->info_dev;
    ia.mean_out = x->mean_out;
    HIPCHK(x, chn::launch_info(ia, x->stream));
  }
  double h[8] = {0};
  unsigned gw[4] = {0, 0, 0, 0};
  if (info) HIPCHK(x, hipMemcpyAsync(h, x->info_dev, sizeof(h), hipMemcpyDeviceToHost, x->stream));
  HIPCHK(x, hipMemcpyAsync(gw, x->guard, sizeof(gw), hipMemcpyDeviceToHost, x->stream));
  HIPCHK(x, hipStreamSynchronize(x->stream));
  const int fstep = gw[1] ? (int)((gw[1] - 1) / 3) : -1, fsub = gw[1] ? (int)((gw[1] - 1) % 3) : -1;
  if (info) {
    info->cfl_max = h[0];
    info->mass_flux = h[1];
    info->utau_lo = h[2];
    info->utau_hi = h[3];
    info->f_mean = h[4];
    info->max_abs_div = h[6];
    for (int p = 0; p < 5; ++p) info->ms_phase[p] = 0.0f;
    for (const auto& r : x->phase_timed) {
      float ms = 0.0f;
      HIPCHK(x, hipEventElapsedTime(&ms, r.a, r.b));
      const int ph = r.kind == CHN_K_ZINV ? 0 : r.kind == CHN_K_XPASS ? 1 : r.kind == CHN_K_ZFWD ? 2
                   : r.kind == CHN_K_ADVANCE ? 3 : 4;
      info->ms_phase[ph] += ms;
    }
    info->fail_step = fstep;
    info->fail_substep = fsub;
    if (fstep >= 0) info->cfl_max = (double)reinterpret_cast<const float&>(gw[0]) * dt;
  }
  x->phase_timed.clear();
  if (!x->timing) x->pool_used = pool_mark;  // the last step's events are free again
  if (fstep >= 0) {
    const float c = reinterpret_cast<const float&>(gw[0]);
    char msg[160];
    std::snprintf(msg, sizeof(msg), "step %d, sub-step %d: CFL %.4g %s; the state is as at the start of that sub-step",
                  fstep, fsub, (double)c * dt, std::isfinite(c) ? "above the limit" : "not finite");
    return fail(x, CHN_EUNSTABLE, msg);
  }
  if (info && (h[5] != 0.0 || !std::isfinite(h[0]))) return fail(x, CHN_EUNSTABLE, "non-finite values after the step");
  return CHN_OK;
}

chn_status chn_get_fields(chn_ctx* x, uint32_t mask, double* const* d_out) {
  if (chn_status s = check(x)) return s;
  if (!x->have_state) return fail(x, CHN_ESTATE, "chn_get_fields before chn_set_state");
  if (!d_out && mask) return fail(x, CHN_EINVAL, "d_out is NULL");
  const size_t CB = 16 * (size_t)x->n2 * x->M;
  const size_t n2b = sizeof(double) * x->n2;
  const bool need_rec = mask & (CHN_F_U1 | CHN_F_U3 | CHN_F_OMEGA1 | CHN_F_OMEGA3);
  if (need_rec) {
    double* po[5] = {x->S[3], x->S[4], x->S[5], x->S[6], x->S[7]};
    x->htab_dt = 0.0;  // overwrites the factor tables of sub-steps 1 and 2
    if (chn_status s = recover<double>(x, po)) return s;
  }
  int k = 0;
  for (uint32_t bit = 0; bit < 9; ++bit) {
    if (!(mask & (1u << bit))) continue;
    double* dst = d_out[k++];
    if (!dst) return fail(x, CHN_EINVAL, "NULL output pointer");
    const void* src = nullptr;
    size_t bytes = CB;
    switch (1u << bit) {
      case CHN_F_V: src = x->v; break;
      case CHN_F_OMEGA2: src = x->om2; break;
      case CHN_F_CHI: src = x->chi; break;
      case CHN_F_U1: src = x->S[3]; break;
      case CHN_F_U3: src = x->S[5]; break;
      case CHN_F_OMEGA1: src = x->S[6]; break;
      case CHN_F_OMEGA3: src = x->S[7]; break;
      case CHN_F_U1MEAN: src = x->U1; bytes = n2b; break;
      case CHN_F_U3MEAN: src = x->U3; bytes = n2b; break;
    }
    HIPCHK(x, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, x->stream));
  }
  return CHN_OK;
}

chn_status chn_nonlinear(chn_ctx* x, const double* const* d_in, double* const* d_out) {
  if (chn_status s = check(x)) return s;
  if (chn_status s = need_fields(x)) return s;
  if (!d_in || !d_out) return fail(x, CHN_EINVAL, "NULL field array");
  for (int f = 0; f < 6; ++f)
    if (!d_in[f]) return fail(x, CHN_EINVAL, "NULL input field");
  for (int f = 0; f < 3; ++f)
    if (!d_out[f]) return fail(x, CHN_EINVAL, "NULL output field");
  if (!x->mixed) {
    const void* in[6];
    void* out[3];
    for (int f = 0; f < 6; ++f) in[f] = d_in[f];
    for (int f = 0; f < 3; ++f) out[f] = d_out[f];
    return plane_phase<double, double>(x, in, true, out);
  }
  const size_t n = 2 * (size_t)x->n2 * x->M;
  x->phase_valid = false;  // the phase buffers now hold the caller's fields
  for (int f = 0; f < 6; ++f)
    HIPCHK(x, chn::launch_convert_d2f(d_in[f], reinterpret_cast<float*>(x->ph[f]), n, x->stream));
  void* out[3];
  for (int f = 0; f < 3; ++f) out[f] = d_out[f];
  return plane_phase<float, double>(x, x->ph, true, out);
}

chn_status chn_plane_products(chn_ctx* x, const void* const* d_in, void* const* d_out) {
  if (chn_status s = check(x)) return s;
  if (!d_in || !d_out) return fail(x, CHN_EINVAL, "NULL field array");
  for (int f = 0; f < 6; ++f)
    if (!d_in[f] && f != 4) return fail(x, CHN_EINVAL, "NULL input field");
  for (int f = 0; f < 3; ++f)
    if (!d_out[f]) return fail(x, CHN_EINVAL, "NULL output field");
  const void* in[6];
  void* out[3];
  for (int f = 0; f < 6; ++f) in[f] = d_in[f];
  for (int f = 0; f < 3; ++f) out[f] = d_out[f];
  const bool om2 = d_in[4] != nullptr;
  return x->mixed ? plane_phase<float, float>(x, in, om2, out) : plane_phase<double, double>(x, in, om2, out);
}

chn_status chn_plane_products_static(chn_ctx* x, const void* const* d_in, void* const* d_out) {
  if (chn_status s = check(x)) return s;
  if (!d_in || !d_out) return fail(x, CHN_EINVAL, "NULL field array");
  for (int f = 0; f < 6; ++f)
    if (!d_in[f] && f != 4) return fail(x, CHN_EINVAL, "NULL input field");
  for (int f = 0; f < 3; ++f)
    if (!d_out[f]) return fail(x, CHN_EINVAL, "NULL output field");
  // one plane of the intermediate: six z-padded fields of n1/2 lines
  const size_t plane = (size_t)6 * x->p3 * x->n1h * (x->mixed ? 8 : 16);
  if (plane > kStaticScratchBytes)
    return fail(x, CHN_EUNSUPPORTED, "one plane of the transform intermediate (" + std::to_string(plane) +
                                         " bytes) exceeds the static scratch of " +
                                         std::to_string(kStaticScratchBytes) + " bytes");
  void* scr = nullptr;
  if (chn_status s = static_scratch(x, &scr)) return s;
  const int chunk = (int)std::min<size_t>((size_t)x->n2, kStaticScratchBytes / plane);
  const void* in[6];
  void* out[3];
  for (int f = 0; f < 6; ++f) in[f] = d_in[f];
  for (int f = 0; f < 3; ++f) out[f] = d_out[f];
  const bool om2 = d_in[4] != nullptr;
  // no timing events either: their creation is left to the allocating entry points
  const bool timing = x->timing, rec = x->phase_rec;
  x->timing = x->phase_rec = false;
  const chn_status st = x->mixed ? plane_phase<float, float>(x, in, om2, out, nullptr, scr, chunk)
                                 : plane_phase<double, double>(x, in, om2, out, nullptr, scr, chunk);
  x->timing = timing;
  x->phase_rec = rec;
  return st;
}

chn_status chn_filter_and_stress(chn_ctx* x, int32_t kcx, int32_t kcz, int32_t q1, int32_t q3, double* d_ubar,
                                 double* d_uubar, double* d_tau) {
  if (chn_status s = check(x)) return s;
  if (!x->have_state) return fail(x, CHN_ESTATE, "chn_filter_and_stress before chn_set_state");
  return filter_stage(x, kcx, kcz, q1, q3, d_ubar, d_uubar, d_tau);
}

extern "C++" {
namespace {
template <typename T> chn_status stats_stage(chn_ctx* x, double* d_spec, double* d_mean) {
  T* po[5];
  phase_ptrs<T>(x, po);
  if (!x->phase_valid) {  // the velocities of a new state (after a step they are current)
    if (chn_status st = recover<T>(x, po)) return st;
    x->phase_valid = true;
  }
  chn::StatsArgs<T> a{};
  for (int i = 0; i < 3; ++i) a.u[i] = reinterpret_cast<const typename Ty<T>::c*>(po[i]);
  a.spec = d_spec;
  a.mean = d_mean;
  a.U1 = x->U1;
  a.U3 = x->U3;
  a.M = x->M;
  a.NP = (size_t)x->n2 * x->M;
  a.n2 = x->n2;
  HIPCHK(x, timed(x, CHN_K_FILTER, [&] { return chn::launch_stats<T>(a, x->stream); }));
  return CHN_OK;
}
}  // namespace
}  // extern "C++"

chn_status chn_accumulate_statistics(chn_ctx* x, double* d_spec, double* d_mean) {
  if (chn_status s = check(x)) return s;
  if (chn_status s = need_fields(x)) return s;
  if (!x->have_state) return fail(x, CHN_ESTATE, "chn_accumulate_statistics before chn_set_state");
  if (!d_spec || !d_mean) return fail(x, CHN_EINVAL, "NULL output pointer");
  return x->mixed ? stats_stage<float>(x, d_spec, d_mean) : stats_stage<double>(x, d_spec, d_mean);
}

chn_status chn_filtered_pressure(chn_ctx* x, int32_t kcx, int32_t kcz, const double* d_uubar, const double* d_ubar,
                                 double* d_p) {
  if (chn_status s = check(x)) return s;
  if (chn_status s = need_fields(x)) return s;
  if (!d_uubar || !d_ubar || !d_p) return fail(x, CHN_EINVAL, "NULL pointer");
  if (kcx < 0 || kcz < 0 || kcx >= x->n1h || kcz >= x->n3 / 2)
    return fail(x, CHN_EINVAL, "need 0 <= kcx < n1/2, 0 <= kcz < n3/2");
  const size_t R = (size_t)(kcx + 1) * (2 * kcz + 1);  // <= M: the scratch below always fits
  chn::PressureArgs a{};
  a.g = x->geom;
  a.uu = d_uubar;
  a.vb = d_ubar + 2 * (size_t)x->n2 * R;  // F(u_2)
  a.p = d_p;
  a.T[0] = x->S[0];
  a.T[1] = x->S[1];
  a.T[2] = x->S[2];
  a.T[3] = x->S[5];
  for (int k = 0; k < 4; ++k) a.Q[k] = reinterpret_cast<double*>(x->inter) + k * (size_t)x->n2 * R;
  a.R = (int)R;
  a.nz = 2 * kcz + 1;
  a.kcz = kcz;
  a.nu = x->nu;
  HIPCHK(x, timed(x, CHN_K_FILTER, [&] { return chn::launch_pressure(a, x->stream); }));
  return CHN_OK;
}

chn_status chn_filtered_enstrophy(chn_ctx* x, int32_t kcx, int32_t kcz, double* d_out) {
  if (chn_status s = check(x)) return s;
  if (chn_status s = need_fields(x)) return s;
  if (!x->have_state) return fail(x, CHN_ESTATE, "chn_filtered_enstrophy before chn_set_state");
  if (!d_out) return fail(x, CHN_EINVAL, "NULL output pointer");
  return filter_stage(x, kcx, kcz, 0, 0, nullptr, nullptr, nullptr, d_out);
}

chn_status chn_get_operators(chn_ctx* x, double* a1, double* b1, double* a2, double* b2, double* quad) {
  if (!x) return CHN_EINVAL;
  const size_t nb = sizeof(double) * 7 * x->n2;
  if (a1) std::memcpy(a1, x->hA1.data(), nb);
  if (b1) std::memcpy(b1, x->hB1.data(), nb);
  if (a2) std::memcpy(a2, x->hA2.data(), nb);
  if (b2) std::memcpy(b2, x->hB2.data(), nb);
  if (quad) std::memcpy(quad, x->hquad.data(), sizeof(double) * x->n2);
  return CHN_OK;
}

chn_status chn_get_mesh(chn_ctx* x, double* y) {
  if (!x) return CHN_EINVAL;
  if (!y) return fail(x, CHN_EINVAL, "y is NULL");
  std::memcpy(y, x->y.data(), sizeof(double) * x->n2);
  return CHN_OK;
}

chn_status chn_get_plan(chn_ctx* x, chn_plan* plan) {
  if (!x || !plan) return CHN_EINVAL;
  plan->x_rows = x->xrows;
  plan->z_lines = x->zK;
  plan->y_chunk = x->ychunk;
  plan->fixed_radix = x->ffix;
  plan->z_pipeline = x->zpipe;
  plan->radix_set = x->radix;
  return CHN_OK;
}

chn_status chn_set_plan(chn_ctx* x, const chn_plan* plan) {
  if (chn_status s = check(x)) return s;
  if (!plan || (plan->fixed_radix != 0 && plan->fixed_radix != 1) || (plan->z_pipeline != 0 && plan->z_pipeline != 1) ||
      plan->radix_set < 0 || plan->radix_set > 3)
    return fail(x, CHN_EINVAL, "schedule fields out of range");
  const int old = x->radix;
  if (chn_status s = set_radix(x, plan->radix_set)) return s;
  if (!plan_fits(x, plan->x_rows, plan->z_lines, plan->y_chunk)) {
    if (chn_status s = set_radix(x, old)) return s;
    return fail(x, CHN_EINVAL, "schedule does not fit this grid or the device's LDS");
  }
  x->xrows = plan->x_rows;
  x->zK = plan->z_lines;
  x->ychunk = plan->y_chunk;
  x->ffix = plan->fixed_radix;
  x->zpipe = plan->z_pipeline;
  return CHN_OK;
}

namespace {
// Autotuner cache: one JSON object per line, {"key": "...", "plan": [x_rows,
// z_lines, y_chunk, fixed_radix, z_pipeline, radix_set]}; the last line of a
// key wins.
std::string tune_path() {
  if (const char* e = std::getenv("CHN_TUNE_CACHE")) return e;
  if (const char* d = std::getenv("XDG_CACHE_HOME"); d && *d) return std::string(d) + "/chn_tune.jsonl";
  if (const char* h = std::getenv("HOME"); h && *h) return std::string(h) + "/.cache/chn_tune.jsonl";
  return "";
}
std::string tune_key(const chn_ctx* x) {
  int dev = 0;
  hipDeviceProp_t pr{};
  std::string arch = "unknown";
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&pr, dev) == hipSuccess) arch = pr.gcnArchName;
  return arch + "/" + std::to_string(x->n1) + "x" + std::to_string(x->n2) + "x" + std::to_string(x->n3) + "/" +
         (x->mixed ? "mixed" : "fp64") + "/planes" + std::to_string(x->ychunk_max);
}
bool tune_lookup(const std::string& path, const std::string& key, chn_plan* p) {
  if (path.empty()) return false;
  FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  const std::string tag = "\"key\": \"" + key + "\"";
  char line[1024];
  bool found = false;
  while (std::fgets(line, sizeof line, f)) {
    const char* k = std::strstr(line, tag.c_str());
    const char* q = std::strstr(line, "\"plan\": [");
    if (!k || !q) continue;
    chn_plan t{};
    if (std::sscanf(q + 9, "%d , %d , %d , %d , %d , %d", &t.x_rows, &t.z_lines, &t.y_chunk, &t.fixed_radix,
                    &t.z_pipeline, &t.radix_set) == 6) {
      *p = t;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}
void tune_store(const std::string& path, const std::string& key, const chn_plan& p) {
  if (path.empty()) return;
  FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "{\"key\": \"%s\", \"plan\": [%d, %d, %d, %d, %d, %d]}\n", key.c_str(), p.x_rows, p.z_lines,
               p.y_chunk, p.fixed_radix, p.z_pipeline, p.radix_set);
  std::fclose(f);
}
}  // namespace

chn_status chn_autotune(chn_ctx* x, int32_t reps, chn_plan* chosen) {
  if (chn_status s = check(x)) return s;
  if (x->planes_only) return fail(x, CHN_EUNSUPPORTED, "autotune needs the context's own field buffers (not planes_only)");
  if (reps < 1) reps = 3;
  const std::string path = tune_path(), key = tune_key(x);
  {
    chn_plan c{};
    if (tune_lookup(path, key, &c)) {
      chn_plan prev{};
      chn_get_plan(x, &prev);
      if (chn_set_plan(x, &c) == CHN_OK) {
        if (chosen) *chosen = c;
        return CHN_OK;
      }
      x->err.clear();  // a stale entry: tune again
      if (chn_status s = chn_set_plan(x, &prev)) return s;
    }
  }
  struct Cand { int xr, K, ych, fx, zp, rs; };
  std::vector<Cand> cand;
  // planes per launch: the largest, and even splits of the planes into 2..12 launches
  std::vector<int> chunks;
  for (int parts : {1, 2, 4, 8, 12}) {
    const int c = std::min(x->ychunk_max, (x->n2 + parts - 1) / parts);
    if (c >= 1 && std::find(chunks.begin(), chunks.end(), c) == chunks.end()) chunks.push_back(c);
  }
  // the pipelined z passes engage where a field of K lines fits their staging
  // registers (8 values per thread inverse, 12 forward, 256 threads)
  auto pipe_engages = [&](int K) { return K * x->n3 <= 8 * 256 || K * x->p3 <= 12 * 256; };
  // candidates of radix sets rs over the planes per launch in ychs
  auto add = [&](int rs, const std::vector<int>& ychs) {
    if (set_radix(x, rs) != CHN_OK) {
      x->err.clear();
      return;
    }
    const int kmax = z_lines_max(x);
    const bool has_fixed = chn::plan_is_576(x->plan1) || chn::plan_is_576(x->plan3) || chn::plan_is_576c(x->plan1) ||
                           chn::plan_is_576c(x->plan3) || chn::plan_is_9216(x->plan3) || chn::plan_is_12288(x->plan1);
    for (int zp = 0; zp <= 1; ++zp)
      for (int fx = 0; fx <= (has_fixed ? 1 : 0); ++fx)
        for (int xr : {8, 4, 2, 1})
          for (int K : {1, 2, 4, 8, 12, 16, kmax})
            for (int c : ychs)
              if (plan_fits(x, xr, K, c) && (zp == 0 || pipe_engages(K)) &&
                  std::none_of(cand.begin(), cand.end(), [&](const Cand& q) {
                    return q.xr == xr && q.K == K && q.ych == c && q.fx == fx && q.zp == zp && q.rs == rs;
                  }))
                cand.push_back({xr, K, c, fx, zp, rs});
  };
  const int rs0 = x->radix;
  hipEvent_t a = nullptr, b = nullptr;
  HIPCHK(x, hipEventCreate(&a));
  if (hipEventCreate(&b) != hipSuccess) {
    (void)hipEventDestroy(a);
    return fail(x, CHN_EDEVICE, "hipEventCreate failed");
  }
  const bool timing = x->timing;
  x->timing = false;
  float best = 0.0f;
  Cand pick{};
  chn_status st = CHN_OK;
  auto time_all = [&]() {
    for (const auto& c : cand) {
      if ((st = set_radix(x, c.rs)) != CHN_OK) return;
      x->xrows = c.xr;
      x->zK = c.K;
      x->ychunk = c.ych;
      x->ffix = c.fx;
      x->zpipe = c.zp;
      auto run = [&]() { return x->mixed ? plane_phase<float, float>(x, x->ph, false, x->H)
                                         : plane_phase<double, double>(x, x->ph, false, x->H); };
      if ((st = run()) != CHN_OK) return;
      hipError_t e = hipEventRecord(a, x->stream);
      for (int r = 0; r < reps && st == CHN_OK && e == hipSuccess; ++r) st = run();
      if (e == hipSuccess) e = hipEventRecord(b, x->stream);
      if (e == hipSuccess) e = hipEventSynchronize(b);
      float ms = 0.0f;
      if (e == hipSuccess) e = hipEventElapsedTime(&ms, a, b);
      if (st == CHN_OK && e != hipSuccess) st = fail(x, CHN_EDEVICE, std::string("autotune timing: ") + hipGetErrorString(e));
      if (st != CHN_OK) return;
      if (best == 0.0f || ms < best) {
        best = ms;
        pick = c;
      }
    }
  };
  // stage 1: the classic radices (an ensemble's channel: its own sets) over
  // every schedule; stage 2: the other radix sets at the planes per launch
  // stage 1 chose
  const int rs1 = x->in_ensemble ? x->radix : 0;
  add(rs1, chunks);
  time_all();
  if (st == CHN_OK && best > 0.0f && !x->in_ensemble) {
    cand.clear();
    for (int rs = 1; rs <= 3; ++rs) add(rs, std::vector<int>{pick.ych});
    time_all();
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  x->timing = timing;
  if (st == CHN_OK && best == 0.0f) st = fail(x, CHN_EINVAL, "no schedule fits");
  if (st != CHN_OK) {
    (void)set_radix(x, rs0);
    return st;
  }
  if ((st = set_radix(x, pick.rs)) != CHN_OK) return st;
  x->xrows = pick.xr;
  x->zK = pick.K;
  x->ychunk = pick.ych;
  x->ffix = pick.fx;
  x->zpipe = pick.zp;
  chn_plan out{};
  chn_get_plan(x, &out);
  tune_store(path, key, out);
  if (chosen) *chosen = out;
  return CHN_OK;
}

chn_status chn_timing_enable(chn_ctx* x, int32_t enable) {
  if (chn_status s = check(x)) return s;
  x->timing = enable != 0;
  x->timed.clear();
  x->pool_used = 0;
  return CHN_OK;
}

chn_status chn_timing_read(chn_ctx* x, int32_t kind, double* total_ms, int32_t* count) {
  if (chn_status s = check(x)) return s;
  if (!total_ms || !count || kind < 0 || kind >= CHN_K_COUNT) return fail(x, CHN_EINVAL, "bad timing query");
  HIPCHK(x, hipStreamSynchronize(x->stream));
  double t = 0.0;
  int n = 0;
  for (const auto& r : x->timed) {
    if (r.kind != kind) continue;
    float ms = 0.0f;
    HIPCHK(x, hipEventElapsedTime(&ms, r.a, r.b));
    t += ms;
    ++n;
  }
  *total_ms = t;
  *count = n;
  return CHN_OK;
}

size_t chn_ens_workspace_bytes(int32_t n, const chn_config* cfgs) {
  EnsLayout L;
  return ens_layout(n, cfgs, &L) ? L.total : 0;
}

chn_status chn_ens_create(int32_t n, const chn_config* cfgs, void* d_ws, size_t ws_bytes, chn_ens** out) {
  if (!out) return fail(nullptr, CHN_EINVAL, "out is NULL");
  *out = nullptr;
  EnsLayout L;
  if (!ens_layout(n, cfgs, &L)) return fail(nullptr, CHN_EINVAL, "invalid ensemble configuration (sizes, or mixed precisions/streams)");
  if (!d_ws || ws_bytes < L.total || reinterpret_cast<uintptr_t>(d_ws) % 256)
    return fail(nullptr, CHN_EINVAL, "ensemble workspace missing, misaligned or too small");
  chn_ens* e = new chn_ens();
  e->n = n;
  e->mixed = cfgs[0].precision == CHN_MIXED;
  e->user = reinterpret_cast<hipStream_t>(cfgs[0].stream);
  char* base = reinterpret_cast<char*>(d_ws);
  for (int i = 0; i < n; ++i) {
    chn_ctx* c = nullptr;
    const chn_status s = chn_create(&cfgs[i], base + L.off[i], L.bytes[i], &c);
    if (s != CHN_OK) {
      g_create_error = "channel " + std::to_string(i) + ": " + g_create_error;
      delete e;
      return s;
    }
    e->ctx.push_back(c);
  }
  if (hipStreamCreate(&e->own) != hipSuccess || hipStreamCreate(&e->own2) != hipSuccess ||
      hipEventCreateWithFlags(&e->ev_in, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&e->ev_out, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&e->ev_lag, hipEventDisableTiming) != hipSuccess ||
      hipEventCreateWithFlags(&e->ev_join, hipEventDisableTiming) != hipSuccess) {
    delete e;
    return fail(nullptr, CHN_EDEVICE, "creating the ensemble stream/events");
  }
  const chn_status s = e->mixed ? ens_build<float>(e, base + L.tables) : ens_build<double>(e, base + L.tables);
  if (s != CHN_OK) {
    g_create_error = e->err;
    delete e;
    return s;
  }
  for (chn_ctx* c : e->ctx) c->in_ensemble = true;
  *out = e;
  return CHN_OK;
}

chn_status chn_ens_destroy(chn_ens* e) {
  delete e;
  return CHN_OK;
}

chn_ctx* chn_ens_context(chn_ens* e, int32_t i) { return (e && i >= 0 && i < e->n) ? e->ctx[i] : nullptr; }

chn_status chn_ens_set_state(chn_ens* e, int32_t i, const double* d_v, const double* d_omega2,
                             const double* d_u1mean, const double* d_u3mean) {
  if (!e) return CHN_EINVAL;
  if (i < 0 || i >= e->n) {
    e->err = "channel index out of range";
    return CHN_EINVAL;
  }
  const chn_status s = chn_set_state(e->ctx[i], d_v, d_omega2, d_u1mean, d_u3mean);
  if (s != CHN_OK) e->err = "channel " + std::to_string(i) + ": " + e->ctx[i]->err;
  return s;
}

chn_status chn_ens_step(chn_ens* e, const double* dt, int32_t nsteps) {
  if (!e || !dt || nsteps < 0) return CHN_EINVAL;
  return e->mixed ? ens_step<float>(e, dt, nsteps) : ens_step<double>(e, dt, nsteps);
}

const char* chn_ens_last_error(const chn_ens* e) { return e ? e->err.c_str() : g_create_error.c_str(); }

const char* chn_last_error(const chn_ctx* x) { return x ? x->err.c_str() : g_create_error.c_str(); }

}  // extern "C"
