// Host side of the C-ABI (include/islbm.h): mesh validation, parameter
// derivation (Sec. 2.1 and Sec. 3), per-axis interpolation tables (Sec. 2.2),
// reduction coefficients (Eqs. (16)-(18)), buffer management and launches.
#include <hip/hip_runtime.h>

#include <cmath>
#include <limits>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/islbm.h"
#include "islbm_launch.hpp"

using islbm::DevState;

struct islbm_ctx {
  DevState s{};
  int lattice = 2, dim = 2, storage = 0, qf = 9, qg = 5;
  int n[3] = {1, 1, 1};
  long long nn = 0;
  double delta = 1, H_lu = 1, heff[3] = {1, 1, 1};
  double Ra = 0, Pr = 0, uf = 0, Thot = 0, Tcold = 0, T0 = 0, dT = 1;
  double nu = 0, alpha = 0, gbeta = 0, aT = 0, omega = 0;
  double const_hot = 0, const_cold = 0;
  std::vector<double> X[3];  // coordinates in lattice units, x_0 .. x_{N+1}
  void* buf[4] = {nullptr, nullptr, nullptr, nullptr};  // fA fB gA gB
  bool own_buf = true;
  int cur = 0;
  size_t fbytes = 0, gbytes = 0;
  void* wtab[3] = {nullptr, nullptr, nullptr};
  double* red = nullptr;
  double* partials = nullptr;
  unsigned int* rctr = nullptr;  // step counters of the stochastic rounding
  int partials_cap = 0, partials_n = 0;
  bool partials_valid = false;
  double* dres = nullptr;
  double* hres = nullptr;
  double* staging = nullptr;
  double* fields_dev = nullptr;
  double* snap = nullptr;        // steady-change snapshot: ux, uy, uz, T (nn doubles each)
  double* snap_part = nullptr;   // its per-workgroup partial sums (4 doubles per workgroup)
  bool snap_valid = false;
  long long snap_t = 0;
  hipStream_t stream = nullptr;
  bool own_stream = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, ev2 = nullptr;
  long long t = 0;
  int no_graph = 0;
  hipGraphExec_t batch[2] = {nullptr, nullptr};  // 64 plain launches from buffer parity 0 / 1
  // graphs of the plain launches left after the 64-step batches, keyed by
  // launch count and the buffer parity they start from (round-robin slots)
  struct Tail {
    hipGraphExec_t exec = nullptr;
    long long steps = 0;
    int parity = 0;
  } tail[4];
  int tail_next = 0;
  long long tail_last = -1;  // key of the previous remainder left ungraphed
  bool graph_warm = false;   // the empty warm-up graph has run on this context
  std::string err;
};

static thread_local std::string g_create_error;

static constexpr size_t kCtrBytes = sizeof(unsigned int);  // saved step counter

static const char* kStatusText[] = {"ok",
                                    "invalid argument",
                                    "mesh violates the spacing convention",
                                    "parameters outside the stable range",
                                    "out of memory",
                                    "HIP device error",
                                    "non-finite value in the reduced state"};

extern "C" const char* islbm_strerror(int code) {
  if (code > 0 || code < -6) return "unknown status";
  return kStatusText[-code];
}

extern "C" const char* islbm_last_error(const islbm_ctx* ctx) {
  return ctx ? ctx->err.c_str() : g_create_error.c_str();
}

static int fail(islbm_ctx* ctx, int code, const std::string& msg) {
  if (ctx) ctx->err = msg;
  else g_create_error = msg;
  return code;
}

static int hipfail(islbm_ctx* ctx, hipError_t e, const char* where) {
  std::string m = std::string(where) + ": " + hipGetErrorString(e);
  return fail(ctx, e == hipErrorOutOfMemory ? ISLBM_ENOMEM : ISLBM_EDEVICE, m);
}

#define HIPCHECK(ctx, call)                                  \
  do {                                                       \
    hipError_t e_ = (call);                                  \
    if (e_ != hipSuccess) return hipfail((ctx), e_, #call);  \
  } while (0)

extern "C" void islbm_default_options(islbm_options* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->T_hot = 0.5;
  o->T_cold = -0.5;
  o->storage = ISLBM_FP32;
}

// Bytes of one stored population value: FP32 and FP32SR 4, FP64 8, FP16DEV
// and BF16DEV 2.
static size_t elem_bytes(int storage) {
  switch (storage) {
    case ISLBM_FP32: return 4;
    case ISLBM_FP64: return 8;
    case ISLBM_FP32SR: return 4;
    default: return 2;
  }
}

static int pitch_for(int n0, int storage) {
  const int align = (int)(256 / elem_bytes(storage));
  return ((n0 + align - 1) / align) * align;
}

extern "C" int islbm_query_bytes(int lattice, const int n[3], int storage, size_t* f_bytes,
                                 size_t* g_bytes) {
  if (!n || (lattice != 2 && lattice != 3) || storage < 0 || storage > 4) return ISLBM_EINVAL;
  const int n2 = lattice == 3 ? n[2] : 1;
  if (n[0] < 3 || n[1] < 3 || n2 < (lattice == 3 ? 3 : 1)) return ISLBM_EINVAL;
  const size_t plane = (size_t)pitch_for(n[0], storage) * n[1] * n2;
  const int qf = lattice == 2 ? 9 : 19, qg = lattice == 2 ? 5 : 7;
  if (f_bytes) *f_bytes = plane * qf * elem_bytes(storage);
  if (g_bytes) *g_bytes = plane * qg * elem_bytes(storage);
  return ISLBM_OK;
}

extern "C" int islbm_mesh_spacing(int kind, int n, double a, double* spacing) {
  if (!spacing || n < 3 || kind < 0 || kind > 3) return ISLBM_EINVAL;
  if ((kind == 1 || kind == 3) && !(a > 0.0)) return ISLBM_EINVAL;
  std::vector<double> x(n + 2);
  for (int j = 0; j <= n + 1; ++j) {
    const double xi = double(j) / double(n + 1);
    switch (kind) {
      case 0: x[j] = (double(j) - 0.5) / double(n); break;
      case 1: x[j] = 0.5 * (std::erf(a * (xi - 0.5)) / std::erf(0.5 * a) + 1.0); break;
      case 2: x[j] = 0.5 * (1.0 - std::cos(M_PI * xi)); break;
      default: x[j] = 0.5 * (std::tanh(a * (xi - 0.5)) / std::tanh(0.5 * a) + 1.0); break;
    }
  }
  for (int m = 0; m <= n; ++m) spacing[m] = x[m + 1] - x[m];
  // the two ghost spacings are exact mirrors of each other
  spacing[n] = spacing[0];
  return ISLBM_OK;
}

// Three-point Lagrange weights at xd over nodes p[0..2] (lattice units);
// one-hot when xd is within 1e-12 of a node.
static void lagrange3(const double* p, double xd, double* w) {
  for (int k = 0; k < 3; ++k)
    if (std::fabs(xd - p[k]) <= 1e-12) {
      w[0] = w[1] = w[2] = 0.0;
      w[k] = 1.0;
      return;
    }
  const double a = p[0] - p[1], c = p[2] - p[1], x = xd - p[1];
  w[0] = x * (x - c) / (a * (a - c));
  w[1] = (x - a) * (x - c) / (a * c);
  w[2] = x * (x - a) / (c * (c - a));
}

static void lagrange3_deriv(const double* p, double xd, double* d) {
  d[0] = ((xd - p[1]) + (xd - p[2])) / ((p[0] - p[1]) * (p[0] - p[2]));
  d[1] = ((xd - p[0]) + (xd - p[2])) / ((p[1] - p[0]) * (p[1] - p[2]));
  d[2] = ((xd - p[0]) + (xd - p[1])) / ((p[2] - p[0]) * (p[2] - p[1]));
}

// Frees everything the context owns.  Errors are ignored on purpose: this
// runs on teardown paths where nothing useful can be done with them.
static void release(islbm_ctx* c) {
  if (!c) return;
  auto dfree = [](void* p) {
    if (p) (void)hipFree(p);
  };
  for (auto& b : c->batch)
    if (b) (void)hipGraphExecDestroy(b);
  for (auto& t : c->tail)
    if (t.exec) (void)hipGraphExecDestroy(t.exec);
  if (c->own_buf)
    for (auto& b : c->buf) dfree(b);
  for (auto& w : c->wtab) dfree(w);
  dfree(c->red);
  dfree(c->partials);
  dfree(c->rctr);
  dfree(c->dres);
  if (c->hres) (void)hipHostFree(c->hres);
  dfree(c->staging);
  dfree(c->fields_dev);
  dfree(c->snap);
  dfree(c->snap_part);
  if (c->ev0) (void)hipEventDestroy(c->ev0);
  if (c->ev1) (void)hipEventDestroy(c->ev1);
  if (c->ev2) (void)hipEventDestroy(c->ev2);
  if (c->own_stream && c->stream) (void)hipStreamDestroy(c->stream);
}

extern "C" void islbm_destroy(islbm_ctx* ctx) {
  if (!ctx) return;
  if (ctx->stream) (void)hipStreamSynchronize(ctx->stream);
  release(ctx);
  delete ctx;
}

static void* fbuf(islbm_ctx* c, int which) { return c->buf[which]; }       // 0 A, 1 B
static void* gbuf(islbm_ctx* c, int which) { return c->buf[2 + which]; }

extern "C" int islbm_create(islbm_ctx** out, int lattice, const int n_in[3],
                            const double* const spacing[3], double Ra, double Pr,
                            const islbm_options* opt_in) {
  if (out) *out = nullptr;
  g_create_error.clear();
  if (!out || !n_in || !spacing) return fail(nullptr, ISLBM_EINVAL, "NULL argument");
  if (lattice != ISLBM_D2Q9_D2Q5 && lattice != ISLBM_D3Q19_D3Q7)
    return fail(nullptr, ISLBM_EINVAL, "unknown lattice");
  if (!(Ra > 0.0) || !(Pr > 0.0) || !std::isfinite(Ra) || !std::isfinite(Pr))
    return fail(nullptr, ISLBM_EINVAL, "Ra and Pr must be positive and finite");
  islbm_options opt;
  if (opt_in) opt = *opt_in;
  else islbm_default_options(&opt);
  if (opt.storage < 0 || opt.storage > 4) return fail(nullptr, ISLBM_EINVAL, "unknown storage");
  const int dim = lattice;
  int n[3] = {n_in[0], n_in[1], dim == 3 ? n_in[2] : 1};
  for (int a = 0; a < dim; ++a) {
    if (n[a] < 3) return fail(nullptr, ISLBM_EINVAL, "every axis needs at least 3 fluid nodes");
    if (!spacing[a]) return fail(nullptr, ISLBM_EINVAL, "NULL spacing array");
  }
  const long long nn = (long long)n[0] * n[1] * n[2];
  if (nn > (1LL << 40)) return fail(nullptr, ISLBM_EINVAL, "mesh too large");

  // ---- mesh: lattice unit, coordinates in lattice units --------------------
  const double delta = spacing[0][0];
  if (!(delta > 0.0) || !std::isfinite(delta)) return fail(nullptr, ISLBM_EMESH, "non-positive lattice unit");
  auto* c = new (std::nothrow) islbm_ctx();
  if (!c) return fail(nullptr, ISLBM_ENOMEM, "host allocation");
  c->lattice = lattice;
  c->dim = dim;
  c->qf = dim == 2 ? 9 : 19;
  c->qg = dim == 2 ? 5 : 7;
  c->storage = opt.storage;
  for (int a = 0; a < 3; ++a) c->n[a] = n[a];
  c->nn = nn;
  c->delta = delta;
  for (int a = 0; a < 3; ++a) {
    if (a >= dim) {
      c->X[a] = {-0.5, 0.5, 1.5};
      c->heff[a] = 1.0;
      continue;
    }
    const double* sp = spacing[a];
    auto& X = c->X[a];
    X.assign(n[a] + 2, 0.0);
    for (int m = 0; m <= n[a]; ++m) {
      const double h = sp[m];
      if (!std::isfinite(h) || h < delta * (1.0 - 1e-12)) {
        delete c;
        return fail(nullptr, ISLBM_EMESH, "a spacing is below the lattice unit or not finite");
      }
      X[m + 1] = X[m] + h / delta;
    }
    if (std::fabs(sp[0] - delta) > 1e-12 * delta || std::fabs(sp[n[a]] - delta) > 1e-12 * delta) {
      delete c;
      return fail(nullptr, ISLBM_EMESH, "ghost spacings must equal the lattice unit on every axis");
    }
    c->heff[a] = 0.5 * (X[n[a]] + X[n[a] + 1]) - 0.5 * (X[0] + X[1]);
  }
  c->H_lu = c->heff[1];

  // ---- parameters (Sec. 2.1, Eqs. (2)-(7), Sec. 3 reference velocity) -----
  c->Ra = Ra;
  c->Pr = Pr;
  c->uf = opt.u_f > 0.0 ? opt.u_f : 0.1 / std::sqrt(3.0);
  c->Thot = opt.T_hot;
  c->Tcold = opt.T_cold;
  c->T0 = 0.5 * (c->Thot + c->Tcold);
  c->dT = (c->Thot - c->Tcold) != 0.0 ? (c->Thot - c->Tcold) : 1.0;
  c->gbeta = c->uf * c->uf / (c->H_lu * c->dT);
  c->nu = c->uf * c->H_lu * std::sqrt(Pr / Ra);
  c->alpha = c->uf * c->H_lu / std::sqrt(Ra * Pr);
  const double s3 = std::sqrt(3.0);
  c->aT = dim == 2 ? 20.0 * s3 * c->alpha - 4.0 : 42.0 * s3 * c->alpha - 6.0;
  c->omega = dim == 2 ? (4.0 + c->aT) / 10.0 : (6.0 + c->aT) / 21.0;
  if (c->aT > 1.0 && !opt.allow_unstable) {
    char msg[200];
    std::snprintf(msg, sizeof msg,
                  "a_T = %.4g > 1 (alpha = %.4g l.u.): the thermal rest equilibrium has a negative "
                  "weight; lower u_f or set allow_unstable",
                  c->aT, c->alpha);
    delete c;
    return fail(nullptr, ISLBM_EPARAM, msg);
  }
  const double snu = 1.0 / (3.0 * c->nu + 0.5);
  const double sq = 8.0 * (2.0 - snu) / (8.0 - snu);
  DevState& s = c->s;
  s.dim = dim;
  s.storage = opt.storage;
  for (int a = 0; a < 3; ++a) s.n[a] = n[a];
  s.pitch = pitch_for(n[0], opt.storage);
  s.plane = (long long)s.pitch * n[1] * n[2];
  // populations interleaved by rows: [z][y][pop][x]
  s.ps = s.pitch;
  s.rsf = (long long)c->qf * s.pitch;
  s.rsg = (long long)c->qg * s.pitch;
  s.s_nu = snu;
  s.s_e = opt.s_e > 0 ? opt.s_e : snu;
  s.s_eps = opt.s_eps > 0 ? opt.s_eps : snu;
  s.s_pi = opt.s_pi > 0 ? opt.s_pi : snu;
  s.s_q = opt.s_q > 0 ? opt.s_q : sq;
  s.s_m = opt.s_m > 0 ? opt.s_m : sq;
  s.q_j = opt.q_j > 0 ? opt.q_j : 3.0 - s3;
  s.q_e = opt.q_e > 0 ? opt.q_e : 4.0 * s3 - 6.0;
  s.q_nu = opt.q_nu > 0 ? opt.q_nu : 4.0 * s3 - 6.0;
  s.aT = c->aT;
  s.gbeta = c->gbeta;
  s.T0 = c->T0;
  s.omega = c->omega;
  s.Thot = c->Thot;
  s.Tcold = c->Tcold;
  s.inv_uf = 1.0 / c->uf;
  s.inv_dT = 1.0 / c->dT;
  s.collide = opt.stream_only ? 0 : 1;
  c->no_graph = opt.no_graph;

  // ---- interpolation tables (Sec. 2.2) ------------------------------------
  const bool dbl = opt.storage == ISLBM_FP64 || opt.storage == ISLBM_FP32SR;  // FP64 arithmetic
  std::vector<std::vector<double>> tab(3);
  bool onehot = true;
  for (int a = 0; a < 3; ++a) {
    const int na = n[a];
    tab[a].assign((size_t)2 * na * 4, 0.0);
    if (a >= dim) continue;
    const auto& X = c->X[a];
    for (int sd = 0; sd < 2; ++sd) {
      const int sgn = sd == 0 ? 1 : -1;
      for (int j = 0; j < na; ++j) {
        double* w = &tab[a][((size_t)sd * na + j) * 4];
        const bool wall = (sgn == 1 && j == 0) || (sgn == -1 && j == na - 1);
        if (wall) continue;  // link leaves the fluid: wall rule, weights 0
        const int b = std::min(std::max(j - 1, 0), na - 3);
        const double p[3] = {X[b + 1], X[b + 2], X[b + 3]};
        lagrange3(p, X[j + 1] - sgn, w);
        const int nz = (w[0] != 0.0) + (w[1] != 0.0) + (w[2] != 0.0);
        if (nz != 1) onehot = false;
      }
    }
  }
  s.uniform = (onehot && !opt.force_interp) ? 1 : 0;

  // ---- reduction coefficients (Eqs. (16)-(18), Sec. 3 definitions) --------
  std::vector<double> red;
  for (int a = 0; a < 3; ++a) {
    s.red_vol[a] = (long long)red.size();
    for (int j = 0; j < n[a]; ++j) {
      const double V = a < dim ? 0.5 * (c->X[a][j + 2] - c->X[a][j]) : 1.0;
      red.push_back(V / c->heff[a]);
    }
  }
  for (int a = 0; a < 3; ++a) {
    s.red_mw[a] = (long long)red.size();
    for (int j = 0; j < n[a]; ++j) red.push_back(a < dim ? 0.5 * (c->X[a][j + 2] - c->X[a][j]) : 1.0);
  }
  const int nx = n[0];
  const auto& X0 = c->X[0];
  std::vector<double> chot(nx, 0.0), ccold(nx, 0.0), cmv(nx, 0.0), cmd(nx, 0.0);
  {
    const double H = c->H_lu;
    const double qh = X0[2] - X0[1];
    chot[0] = -H * (2.0 * qh + 1.0) / qh;
    chot[1] += H / (qh * (2.0 * qh + 1.0));
    const double qc = X0[nx] - X0[nx - 1];
    ccold[nx - 1] = H * (2.0 * qc + 1.0) / qc;
    ccold[nx - 2] += -H / (qc * (2.0 * qc + 1.0));
    const double Th = (c->Thot - c->T0) / c->dT, Tc = (c->Tcold - c->T0) / c->dT;
    c->const_hot = 4.0 * H * (qh + 1.0) * Th / (2.0 * qh + 1.0);
    c->const_cold = -4.0 * H * (qc + 1.0) * Tc / (2.0 * qc + 1.0);
    // mid-plane x* = 1/2
    const double xc = 0.5 * (0.5 * (X0[0] + X0[1]) + 0.5 * (X0[nx] + X0[nx + 1]));
    int k = 0;
    for (int i = 1; i < nx; ++i)
      if (std::fabs(X0[i + 1] - xc) < std::fabs(X0[k + 1] - xc) - 1e-12) k = i;
    std::vector<int> bases;
    const bool tie = k + 1 < nx && std::fabs(std::fabs(X0[k + 2] - xc) - std::fabs(X0[k + 1] - xc)) <= 1e-12;
    auto clampb = [&](int b) { return std::min(std::max(b, 0), nx - 3); };
    bases.push_back(clampb(k - 1));
    if (tie && clampb(k) != bases[0]) bases.push_back(clampb(k));
    const double sRaPr = std::sqrt(Ra * Pr);
    for (int b : bases) {
      const double p[3] = {X0[b + 1], X0[b + 2], X0[b + 3]};
      double w[3], d[3];
      lagrange3(p, xc, w);
      lagrange3_deriv(p, xc, d);
      for (int m = 0; m < 3; ++m) {
        cmv[b + m] += sRaPr * w[m] / double(bases.size());
        cmd[b + m] += -H * d[m] / double(bases.size());
      }
    }
  }
  s.red_chot = (long long)red.size();
  red.insert(red.end(), chot.begin(), chot.end());
  s.red_ccold = (long long)red.size();
  red.insert(red.end(), ccold.begin(), ccold.end());
  s.red_cmv = (long long)red.size();
  red.insert(red.end(), cmv.begin(), cmv.end());
  s.red_cmd = (long long)red.size();
  red.insert(red.end(), cmd.begin(), cmd.end());

  // ---- device resources ------------------------------------------------------
  int ndev = 0;
  hipError_t e = hipGetDeviceCount(&ndev);
  if (e != hipSuccess || ndev <= 0) {
    delete c;
    return fail(nullptr, ISLBM_EDEVICE, "no HIP device");
  }
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess || std::strncmp(prop.gcnArchName, "gfx950", 6) != 0) {
    delete c;
    return fail(nullptr, ISLBM_EDEVICE, "the current device is not gfx950");
  }
  auto bail = [&](int code) {
    std::string m = c->err;
    release(c);
    delete c;
    g_create_error = m;
    return code;
  };
  int rc;
  if (opt.stream) {
    c->stream = static_cast<hipStream_t>(opt.stream);
  } else {
    if ((e = hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking)) != hipSuccess)
      return bail(hipfail(c, e, "hipStreamCreate"));
    c->own_stream = true;
  }
  islbm_query_bytes(lattice, n, opt.storage, &c->fbytes, &c->gbytes);
  {
    // the step kernels address a tile's rows (at most 6 z-planes and 6 rows
    // of halo and tile) by 32-bit byte offsets from its first row
    const double rows = dim == 3 ? 6.0 * n[1] + 6.0 : 6.0;
    const double span = (rows * double(s.rsf) + double(s.pitch)) * double(elem_bytes(opt.storage));
    // and form row offsets with 24-bit multiplies
    const bool fits24 = s.rsf < (1LL << 24) && n[0] < (1 << 24) && n[1] < (1 << 24) && n[2] < (1 << 24) &&
                        rows < double(1 << 24);
    if (span >= 4294967296.0 || !fits24) {
      c->err = "mesh too large: the rows of one tile exceed 32-bit offsets";
      return bail(ISLBM_EINVAL);
    }
  }
  // read + write buffers of one step against the 256 MB last-level cache
  const size_t ws = 2 * (c->fbytes + c->gbytes);
  s.large = ws > (size_t(1) << 30) ? 2 : (ws > (size_t(192) << 20) ? 1 : 0);
  const bool given = opt.buffers[0] || opt.buffers[1] || opt.buffers[2] || opt.buffers[3];
  if (given) {
    for (int i = 0; i < 4; ++i)
      if (!opt.buffers[i]) {
        c->err = "buffers: all four or none";
        return bail(ISLBM_EINVAL);
      }
    for (int i = 0; i < 4; ++i) c->buf[i] = opt.buffers[i];
    c->own_buf = false;
  } else {
    for (int i = 0; i < 4; ++i)
      if ((e = hipMalloc(&c->buf[i], i < 2 ? c->fbytes : c->gbytes)) != hipSuccess)
        return bail(hipfail(c, e, "hipMalloc(populations)"));
  }
  const size_t wsz = dbl ? sizeof(double) : sizeof(float);
  for (int a = 0; a < 3; ++a) {
    const size_t cnt = tab[a].size();
    if ((e = hipMalloc(&c->wtab[a], cnt * wsz + 16)) != hipSuccess) return bail(hipfail(c, e, "hipMalloc(tables)"));
    if (dbl) {
      e = hipMemcpy(c->wtab[a], tab[a].data(), cnt * sizeof(double), hipMemcpyHostToDevice);
    } else {
      std::vector<float> tf(tab[a].begin(), tab[a].end());
      e = hipMemcpy(c->wtab[a], tf.data(), cnt * sizeof(float), hipMemcpyHostToDevice);
    }
    if (e != hipSuccess) return bail(hipfail(c, e, "hipMemcpy(tables)"));
    s.wtab[a] = c->wtab[a];
  }
  if ((e = hipMalloc(&c->red, red.size() * sizeof(double))) != hipSuccess) return bail(hipfail(c, e, "hipMalloc(red)"));
  if ((e = hipMemcpy(c->red, red.data(), red.size() * sizeof(double), hipMemcpyHostToDevice)) != hipSuccess)
    return bail(hipfail(c, e, "hipMemcpy(red)"));
  s.red = c->red;
  c->partials_cap = std::max(islbm::step_blocks(s), islbm::reduce_state_blocks(s));
  if ((e = hipMalloc(&c->partials, (size_t)c->partials_cap * islbm::kRedSlots * sizeof(double))) != hipSuccess)
    return bail(hipfail(c, e, "hipMalloc(partials)"));
  if ((e = hipMalloc(&c->dres, islbm::kRedSlots * sizeof(double))) != hipSuccess) return bail(hipfail(c, e, "hipMalloc"));
  if ((e = hipHostMalloc(&c->hres, islbm::kRedSlots * sizeof(double), hipHostMallocDefault)) != hipSuccess)
    return bail(hipfail(c, e, "hipHostMalloc"));
  if ((e = hipEventCreate(&c->ev0)) != hipSuccess || (e = hipEventCreate(&c->ev1)) != hipSuccess ||
      (e = hipEventCreate(&c->ev2)) != hipSuccess)
    return bail(hipfail(c, e, "hipEventCreate"));
  if ((e = hipMalloc(&c->rctr, 2 * sizeof(unsigned int))) != hipSuccess) return bail(hipfail(c, e, "hipMalloc(rctr)"));
  if ((e = islbm::launch_fill_zero(c->rctr, 2 * sizeof(unsigned int), c->stream)) != hipSuccess)
    return bail(hipfail(c, e, "fill"));
  s.rctr = c->rctr;
  s.rpar = 0;
  // rest state: all deviations zero (f = w, g = 0); it is its own collision
  for (int i = 0; i < 4; ++i) {
    e = islbm::launch_fill_zero(c->buf[i], i < 2 ? c->fbytes : c->gbytes, c->stream);
    if (e != hipSuccess) return bail(hipfail(c, e, "fill"));
  }
  rc = ISLBM_OK;
  c->cur = 0;
  c->t = 0;
  *out = c;
  return rc;
}

// One fused launch from the current buffers into the other pair.
static hipError_t one_step(islbm_ctx* c, bool reduce) {
  const int in = c->cur, outb = c->cur ^ 1;
  c->s.rpar = in;
  hipError_t e = islbm::launch_step(c->s, fbuf(c, in), gbuf(c, in), fbuf(c, outb), gbuf(c, outb), reduce,
                                    c->partials, c->stream);
  if (e == hipSuccess) {
    c->cur = outb;
    c->t += 1;
  }
  return e;
}

// Replays of an even batch of plain steps through one HIP graph (the batch
// returns the state to the same buffer pair, so the graph is reusable).
static constexpr int kGraphBatch = 64;
// Remainders of at least this many plain launches are replayed from a graph
// once the same remainder recurs (or islbm_plan_steps asked for it).
static constexpr int kTailMin = 4;

// Captures `count` plain launches starting from buffer parity `parity` into
// an executable graph (nothing runs).
static hipError_t capture_plain(islbm_ctx* c, long long count, int parity, hipGraphExec_t* out) {
  *out = nullptr;
  hipStream_t cap;
  hipError_t e = hipStreamCreateWithFlags(&cap, hipStreamNonBlocking);
  if (e != hipSuccess) return e;
  hipGraph_t g = nullptr;
  const int rpar = c->s.rpar;
  e = hipStreamBeginCapture(cap, hipStreamCaptureModeThreadLocal);
  if (e == hipSuccess) {
    int cur = parity;
    for (long long i = 0; i < count && e == hipSuccess; ++i) {
      c->s.rpar = cur;
      e = islbm::launch_step(c->s, fbuf(c, cur), gbuf(c, cur), fbuf(c, cur ^ 1), gbuf(c, cur ^ 1), false,
                             c->partials, cap);
      cur ^= 1;
    }
    hipError_t e2 = hipStreamEndCapture(cap, &g);
    if (e == hipSuccess) e = e2;
  }
  c->s.rpar = rpar;
  if (e == hipSuccess) e = hipGraphInstantiate(out, g, nullptr, nullptr, 0);
  if (g) (void)hipGraphDestroy(g);
  (void)hipStreamDestroy(cap);
  if (e != hipSuccess) *out = nullptr;
  return e;
}

// The batch graph for the current buffer parity, captured on first use.
static hipGraphExec_t batch_graph(islbm_ctx* c, hipError_t* err) {
  *err = hipSuccess;
  hipGraphExec_t& g = c->batch[c->cur];
  if (!g) *err = capture_plain(c, kGraphBatch, c->cur, &g);
  return g;
}

static islbm_ctx::Tail* find_tail(islbm_ctx* c, long long count, int parity) {
  for (auto& t : c->tail)
    if (t.exec && t.steps == count && t.parity == parity) return &t;
  return nullptr;
}

static hipError_t add_tail(islbm_ctx* c, long long count, int parity) {
  islbm_ctx::Tail& t = c->tail[c->tail_next];
  if (t.exec) {
    hipError_t e = hipStreamSynchronize(c->stream);  // a replay of it may still be queued
    if (e != hipSuccess) return e;
    (void)hipGraphExecDestroy(t.exec);
    t.exec = nullptr;
  }
  hipError_t e = capture_plain(c, count, parity, &t.exec);
  if (e != hipSuccess) return e;
  t.steps = count;
  t.parity = parity;
  c->tail_next = (c->tail_next + 1) % 4;
  return hipSuccess;
}

// How a run of nsteps launches splits: batches of kGraphBatch plain launches
// (when there are at least two batches' worth), then `rest` plain launches,
// then the reducing one.
static long long batches_of(const islbm_ctx* c, long long plain) {
  return (!c->no_graph && plain >= 2 * kGraphBatch) ? plain / kGraphBatch : 0;
}

// mid (optional): an event recorded between the plain launches and the
// final, reducing one.
static int enqueue_steps(islbm_ctx* c, long long nsteps, hipEvent_t mid = nullptr) {
  if (nsteps <= 0) return ISLBM_OK;
  long long plain = nsteps - 1;  // the last launch reduces
  if (batches_of(c, plain) > 0) {
    hipError_t ge;
    hipGraphExec_t g = batch_graph(c, &ge);
    if (ge != hipSuccess) c->no_graph = 1;
    if (g) {
      while (plain >= kGraphBatch) {
        hipError_t e = hipGraphLaunch(g, c->stream);
        if (e != hipSuccess) return hipfail(c, e, "hipGraphLaunch");
        c->t += kGraphBatch;
        plain -= kGraphBatch;
      }
    }
  }
  if (!c->no_graph && plain >= kTailMin) {
    const long long key = 2 * plain + c->cur;
    islbm_ctx::Tail* t = find_tail(c, plain, c->cur);
    if (!t && key == c->tail_last) {
      if (add_tail(c, plain, c->cur) == hipSuccess) t = find_tail(c, plain, c->cur);
      else c->no_graph = 1;
    }
    c->tail_last = key;
    if (t) {
      hipError_t e = hipGraphLaunch(t->exec, c->stream);
      if (e != hipSuccess) return hipfail(c, e, "hipGraphLaunch");
      c->t += plain;
      if (plain & 1) c->cur ^= 1;
      plain = 0;
    }
  }
  for (long long i = 0; i < plain; ++i) {
    hipError_t e = one_step(c, false);
    if (e != hipSuccess) return hipfail(c, e, "step kernel");
  }
  if (mid) HIPCHECK(c, hipEventRecord(mid, c->stream));
  hipError_t e = one_step(c, true);
  if (e != hipSuccess) return hipfail(c, e, "step kernel (reducing)");
  c->partials_valid = true;
  c->partials_n = islbm::step_blocks(c->s);
  return ISLBM_OK;
}

extern "C" int islbm_plan_steps(islbm_ctx* ctx, long long nsteps) {
  if (!ctx || nsteps < 0) return ISLBM_EINVAL;
  if (ctx->no_graph || nsteps == 0) return ISLBM_OK;
  long long plain = nsteps - 1;
  const long long nb = batches_of(ctx, plain);
  if (nb > 0) {
    hipError_t e;
    (void)batch_graph(ctx, &e);
    if (e != hipSuccess) return hipfail(ctx, e, "graph capture");
    plain -= nb * kGraphBatch;
  }
  if (plain >= kTailMin && !find_tail(ctx, plain, ctx->cur)) {
    hipError_t e = add_tail(ctx, plain, ctx->cur);
    if (e != hipSuccess) return hipfail(ctx, e, "graph capture");
  }
  // The runtime sets up its graph-launch path on the first launch in a
  // process (measured: a 20-step call on 1024^2 took 418-454 us the first
  // time against 385-392 us after).  An empty graph, launched once per
  // context, does that set-up here instead; it runs no step.
  if (!ctx->graph_warm) {
    hipGraph_t g = nullptr;
    hipGraphNode_t node;
    hipGraphExec_t x = nullptr;
    hipError_t e = hipGraphCreate(&g, 0);
    if (e == hipSuccess) e = hipGraphAddEmptyNode(&node, g, nullptr, 0);
    if (e == hipSuccess) e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    if (e == hipSuccess) e = hipGraphLaunch(x, ctx->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(ctx->stream);
    if (x) (void)hipGraphExecDestroy(x);
    if (g) (void)hipGraphDestroy(g);
    if (e != hipSuccess) return hipfail(ctx, e, "graph warm-up");
    ctx->graph_warm = true;
  }
  return ISLBM_OK;
}

extern "C" int islbm_step(islbm_ctx* ctx, long long nsteps) {
  if (!ctx || nsteps < 0) return ISLBM_EINVAL;
  return enqueue_steps(ctx, nsteps);
}

extern "C" int islbm_time_steps(islbm_ctx* ctx, long long nsteps, double* ms) {
  if (!ctx || nsteps < 0 || !ms) return ISLBM_EINVAL;
  HIPCHECK(ctx, hipEventRecord(ctx->ev0, ctx->stream));
  int rc = enqueue_steps(ctx, nsteps);
  if (rc != ISLBM_OK) return rc;
  HIPCHECK(ctx, hipEventRecord(ctx->ev1, ctx->stream));
  HIPCHECK(ctx, hipEventSynchronize(ctx->ev1));
  float f = 0.f;
  HIPCHECK(ctx, hipEventElapsedTime(&f, ctx->ev0, ctx->ev1));
  *ms = f;
  return ISLBM_OK;
}

extern "C" int islbm_time_steps_split(islbm_ctx* ctx, long long nsteps, double* ms_total, double* ms_plain,
                                      double* ms_reduce) {
  if (!ctx || nsteps < 1 || !ms_total || !ms_plain || !ms_reduce) return ISLBM_EINVAL;
  HIPCHECK(ctx, hipEventRecord(ctx->ev0, ctx->stream));
  int rc = enqueue_steps(ctx, nsteps, ctx->ev2);
  if (rc != ISLBM_OK) return rc;
  HIPCHECK(ctx, hipEventRecord(ctx->ev1, ctx->stream));
  HIPCHECK(ctx, hipEventSynchronize(ctx->ev1));
  float tot = 0.f, plain = 0.f;
  HIPCHECK(ctx, hipEventElapsedTime(&tot, ctx->ev0, ctx->ev1));
  HIPCHECK(ctx, hipEventElapsedTime(&plain, ctx->ev0, ctx->ev2));
  *ms_total = tot;
  *ms_plain = plain;
  *ms_reduce = double(tot) - double(plain);
  return ISLBM_OK;
}

extern "C" int islbm_copy_bytes(void* dst, const void* src, size_t bytes, void* stream) {
  if (!dst || !src || bytes == 0 || (bytes & 15) || (reinterpret_cast<size_t>(dst) & 15) ||
      (reinterpret_cast<size_t>(src) & 15))
    return ISLBM_EINVAL;
  hipError_t e = islbm::launch_copy16(dst, src, bytes, static_cast<hipStream_t>(stream));
  return e == hipSuccess ? ISLBM_OK : ISLBM_EDEVICE;
}

extern "C" int islbm_sync(islbm_ctx* ctx) {
  if (!ctx) return ISLBM_EINVAL;
  HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
  return ISLBM_OK;
}

extern "C" long long islbm_time(const islbm_ctx* ctx) { return ctx ? ctx->t : -1; }

extern "C" int islbm_set_time(islbm_ctx* ctx, long long t) {
  if (!ctx || t < 0) return ISLBM_EINVAL;
  ctx->t = t;
  return ISLBM_OK;
}

extern "C" int islbm_info(const islbm_ctx* ctx, double* delta, double* H_lu, double* nu, double* alpha,
                          double* a_T, double* gbeta) {
  if (!ctx) return ISLBM_EINVAL;
  if (delta) *delta = ctx->delta;
  if (H_lu) *H_lu = ctx->H_lu;
  if (nu) *nu = ctx->nu;
  if (alpha) *alpha = ctx->alpha;
  if (a_T) *a_T = ctx->aT;
  if (gbeta) *gbeta = ctx->gbeta;
  return ISLBM_OK;
}

extern "C" int islbm_nu_re(islbm_ctx* ctx, islbm_stats* out) {
  if (!ctx || !out) return ISLBM_EINVAL;
  int nb = ctx->partials_n;
  if (!ctx->partials_valid) {
    hipError_t e = islbm::launch_reduce_state(ctx->s, fbuf(ctx, ctx->cur), gbuf(ctx, ctx->cur), ctx->partials,
                                              ctx->stream);
    if (e != hipSuccess) return hipfail(ctx, e, "reduce kernel");
    nb = islbm::reduce_state_blocks(ctx->s);
  }
  hipError_t e = islbm::launch_finish(ctx->partials, nb, ctx->dres, ctx->stream);
  if (e != hipSuccess) return hipfail(ctx, e, "finish kernel");
  HIPCHECK(ctx, hipMemcpyAsync(ctx->hres, ctx->dres, islbm::kRedSlots * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
  HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
  const double* r = ctx->hres;
  const double sRaPr = std::sqrt(ctx->Ra * ctx->Pr), sRaoPr = std::sqrt(ctx->Ra / ctx->Pr);
  islbm_stats st;
  st.nu_vol = sRaPr * r[0] + 1.0;
  st.re_vol = sRaoPr * r[1];
  st.re_uv = sRaoPr * r[2];
  st.mass = r[3];
  st.rho_sum = r[4];
  st.nu_hot = r[5] + ctx->const_hot;
  st.nu_cold = r[6] + ctx->const_cold;
  st.nu_mid = r[7];
  st.umax = r[8];
  st.vmax = r[9];
  st.wmax = r[10];
  st.nonfinite = (long long)r[11];
  st.re_rms = sRaoPr * std::sqrt(r[12]);
  st.step = ctx->t;
  *out = st;
  return st.nonfinite ? ISLBM_ENONFINITE : ISLBM_OK;
}

extern "C" int islbm_steady_change(islbm_ctx* ctx, double* du, double* dT, long long* steps) {
  if (!ctx || !du || !dT) return ISLBM_EINVAL;
  const int nb = islbm::reduce_state_blocks(ctx->s);
  if (!ctx->snap) HIPCHECK(ctx, hipMalloc(&ctx->snap, (size_t)ctx->nn * 4 * sizeof(double)));
  if (!ctx->snap_part) HIPCHECK(ctx, hipMalloc(&ctx->snap_part, (size_t)nb * 4 * sizeof(double)));
  const bool first = !ctx->snap_valid;
  hipError_t e = islbm::launch_steady_change(ctx->s, fbuf(ctx, ctx->cur), gbuf(ctx, ctx->cur), ctx->snap,
                                             first ? 1 : 0, ctx->snap_part, ctx->stream);
  if (e != hipSuccess) return hipfail(ctx, e, "steady-change kernel");
  std::vector<double> h((size_t)nb * 4);
  HIPCHECK(ctx, hipMemcpyAsync(h.data(), ctx->snap_part, h.size() * sizeof(double), hipMemcpyDeviceToHost,
                               ctx->stream));
  HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
  double sum[4] = {0.0, 0.0, 0.0, 0.0};
  for (int b = 0; b < nb; ++b)
    for (int i = 0; i < 4; ++i) sum[i] += h[(size_t)b * 4 + i];
  const double inf = std::numeric_limits<double>::infinity();
  auto ratio = [&](double num, double den) { return den > 0.0 ? num / den : (num > 0.0 ? inf : 0.0); };
  *du = first ? inf : ratio(sum[0], sum[1]);
  *dT = first ? inf : ratio(sum[2], sum[3]);
  if (steps) *steps = first ? 0 : ctx->t - ctx->snap_t;
  ctx->snap_valid = true;
  ctx->snap_t = ctx->t;
  return ISLBM_OK;
}

static int ensure_staging(islbm_ctx* c) {
  if (c->staging) return ISLBM_OK;
  hipError_t e = hipMalloc(&c->staging, (size_t)c->nn * sizeof(double));
  if (e != hipSuccess) return hipfail(c, e, "hipMalloc(staging)");
  return ISLBM_OK;
}

extern "C" int islbm_get_populations(islbm_ctx* ctx, double* f, double* g) {
  if (!ctx) return ISLBM_EINVAL;
  int rc = ensure_staging(ctx);
  if (rc) return rc;
  const size_t bytes = (size_t)ctx->nn * sizeof(double);
  for (int set = 0; set < 2; ++set) {
    double* host = set == 0 ? f : g;
    if (!host) continue;
    const int q = set == 0 ? ctx->qf : ctx->qg;
    const char* base = static_cast<const char*>(set == 0 ? fbuf(ctx, ctx->cur) : gbuf(ctx, ctx->cur));
    for (int p = 0; p < q; ++p) {
      const void* row0 = base + (size_t)p * ctx->s.ps * elem_bytes(ctx->storage);
      hipError_t e = islbm::launch_convert_out(ctx->s, row0, ctx->staging, p, set == 0, ctx->stream);
      if (e != hipSuccess) return hipfail(ctx, e, "convert kernel");
      HIPCHECK(ctx, hipMemcpyAsync(host + (size_t)p * ctx->nn, ctx->staging, bytes, hipMemcpyDeviceToHost,
                                   ctx->stream));
      HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    }
  }
  return ISLBM_OK;
}

extern "C" int islbm_set_populations(islbm_ctx* ctx, const double* f, const double* g, int post_collision) {
  if (!ctx || !f || !g) return ISLBM_EINVAL;
  int rc = ensure_staging(ctx);
  if (rc) return rc;
  const size_t bytes = (size_t)ctx->nn * sizeof(double);
  // pre-collision input is staged in the other buffer pair, then collided
  const int dst = post_collision ? ctx->cur : (ctx->cur ^ 1);
  for (int set = 0; set < 2; ++set) {
    const double* host = set == 0 ? f : g;
    const int q = set == 0 ? ctx->qf : ctx->qg;
    char* base = static_cast<char*>(set == 0 ? fbuf(ctx, dst) : gbuf(ctx, dst));
    for (int p = 0; p < q; ++p) {
      HIPCHECK(ctx, hipMemcpyAsync(ctx->staging, host + (size_t)p * ctx->nn, bytes, hipMemcpyHostToDevice,
                                   ctx->stream));
      void* row0 = base + (size_t)p * ctx->s.ps * elem_bytes(ctx->storage);
      hipError_t e = islbm::launch_convert_in(ctx->s, ctx->staging, row0, p, set == 0, ctx->stream);
      if (e != hipSuccess) return hipfail(ctx, e, "convert kernel");
      HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
    }
  }
  if (!post_collision) {
    hipError_t e = islbm::launch_collide_only(ctx->s, fbuf(ctx, dst), gbuf(ctx, dst), fbuf(ctx, ctx->cur),
                                              gbuf(ctx, ctx->cur), ctx->stream);
    if (e != hipSuccess) return hipfail(ctx, e, "collide kernel");
  }
  ctx->partials_valid = false;
  ctx->snap_valid = false;
  HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
  return ISLBM_OK;
}

extern "C" int islbm_init_fields_device(islbm_ctx* ctx, const double* ux, const double* uy, const double* uz,
                                        const double* T) {
  if (!ctx || !ux || !uy || !T || (ctx->dim == 3 && !uz)) return ISLBM_EINVAL;
  hipError_t e = islbm::launch_init_eq(ctx->s, ux, uy, uz, T, fbuf(ctx, ctx->cur), gbuf(ctx, ctx->cur),
                                       ctx->stream);
  if (e != hipSuccess) return hipfail(ctx, e, "init kernel");
  ctx->partials_valid = false;
  ctx->snap_valid = false;
  return ISLBM_OK;
}

extern "C" int islbm_init_fields(islbm_ctx* ctx, const double* ux, const double* uy, const double* uz,
                                 const double* T) {
  if (!ctx || !ux || !uy || !T || (ctx->dim == 3 && !uz)) return ISLBM_EINVAL;
  const int nf = ctx->dim == 3 ? 4 : 3;
  double* dev = nullptr;
  const size_t bytes = (size_t)ctx->nn * sizeof(double);
  HIPCHECK(ctx, hipMalloc(&dev, bytes * nf));
  const double* hs[4] = {ux, uy, T, uz};
  int rc = ISLBM_OK;
  for (int i = 0; i < nf && rc == ISLBM_OK; ++i) {
    hipError_t e = hipMemcpyAsync(dev + i * (size_t)ctx->nn, hs[i], bytes, hipMemcpyHostToDevice, ctx->stream);
    if (e != hipSuccess) rc = hipfail(ctx, e, "hipMemcpyAsync");
  }
  if (rc == ISLBM_OK)
    rc = islbm_init_fields_device(ctx, dev, dev + ctx->nn, ctx->dim == 3 ? dev + 3 * (size_t)ctx->nn : nullptr,
                                  dev + 2 * (size_t)ctx->nn);
  hipError_t e = hipStreamSynchronize(ctx->stream);
  (void)hipFree(dev);
  if (rc == ISLBM_OK && e != hipSuccess) rc = hipfail(ctx, e, "hipStreamSynchronize");
  return rc;
}

extern "C" int islbm_fields_device(islbm_ctx* ctx, double* rho, double* ux, double* uy, double* uz, double* T) {
  if (!ctx) return ISLBM_EINVAL;
  hipError_t e = islbm::launch_fields(ctx->s, fbuf(ctx, ctx->cur), gbuf(ctx, ctx->cur), rho, ux, uy,
                                      ctx->dim == 3 ? uz : nullptr, T, ctx->stream);
  if (e != hipSuccess) return hipfail(ctx, e, "fields kernel");
  return ISLBM_OK;
}

extern "C" int islbm_fields(islbm_ctx* ctx, double* rho, double* ux, double* uy, double* uz, double* T) {
  if (!ctx) return ISLBM_EINVAL;
  const size_t nn = (size_t)ctx->nn;
  if (!ctx->fields_dev) HIPCHECK(ctx, hipMalloc(&ctx->fields_dev, nn * 5 * sizeof(double)));
  double* d = ctx->fields_dev;
  int rc = islbm_fields_device(ctx, d, d + nn, d + 2 * nn, d + 3 * nn, d + 4 * nn);
  if (rc) return rc;
  double* hs[5] = {rho, ux, uy, ctx->dim == 3 ? uz : nullptr, T};
  for (int i = 0; i < 5; ++i)
    if (hs[i]) HIPCHECK(ctx, hipMemcpyAsync(hs[i], d + i * nn, nn * sizeof(double), hipMemcpyDeviceToHost, ctx->stream));
  HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
  return ISLBM_OK;
}

extern "C" int islbm_state_bytes(const islbm_ctx* ctx, size_t* bytes) {
  if (!ctx || !bytes) return ISLBM_EINVAL;
  *bytes = ctx->fbytes + ctx->gbytes + kCtrBytes;
  return ISLBM_OK;
}

extern "C" int islbm_save_state(islbm_ctx* ctx, void* host, size_t bytes) {
  if (!ctx || !host || bytes < ctx->fbytes + ctx->gbytes + kCtrBytes) return ISLBM_EINVAL;
  char* h = static_cast<char*>(host);
  HIPCHECK(ctx, hipMemcpyAsync(h, fbuf(ctx, ctx->cur), ctx->fbytes, hipMemcpyDeviceToHost, ctx->stream));
  HIPCHECK(ctx, hipMemcpyAsync(h + ctx->fbytes, gbuf(ctx, ctx->cur), ctx->gbytes, hipMemcpyDeviceToHost,
                               ctx->stream));
  // the step counter the next launch reads (stochastic rounding of 2-byte storage)
  HIPCHECK(ctx, hipMemcpyAsync(h + ctx->fbytes + ctx->gbytes, ctx->rctr + ctx->cur, kCtrBytes,
                               hipMemcpyDeviceToHost, ctx->stream));
  HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
  return ISLBM_OK;
}

extern "C" int islbm_load_state(islbm_ctx* ctx, const void* host, size_t bytes) {
  if (!ctx || !host || bytes != ctx->fbytes + ctx->gbytes + kCtrBytes) return ISLBM_EINVAL;
  const char* h = static_cast<const char*>(host);
  HIPCHECK(ctx, hipMemcpyAsync(fbuf(ctx, ctx->cur), h, ctx->fbytes, hipMemcpyHostToDevice, ctx->stream));
  HIPCHECK(ctx, hipMemcpyAsync(gbuf(ctx, ctx->cur), h + ctx->fbytes, ctx->gbytes, hipMemcpyHostToDevice,
                               ctx->stream));
  HIPCHECK(ctx, hipMemcpyAsync(ctx->rctr + ctx->cur, h + ctx->fbytes + ctx->gbytes, kCtrBytes,
                               hipMemcpyHostToDevice, ctx->stream));
  HIPCHECK(ctx, hipStreamSynchronize(ctx->stream));
  ctx->partials_valid = false;
  ctx->snap_valid = false;
  return ISLBM_OK;
}
