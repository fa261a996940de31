// Host runtime of gedmg: context setup (CSR pattern, element colouring,
// element -> CSR offset map, network packing) and the assembly driver.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <numeric>
#include <vector>

#include "gedmg_internal.h"

using namespace gedmg;

#define GEDMG_HIP(ctx, expr)                                                     \
  do {                                                                           \
    hipError_t e_ = (expr);                                                      \
    if (e_ != hipSuccess) {                                                      \
      (ctx)->err = std::string(#expr) + ": " + hipGetErrorString(e_);            \
      return GEDMG_E_HIP;                                                        \
    }                                                                            \
  } while (0)

namespace gedmg {

hipError_t launch_energy_jet_f64(int H, const JetArgs& a, hipStream_t s, int num_cu);
hipError_t launch_energy_jet_lp(int precision, int H, const JetArgs& a, hipStream_t s, int num_cu);

static double softplus_h(double t) { return std::max(t, 0.0) + std::log1p(std::exp(-std::fabs(t))); }
static double logistic_h(double t) {
  const double e = std::exp(-std::fabs(t));
  return t >= 0 ? 1.0 / (1.0 + e) : e / (1.0 + e);
}

NetRef pack_network(const NetLayout& lay, const double* raw, std::vector<double>& p) {
  p.assign(lay.total, 0.0);
  const int H = lay.H, n = lay.n_in, L = lay.L;
  auto pass = [&](double w, int i) { return ((lay.mask >> i) & 1) ? softplus_h(w) : w; };
  for (int r = 0; r < H; ++r)
    for (int i = 0; i < n; ++i) p[lay.W0 + r * n + i] = pass(raw[lay.W0 + r * n + i], i);
  for (int r = 0; r < H; ++r) p[lay.b0 + r] = raw[lay.b0 + r];
  for (int k = 1; k < L; ++k) {
    for (int t = 0; t < H * H; ++t) p[lay.Wz[k] + t] = softplus_h(raw[lay.Wz[k] + t]);
    for (int r = 0; r < H; ++r)
      for (int i = 0; i < n; ++i) p[lay.Wx[k] + r * n + i] = pass(raw[lay.Wx[k] + r * n + i], i);
    for (int r = 0; r < H; ++r) p[lay.b[k] + r] = raw[lay.b[k] + r];
  }
  for (int r = 0; r < H; ++r) p[lay.wz + r] = softplus_h(raw[lay.wz + r]);
  for (int i = 0; i < n; ++i) p[lay.wx + i] = pass(raw[lay.wx + i], i);
  p[lay.bout] = raw[lay.bout];
  // reference state x = 0: pre-activations, N(0) and dN/dx_{n-1}
  std::vector<double> z(H), zt(H), a(H), at(H);
  for (int r = 0; r < H; ++r) {
    a[r] = p[lay.b0 + r];
    at[r] = p[lay.W0 + r * n + (n - 1)];
  }
  for (int k = 0; k < L; ++k) {
    if (k > 0) {
      for (int r = 0; r < H; ++r) {
        double s = p[lay.b[k] + r], st = p[lay.Wx[k] + r * n + (n - 1)];
        for (int m = 0; m < H; ++m) {
          s += p[lay.Wz[k] + r * H + m] * z[m];
          st += p[lay.Wz[k] + r * H + m] * zt[m];
        }
        a[r] = s;
        at[r] = st;
      }
    }
    for (int r = 0; r < H; ++r) {
      p[lay.a0 + k * H + r] = a[r];
      p[lay.s0 + k * H + r] = logistic_h(a[r]);
      p[lay.sb0 + k * H + r] = logistic_h(-a[r]);
      z[r] = softplus_h(a[r]);
      zt[r] = logistic_h(a[r]) * at[r];
    }
  }
  NetRef ref;
  ref.N0 = p[lay.bout];
  ref.n0 = p[lay.wx + n - 1];
  for (int r = 0; r < H; ++r) {
    ref.N0 += p[lay.wz + r] * z[r];
    ref.n0 += p[lay.wz + r] * zt[r];
  }
  return ref;
}

hipError_t launch_energy_jet(int precision, int H, const JetArgs& a, hipStream_t s, int num_cu) {
  if (a.L == 0) return launch_closed_form_jet(a, s);  // no layer products: FP64 whatever the precision
  if (precision == GEDMG_FP64) return launch_energy_jet_f64(H, a, s, num_cu);
  return launch_energy_jet_lp(precision, H, a, s, num_cu);
}

// Tables of the table-driven FP64 exp / log1p (device_common.h), in extended
// precision: exp 2^(j/64) = hi + lo; log over the 64 intervals of
// z in [0.6875, 1.375) that the high-word index selects: 1/c with c the
// interval's centre (exactly 1 on the two intervals next to 1, so small
// arguments keep relative precision) and -log(1/c) = hi + lo.
void build_math_tables(std::vector<double>& t) {
  t.assign(kMathTabDoubles, 0.0);
  for (int j = 0; j < 64; ++j) {
    const long double v = exp2l((long double)j / 64.0L);
    const double hi = (double)v;
    t[2 * j] = hi;
    t[2 * j + 1] = (double)(v - (long double)hi);
  }
  auto from_hi = [](uint32_t hw) {
    const uint64_t u = (uint64_t)hw << 32;
    double d;
    std::memcpy(&d, &u, 8);
    return d;
  };
  for (int i = 0; i < 64; ++i) {
    const double zlo = from_hi(0x3FE60000u + ((uint32_t)i << 14));
    const double zhi = from_hi(0x3FE60000u + ((uint32_t)(i + 1) << 14));
    const double invc = (i == 39 || i == 40) ? 1.0 : (double)(2.0L / ((long double)zlo + (long double)zhi));
    const long double lc = -logl((long double)invc);
    const double hi = (double)lc;
    double* e = &t[128 + 4 * i];
    e[0] = invc;
    e[1] = hi;
    e[2] = (double)(lc - (long double)hi);
    e[3] = 0.0;
  }
}

}  // namespace gedmg

namespace {

// Round to nearest even of a double to bf16 / fp16 bit patterns (host side,
// for the low-precision copies of the hidden weights).
uint16_t to_bf16(double v) {
  float f = (float)v;
  uint32_t u;
  std::memcpy(&u, &f, 4);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

uint16_t to_f16(double v) {
  const _Float16 h = (_Float16)(float)v;
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}

int check_net(gedmg_ctx* c, const gedmg_icnn* n, int n_in, bool energy) {
  if (!n) { c->err = "null network descriptor"; return GEDMG_E_ARG; }
  if (n->n_in != n_in) { c->err = "network input count not supported"; return GEDMG_E_SHAPE; }
  if (n->n_hidden == 0) return GEDMG_OK;  // closed-form model, no parameters
  if (!n->theta) { c->err = "null network parameters"; return GEDMG_E_ARG; }
  if (n->n_hidden < 1 || n->n_hidden > kMaxHidden) { c->err = "n_hidden must be 0..3"; return GEDMG_E_SHAPE; }
  const int H = n->width;
  const bool ok = energy ? (H == 16 || H == 32 || H == 64) : (H == 16 || H == 32);
  if (!ok) { c->err = "network width not supported"; return GEDMG_E_SHAPE; }
  return GEDMG_OK;
}

int upload_params(gedmg_ctx* c, const double* te, const double* ty) {
  if (c->closed_energy) te = nullptr;  // closed-form models have no parameters
  if (c->closed_yield) ty = nullptr;
  if (te) {
    std::copy(te, te + c->elay.n_raw, c->eraw.begin());
    std::vector<double> p;
    c->eref = pack_network(c->elay, te, p);
    GEDMG_HIP(c, hipMemcpyAsync(c->denet, p.data(), p.size() * 8, hipMemcpyHostToDevice, c->stream));
    const int H = c->elay.H, L = c->elay.L, HP = H + 8;
    std::vector<uint16_t> wb((size_t)std::max(L - 1, 1) * H * HP, 0), wf(wb.size(), 0);
    for (int k = 1; k < L; ++k)
      for (int r = 0; r < H; ++r)
        for (int m = 0; m < H; ++m) {
          const double w = p[c->elay.Wz[k] + r * H + m];
          wb[((size_t)(k - 1) * H + r) * HP + m] = to_bf16(w);
          wf[((size_t)(k - 1) * H + r) * HP + m] = to_f16(w);
        }
    GEDMG_HIP(c, hipMemcpyAsync(c->dw_bf16, wb.data(), wb.size() * 2, hipMemcpyHostToDevice, c->stream));
    GEDMG_HIP(c, hipMemcpyAsync(c->dw_f16, wf.data(), wf.size() * 2, hipMemcpyHostToDevice, c->stream));
    // FP64 operands, lane-ordered so each matrix-core step is one coalesced load
    std::vector<double> wo((size_t)std::max(L - 1, 1) * 2 * H * H, 0.0);
    for (int k = 1; k < L; ++k)
      for (int t = 0; t < H / 16; ++t)
        for (int st = 0; st < H / 4; ++st)
          for (int l = 0; l < 64; ++l) {
            const size_t base = ((((size_t)(k - 1) * 2) * (H / 16) + t) * (H / 4) + st) * 64 + l;
            const size_t tstride = (size_t)(H / 16) * (H / 4) * 64;
            wo[base] = p[c->elay.Wz[k] + (16 * t + l % 16) * H + 4 * st + l / 16];
            wo[base + tstride] = p[c->elay.Wz[k] + (4 * st + l / 16) * H + 16 * t + l % 16];
          }
    GEDMG_HIP(c, hipMemcpyAsync(c->dwop, wo.data(), wo.size() * 8, hipMemcpyHostToDevice, c->stream));
    GEDMG_HIP(c, hipStreamSynchronize(c->stream));
  }
  if (ty) {
    std::copy(ty, ty + c->ylay.n_raw, c->yraw.begin());
    std::vector<double> p;
    c->yref = pack_network(c->ylay, ty, p);
    GEDMG_HIP(c, hipMemcpyAsync(c->dynet, p.data(), p.size() * 8, hipMemcpyHostToDevice, c->stream));
    GEDMG_HIP(c, hipStreamSynchronize(c->stream));
  }
  return GEDMG_OK;
}

void free_all(gedmg_ctx* c) {
  void* ptrs[] = {c->dX, c->dconn, c->dperm, c->dXs, c->dconn_s, c->dseg, c->drowptr, c->dcol,
                  c->denet, c->dynet, c->dw_bf16, c->dw_f16, c->dwop, c->dmtab, c->dx, c->djet, c->dphiq, c->dsens,
                  c->dstatus};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
}

template <typename T>
int dalloc(gedmg_ctx* c, T** p, size_t n) {
  if (hipMalloc((void**)p, std::max<size_t>(n, 1) * sizeof(T)) != hipSuccess) {
    *p = nullptr;
    c->err = "device allocation failed";
    return GEDMG_E_NOMEM;
  }
  return GEDMG_OK;
}

}  // namespace

namespace gedmg {

__global__ void fill_zero_kernel(double* p, long n) {
  for (long i = (long)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (long)gridDim.x * blockDim.x) p[i] = 0.0;
}

Material element_material(const gedmg_ctx* c) {
  Material m = c->mat;
  if (c->closed_energy) {  // the jet already is psi_NH: unit scale, no separate volumetric term
    m.mu = 1.0;
    m.lam = 0.0;
  }
  return m;
}

int assemble_impl(gedmg_ctx* c, const double* u, const double* phi, const double* kappa_n, int precision,
                  double* R, double* K_vals, double* kappa_trial, const AssembleScratch& sc, bool fill_kernel,
                  bool refine64) {
  if (!u || !phi || !kappa_n || !R || !kappa_trial) { c->err = "null array argument"; return GEDMG_E_ARG; }
  if (precision != GEDMG_FP64 && precision != GEDMG_BF16 && precision != GEDMG_FP16) {
    c->err = "unknown precision";
    return GEDMG_E_ARG;
  }
  if (reinterpret_cast<uintptr_t>(K_vals) % 16 != 0) {
    c->err = "K_vals must be 16-byte aligned";
    return GEDMG_E_ARG;
  }
  constexpr int NEV = 6;
  hipEvent_t ev[NEV] = {};
  const bool prof = c->prof && !fill_kernel;
  if (prof) {
    for (int i = 0; i < NEV; ++i) {
      GEDMG_HIP(c, hipEventCreate(&ev[i]));
      c->prof_ev.push_back(ev[i]);
    }
    c->prof_calls++;
    GEDMG_HIP(c, hipEventRecord(ev[0], c->stream));
  }
  if (fill_kernel) {
    const long nb = std::min<long>((c->ndof + 255) / 256, 2048);
    hipLaunchKernelGGL(fill_zero_kernel, dim3((unsigned)std::max(nb, 1L)), dim3(256), 0, c->stream, R, c->ndof);
    GEDMG_HIP(c, hipGetLastError());
  } else {
    GEDMG_HIP(c, hipMemsetAsync(R, 0, sizeof(double) * c->ndof, c->stream));
  }
  if (prof) GEDMG_HIP(c, hipEventRecord(ev[1], c->stream));
  KinArgs ka{c->dX, c->dconn, u, phi, c->n_nodes, c->n_elems, sc.x, sc.phiq, c->dstatus};
  GEDMG_HIP(c, launch_qp_inputs(c->dim, ka, c->stream));
  if (prof) GEDMG_HIP(c, hipEventRecord(ev[2], c->stream));
  const int64_t nq = (int64_t)c->n_elems * c->nqp;
  JetArgs ja{sc.x, sc.jet, c->denet, precision == GEDMG_FP16 ? c->dw_f16 : c->dw_bf16, c->dwop,
             (int)nq, c->elay.L, K_vals ? 1 : 0, c->dmtab, c->mat.mu, c->mat.lam};
  GEDMG_HIP(c, launch_energy_jet(precision, c->elay.H, ja, c->stream, c->num_cu));
  if (refine64 && precision != GEDMG_FP64 && c->elay.L > 0) {
    // FP64 value and gradient over the low-precision ones (reverse mode, the
    // Hessian entries stay those of the low-precision jet): the residual and the
    // history are then those of the FP64 path, the tangent is the mixed one
    JetArgs jr = ja;
    jr.with_hessian = 0;
    GEDMG_HIP(c, launch_energy_jet(GEDMG_FP64, c->elay.H, jr, c->stream, c->num_cu));
  }
  if (prof) GEDMG_HIP(c, hipEventRecord(ev[3], c->stream));
  const Material em = element_material(c);
  HistArgs ha{sc.x, sc.jet, sc.phiq, kappa_n, c->dynet, kappa_trial, sc.sens, c->dstatus, (long)nq,
              em, c->eref.n0, c->yref.N0, c->ylay.L, c->max_local, c->frozen_history, c->dmtab};
  GEDMG_HIP(c, launch_history(ha, c->ylay.H, c->stream));
  if (prof) GEDMG_HIP(c, hipEventRecord(ev[4], c->stream));
  ElemArgs ea{};
  ea.Xs = c->dXs; ea.conn_s = c->dconn_s; ea.perm = c->dperm; ea.seg = c->dseg;
  ea.u = u; ea.phi = phi; ea.jet = sc.jet; ea.kappa = kappa_trial; ea.sens = sc.sens;
  ea.R = R; ea.K = K_vals; ea.status = c->dstatus;
  ea.n_nodes = c->n_nodes; ea.n_elems = c->n_elems;
  ea.m = em; ea.n0 = c->eref.n0;
  for (size_t k = 0; k + 1 < c->color_begin.size(); ++k) {
    ea.e_begin = c->color_begin[k];
    ea.e_end = c->color_begin[k + 1];
    GEDMG_HIP(c, launch_element(c->dim, K_vals != nullptr, ea, c->stream));
  }
  if (prof) GEDMG_HIP(c, hipEventRecord(ev[5], c->stream));
  return GEDMG_OK;
}

}  // namespace gedmg

static void prof_clear(gedmg_ctx* c);

extern "C" {

const char* gedmg_last_error(const gedmg_ctx* ctx) { return ctx ? ctx->err.c_str() : "null context"; }

int gedmg_create(gedmg_ctx** out, const gedmg_mesh* mesh, const gedmg_material* mat,
                 const gedmg_icnn* energy, const gedmg_icnn* yield, void* hip_stream) {
  if (!out || !mesh || !mat) return GEDMG_E_ARG;
  *out = nullptr;
  gedmg_ctx* c = new gedmg_ctx();
  auto fail = [&](int code) {
    free_all(c);
    *out = c;  // keep the context alive so the caller can read the message
    return code;
  };
  if (mesh->dim != 2 && mesh->dim != 3) { c->err = "dim must be 2 or 3"; return fail(GEDMG_E_SHAPE); }
  if (!mesh->X || !mesh->conn || mesh->n_nodes <= 0 || mesh->n_elems <= 0) {
    c->err = "empty or null mesh";
    return fail(GEDMG_E_ARG);
  }
  int rc = check_net(c, energy, 3, true);
  if (rc) return fail(rc);
  rc = check_net(c, yield, 1, false);
  if (rc) return fail(rc);
  c->stream = (hipStream_t)hip_stream;
  GEDMG_HIP(c, hipGetDevice(&c->device));
  if ((rc = static_scratch_init(c->device, c->err))) return fail(rc);
  GEDMG_HIP(c, hipDeviceGetAttribute(&c->num_cu, hipDeviceAttributeMultiprocessorCount, c->device));
  c->dim = mesh->dim;
  c->nen = c->dim == 3 ? 8 : 4;
  c->nqp = c->nen;
  c->nd = c->dim + 1;
  c->n_nodes = mesh->n_nodes;
  c->n_elems = mesh->n_elems;
  c->ndof = (int64_t)c->n_nodes * c->nd;
  c->mat = Material{mat->mu_e, mat->lambda_e, mat->eta_d, mat->kappa_d, mat->c_d, mat->beta_d, mat->gamma_d};
  const int nn = c->n_nodes, ne = c->n_elems, nen = c->nen, nd = c->nd;
  const int32_t* conn = mesh->conn;
  for (long t = 0; t < (long)ne * nen; ++t)
    if (conn[t] < 0 || conn[t] >= nn) { c->err = "connectivity index out of range"; return fail(GEDMG_E_ARG); }

  // ---- node adjacency -> CSR of (dim+1)^2 blocks
  std::vector<int> deg(nn, 0);
  std::vector<std::vector<int>> nbr(nn);
  for (int e = 0; e < ne; ++e)
    for (int a = 0; a < nen; ++a)
      for (int b = 0; b < nen; ++b) nbr[conn[(long)e * nen + a]].push_back(conn[(long)e * nen + b]);
  int64_t nnz = 0;
  for (int n = 0; n < nn; ++n) {
    auto& v = nbr[n];
    std::sort(v.begin(), v.end());
    v.erase(std::unique(v.begin(), v.end()), v.end());
    nnz += (int64_t)v.size() * nd * nd;
  }
  if (nnz >= (int64_t)INT32_MAX) { c->err = "CSR pattern exceeds 2^31 entries"; return fail(GEDMG_E_SHAPE); }
  c->nnz = nnz;
  std::vector<int32_t> rowptr(c->ndof + 1), col(nnz), rowstride(nn), base(nn);
  {
    int64_t off = 0;
    for (int n = 0; n < nn; ++n) {
      const int len = (int)nbr[n].size() * nd;
      base[n] = (int32_t)off;
      rowstride[n] = len;
      for (int cc = 0; cc < nd; ++cc) {
        rowptr[(int64_t)n * nd + cc] = (int32_t)off;
        int64_t p = off;
        for (int m : nbr[n])
          for (int k = 0; k < nd; ++k) col[p++] = m * nd + k;
        off += len;
      }
    }
    rowptr[c->ndof] = (int32_t)off;
  }
  std::vector<int32_t> blk((size_t)ne * nen * nen);
  for (int e = 0; e < ne; ++e)
    for (int a = 0; a < nen; ++a) {
      const int na = conn[(long)e * nen + a];
      const auto& v = nbr[na];
      for (int b = 0; b < nen; ++b) {
        const int nb = conn[(long)e * nen + b];
        const int pos = (int)(std::lower_bound(v.begin(), v.end(), nb) - v.begin());
        blk[((size_t)e * nen + a) * nen + b] = base[na] + pos * nd;
      }
    }
  // ---- greedy colouring: elements of one colour share no node
  std::vector<uint64_t> used(nn, 0);
  std::vector<int> color(ne);
  int ncol = 0;
  for (int e = 0; e < ne; ++e) {
    uint64_t m = 0;
    for (int a = 0; a < nen; ++a) m |= used[conn[(long)e * nen + a]];
    if (m == ~0ull) { c->err = "colouring needs more than 64 colours"; return fail(GEDMG_E_SHAPE); }
    int k = 0;
    while (m >> k & 1ull) ++k;
    color[e] = k;
    ncol = std::max(ncol, k + 1);
    for (int a = 0; a < nen; ++a) used[conn[(long)e * nen + a]] |= 1ull << k;
  }
  // first writer of every node-pair block: the element of lowest colour that
  // contains both nodes (one element per colour at most, colours run in order)
  std::vector<uint64_t> first((size_t)ne, 0);
  {
    std::vector<int> mincol((size_t)(nnz / nd), 1 << 30);
    for (int e = 0; e < ne; ++e)
      for (int ab = 0; ab < nen * nen; ++ab) {
        const size_t b = (size_t)blk[(size_t)e * nen * nen + ab] / nd;
        mincol[b] = std::min(mincol[b], color[e]);
      }
    for (int e = 0; e < ne; ++e)
      for (int ab = 0; ab < nen * nen; ++ab)
        if (mincol[(size_t)blk[(size_t)e * nen * nen + ab] / nd] == color[e]) first[e] |= 1ull << ab;
  }
  std::vector<int32_t> perm(ne);
  c->color_begin.assign(ncol + 1, 0);
  for (int e = 0; e < ne; ++e) c->color_begin[color[e] + 1]++;
  for (int k = 0; k < ncol; ++k) c->color_begin[k + 1] += c->color_begin[k];
  {
    std::vector<int> fill(c->color_begin.begin(), c->color_begin.end() - 1);
    for (int e = 0; e < ne; ++e) perm[fill[color[e]]++] = e;
  }

  // ---- element-kernel mesh data by colour slot: node coordinates,
  // connectivity, and the CSR offset of every nd-long segment (element row
  // (a, c), node block column b) with the first-writer flag in bit 31 (the
  // offsets are below 2^31 by the check on nnz)
  const int nseg = nen * nd * nen;
  std::vector<double> Xs((size_t)ne * c->dim * nen);
  std::vector<int32_t> conn_s((size_t)ne * nen), seg((size_t)ne * nseg);
  for (int sl = 0; sl < ne; ++sl) {
    const int e = perm[sl];
    for (int a = 0; a < nen; ++a) {
      const int na = conn[(long)e * nen + a];
      conn_s[(size_t)sl * nen + a] = na;
      for (int d = 0; d < c->dim; ++d) Xs[((size_t)sl * c->dim + d) * nen + a] = mesh->X[(size_t)d * nn + na];
      for (int cr = 0; cr < nd; ++cr)
        for (int b = 0; b < nen; ++b) {
          const uint32_t off = (uint32_t)blk[((size_t)e * nen + a) * nen + b] + (uint32_t)cr * (uint32_t)rowstride[na];
          const uint32_t fw = (uint32_t)((first[e] >> (a * nen + b)) & 1ull);
          seg[(size_t)sl * nseg + (size_t)(a * nd + cr) * nen + b] = (int32_t)(off | (fw << 31));
        }
    }
  }

  // ---- device copies
  const int64_t nq = (int64_t)ne * c->nqp;
  if ((rc = dalloc(c, &c->dX, (size_t)c->dim * nn)) || (rc = dalloc(c, &c->dconn, (size_t)ne * nen)) ||
      (rc = dalloc(c, &c->dperm, ne)) || (rc = dalloc(c, &c->dXs, Xs.size())) ||
      (rc = dalloc(c, &c->dconn_s, conn_s.size())) || (rc = dalloc(c, &c->dseg, seg.size())) ||
      (rc = dalloc(c, &c->drowptr, rowptr.size())) ||
      (rc = dalloc(c, &c->dcol, nnz)) || (rc = dalloc(c, &c->dx, (size_t)nq * 3)) ||
      (rc = dalloc(c, &c->djet, (size_t)nq * 10)) || (rc = dalloc(c, &c->dphiq, (size_t)nq)) ||
      (rc = dalloc(c, &c->dsens, (size_t)nq * 2)) || (rc = dalloc(c, &c->dstatus, 4)))
    return fail(rc);
  GEDMG_HIP(c, hipMemcpy(c->dX, mesh->X, sizeof(double) * c->dim * nn, hipMemcpyHostToDevice));
  GEDMG_HIP(c, hipMemcpy(c->dconn, conn, sizeof(int32_t) * ne * nen, hipMemcpyHostToDevice));
  GEDMG_HIP(c, hipMemcpy(c->dperm, perm.data(), sizeof(int32_t) * ne, hipMemcpyHostToDevice));
  GEDMG_HIP(c, hipMemcpy(c->dXs, Xs.data(), sizeof(double) * Xs.size(), hipMemcpyHostToDevice));
  GEDMG_HIP(c, hipMemcpy(c->dconn_s, conn_s.data(), sizeof(int32_t) * conn_s.size(), hipMemcpyHostToDevice));
  GEDMG_HIP(c, hipMemcpy(c->dseg, seg.data(), sizeof(int32_t) * seg.size(), hipMemcpyHostToDevice));
  GEDMG_HIP(c, hipMemcpy(c->drowptr, rowptr.data(), sizeof(int32_t) * rowptr.size(), hipMemcpyHostToDevice));
  GEDMG_HIP(c, hipMemcpy(c->dcol, col.data(), sizeof(int32_t) * nnz, hipMemcpyHostToDevice));
  GEDMG_HIP(c, hipMemset(c->dstatus, 0, 4 * sizeof(int)));

  // ---- networks (n_hidden == 0: the closed-form model of Sec. 4.1, no parameters)
  c->closed_energy = energy->n_hidden == 0;
  c->closed_yield = yield->n_hidden == 0;
  c->elay = c->closed_energy ? make_layout_hd(3, 0, 0, 0)
                             : make_layout_hd(3, energy->width, energy->n_hidden, energy->monotone_mask);
  c->ylay = c->closed_yield ? make_layout_hd(1, 0, 0, 0)
                            : make_layout_hd(1, yield->width, yield->n_hidden, yield->monotone_mask);
  c->eraw.assign(c->elay.n_raw, 0.0);
  c->yraw.assign(c->ylay.n_raw, 0.0);
  const size_t wlp = (size_t)std::max(c->elay.L - 1, 1) * c->elay.H * (c->elay.H + 8);
  if ((rc = dalloc(c, &c->denet, c->elay.total)) || (rc = dalloc(c, &c->dynet, c->ylay.total)) ||
      (rc = dalloc(c, &c->dw_bf16, wlp)) || (rc = dalloc(c, &c->dw_f16, wlp)) ||
      (rc = dalloc(c, &c->dwop, (size_t)std::max(c->elay.L - 1, 1) * 2 * c->elay.H * c->elay.H)) ||
      (rc = dalloc(c, &c->dmtab, kMathTabDoubles)))
    return fail(rc);
  {
    std::vector<double> mt;
    build_math_tables(mt);
    GEDMG_HIP(c, hipMemcpy(c->dmtab, mt.data(), sizeof(double) * mt.size(), hipMemcpyHostToDevice));
  }
  if ((rc = upload_params(c, energy->theta, yield->theta))) return fail(rc);
  *out = c;
  return GEDMG_OK;
}

int gedmg_destroy(gedmg_ctx* ctx) {
  if (!ctx) return GEDMG_E_ARG;
  if (ctx->stream || ctx->dX) (void)hipStreamSynchronize(ctx->stream);
  release_newton_work(ctx);
  prof_clear(ctx);
  free_all(ctx);
  delete ctx;
  return GEDMG_OK;
}

int gedmg_set_params(gedmg_ctx* ctx, const double* te, const double* ty) {
  if (!ctx) return GEDMG_E_ARG;
  return upload_params(ctx, te, ty);
}

int gedmg_csr(gedmg_ctx* ctx, int64_t* n_rows, int64_t* nnz, const int32_t** rowptr, const int32_t** col) {
  if (!ctx) return GEDMG_E_ARG;
  if (n_rows) *n_rows = ctx->ndof;
  if (nnz) *nnz = ctx->nnz;
  if (rowptr) *rowptr = ctx->drowptr;
  if (col) *col = ctx->dcol;
  return GEDMG_OK;
}

int gedmg_assemble(gedmg_ctx* c, const double* u, const double* phi, const double* kappa_n,
                   int precision, double* R, double* K_vals, double* kappa_trial) {
  if (!c) return GEDMG_E_ARG;
  const AssembleScratch sc{c->dx, c->djet, c->dphiq, c->dsens};
  return assemble_impl(c, u, phi, kappa_n, precision, R, K_vals, kappa_trial, sc, false, false);
}

static void prof_clear(gedmg_ctx* c) {
  for (hipEvent_t e : c->prof_ev) (void)hipEventDestroy(e);
  c->prof_ev.clear();
  c->prof_calls = 0;
}

int gedmg_profile(gedmg_ctx* c, int enable) {
  if (!c) return GEDMG_E_ARG;
  GEDMG_HIP(c, hipStreamSynchronize(c->stream));
  prof_clear(c);
  c->prof = enable != 0;
  return GEDMG_OK;
}

int gedmg_profile_read(gedmg_ctx* c, double* out, int32_t* n_calls) {
  if (!c || !out) return GEDMG_E_ARG;
  GEDMG_HIP(c, hipStreamSynchronize(c->stream));
  for (int i = 0; i < 5; ++i) out[i] = 0.0;
  for (size_t b = 0; b + 6 <= c->prof_ev.size(); b += 6) {
    float ms;
    const int map[5] = {1, 2, 3, 4, 0};  // inputs, jets, history, elements, fills
    for (int ph = 0; ph < 5; ++ph) {
      const int i0 = map[ph];
      GEDMG_HIP(c, hipEventElapsedTime(&ms, c->prof_ev[b + i0], c->prof_ev[b + i0 + 1]));
      out[ph] += ms;
    }
  }
  if (n_calls) *n_calls = c->prof_calls;
  return GEDMG_OK;
}

int gedmg_energy_jet(gedmg_ctx* c, const double* x, int64_t n, int precision, double* jet) {
  if (!c) return GEDMG_E_ARG;
  if (n < 0 || n > INT32_MAX || (n > 0 && (!x || !jet))) { c->err = "bad jet arguments"; return GEDMG_E_ARG; }
  if (precision != GEDMG_FP64 && precision != GEDMG_BF16 && precision != GEDMG_FP16) {
    c->err = "unknown precision";
    return GEDMG_E_ARG;
  }
  JetArgs ja{x, jet, c->denet, precision == GEDMG_FP16 ? c->dw_f16 : c->dw_bf16, c->dwop, (int)n,
             c->elay.L, 1, c->dmtab, c->mat.mu, c->mat.lam};
  GEDMG_HIP(c, launch_energy_jet(precision, c->elay.H, ja, c->stream, c->num_cu));
  return GEDMG_OK;
}

int gedmg_status(gedmg_ctx* c) {
  if (!c) return GEDMG_E_ARG;
  GEDMG_HIP(c, hipStreamSynchronize(c->stream));
  int st = 0;
  GEDMG_HIP(c, hipMemcpy(&st, c->dstatus, sizeof(int), hipMemcpyDeviceToHost));
  GEDMG_HIP(c, hipMemset(c->dstatus, 0, sizeof(int)));
  if (st == GEDMG_E_JNONPOS) c->err = "det F <= 0 at a quadrature point";
  if (st == GEDMG_E_LOCAL_NOCONV) c->err = "history update did not converge";
  return st;
}

}  // extern "C"
