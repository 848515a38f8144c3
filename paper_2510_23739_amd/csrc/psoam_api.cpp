// C entry points of the psoam library: operator applies, proximal maps and
// the proximal-gradient solver (Alg. alg:prox-outer with the inner dual
// iteration of Alg. alg:prox-inner for the TV part).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <limits>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <vector>

#include <sys/stat.h>

#include "psoam_internal.h"

namespace psoam {
int create_plan(const psoam_geom* gp, const psoam_species* sp, const float* phi,
                const int32_t* t0, const float* taps, int32_t sir_w, int32_t prec,
                hipStream_t stream, psoam_plan** out);
void free_plan(psoam_plan* P);
int create_plan_acoustic(const psoam_geom* gp, const int32_t* t0, const float* taps,
                         int32_t sir_w, int32_t prec, hipStream_t stream, psoam_plan** out);
int create_plan_factorised(const psoam_geom* gp, const psoam_species* sp, const float* phi,
                           const float* spr, const float* eir, const psoam_shell* sh,
                           int32_t prec, hipStream_t stream, psoam_plan** out);
const char* last_error_cstr();

namespace {

inline hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

// Next FISTA step t' and extrapolation weight (Beck-Teboulle (t-1)/t', or the
// printed (t-1)/(t+1)).
inline void momentum_step(double& t, double& beta, bool literal) {
  const double tn = 0.5 * (1.0 + std::sqrt(1.0 + 4.0 * t * t));
  beta = literal ? (t - 1.0) / (t + 1.0) : (t - 1.0) / tn;
  t = tn;
}

inline double inv_mu_tv(const psoam_geom& g) {
  // 1 / eig_max(grad^T grad) = 1 / sum_d 4 sin^2(pi (n_d - 1) / (2 n_d))
  const int n[3] = {g.ny, g.nx, g.nz};
  double mu = 0.0;
  for (int d = 0; d < 3; ++d) {
    const double s = std::sin(M_PI * (n[d] - 1) / (2.0 * n[d]));
    mu += 4.0 * s * s;
  }
  return mu > 0.0 ? 1.0 / mu : 0.0;
}

struct SolveBufs {
  float* cprev;
  float* cnext;
  float* xi;
  float* g;
  float* zb;
  float* u[3];
  float* w;
};

int ensure_solve_ws(psoam_plan* P, SolveBufs& B) {
  const size_t sv = P->c_elems();
  const size_t need = sizeof(float) * sv * (5 + 9 + 1) + 256 * 16;
  if (P->solve_ws.bytes < need) {
    if (P->solve_ws.base) PSOAM_HIP(hipFree(P->solve_ws.base));
    P->solve_ws.base = nullptr;
    P->solve_ws.bytes = 0;
    PSOAM_HIP(hipMalloc(&P->solve_ws.base, need));
    P->solve_ws.bytes = need;
  }
  size_t np = std::max(band_partials(P->inner ? P->inner : P, 1), (size_t)2 * reduce_blocks((int64_t)sv));
  if (P->inner) np = std::max({np, sep_blocks(P), reduce_blocks((int64_t)P->y_elems())});
  if (P->fact) np = std::max(np, eir_blocks(P));
  if (P->n_partial < np) {
    if (P->d_partial) PSOAM_HIP(hipFree(P->d_partial));
    P->d_partial = nullptr;
    PSOAM_HIP(hipMalloc(&P->d_partial, sizeof(double) * np));
    P->n_partial = np;
  }
  if (!P->d_scalars) PSOAM_HIP(hipMalloc(&P->d_scalars, sizeof(double) * 16));
  if (!P->d_ctl) PSOAM_HIP(hipMalloc(&P->d_ctl, sizeof(int) * 4));
  auto align = [](char* p) { return (float*)(((uintptr_t)p + 255) & ~(uintptr_t)255); };
  char* p = (char*)P->solve_ws.base;
  float** slots[] = {&B.cprev, &B.cnext, &B.xi, &B.g, &B.zb, &B.u[0], &B.u[1], &B.u[2], &B.w};
  const size_t lens[] = {sv, sv, sv, sv, sv, 3 * sv, 3 * sv, 3 * sv, sv};
  for (int i = 0; i < 9; ++i) {
    float* a = align(p);
    *slots[i] = a;
    p = (char*)(a + lens[i]);
  }
  return PSOAM_OK;
}

// device objective trace of at least n doubles (device stopping tests)
int ensure_trace(psoam_plan* P, size_t n) {
  if (P->n_trace < n) {
    if (P->d_trace) PSOAM_HIP(hipFree(P->d_trace));
    P->d_trace = nullptr;
    P->n_trace = 0;
    PSOAM_HIP(hipMalloc(&P->d_trace, sizeof(double) * n));
    P->n_trace = n;
  }
  return PSOAM_OK;
}

// Kernels launched on this thread while a guard lives check the solve's stop
// flag (device stopping tests) and return at once once it is set.
struct GateGuard {
  explicit GateGuard(const int* g) { set_gate(g); }
  ~GateGuard() { set_gate(nullptr); }
  GateGuard(const GateGuard&) = delete;
  GateGuard& operator=(const GateGuard&) = delete;
};

// x = prox of theta*TV at z by n_inner dual steps (u buffers given), then the
// final map (mode 0 plain, 1 max(.,0), 2 max(. - th1, 0)).  u_start: dual
// start (null = 0).  Returns the buffer holding the last dual iterate via
// *u_last (null if n_inner == 0).
int tv_prox_core(const psoam_plan* P, float* x, const float* z, float theta, int n_inner,
                 int mode, float th1, float* const u[3], float* w, const float* u_start,
                 bool literal, const float** u_last, hipStream_t s) {
  const float inv_mu = (float)inv_mu_tv(P->g);
  (void)w;  // the fused dual step keeps w on chip; the workspace slot stays in the layout
  if (u_last) *u_last = nullptr;
  if (n_inner <= 0 || theta == 0.0f) {
    PSOAM_HIP(launch_tv_final(P, x, z, nullptr, mode, th1, s));
    return PSOAM_OK;
  }
  double t = 1.0, beta_prev = 0.0;
  const float* cur = u_start;   // u_j
  const float* prev = nullptr;  // u_{j-1}
  int slot = 0;
  for (int j = 0; j < n_inner; ++j) {
    // eta_j = u_j + beta_{j-1} (u_j - u_{j-1})
    float* nxt = u[slot];
    if (nxt == cur || nxt == prev) {
      slot = (slot + 1) % 3;
      nxt = u[slot];
      if (nxt == cur || nxt == prev) {
        slot = (slot + 1) % 3;
        nxt = u[slot];
      }
    }
    PSOAM_HIP(launch_tv_step(P, nxt, z, cur, prev, (float)beta_prev, inv_mu, theta, s));
    slot = (slot + 1) % 3;
    double beta;
    momentum_step(t, beta, literal);
    beta_prev = beta;
    prev = cur;
    cur = nxt;
  }
  PSOAM_HIP(launch_tv_final(P, x, z, cur, mode, th1, s));
  if (u_last) *u_last = cur;
  return PSOAM_OK;
}

double mu_tv(const psoam_geom& g) {
  const int n[3] = {g.ny, g.nx, g.nz};
  double mu = 0.0;
  for (int d = 0; d < 3; ++d) {
    const double sn = std::sin(M_PI * (n[d] - 1) / (2.0 * n[d]));
    mu += 4.0 * sn * sn;
  }
  return mu;
}

// pulses of u2 rounded up to its groups of four
static size_t r3_kv(const psoam_plan* P) {
  return (size_t)((P->g.n_pulses + 3) / 4 * 4) * P->v_elems();
}

// floats of one set of duals of the full regulariser: u1 [3][S][V],
// u2 [3][ceil(K/4)][V][4], u3 [S][V], each 256-byte aligned
size_t r3_set_floats(const psoam_plan* P) {
  auto al = [](size_t n) { return (n + 63) / 64 * 64; };
  const size_t sv = P->c_elems(), kv = r3_kv(P);
  return al(3 * sv) + al(3 * kv) + al(sv);
}

struct R3Bufs {
  float* u1[3];
  float* u2[3];
  float* u3[3];
  float* w;
  float* pq;  // projections of eta2 through the switching coefficients, [6][S][V]
};

// three dual sets and w carved from a 256-byte aligned block
R3Bufs r3_carve(const psoam_plan* P, void* base) {
  auto al = [](size_t n) { return (n + 63) / 64 * 64; };
  const size_t sv = P->c_elems(), kv = r3_kv(P);
  float* p = (float*)base;
  R3Bufs B;
  for (int i = 0; i < 3; ++i) {
    B.u1[i] = p;
    p += al(3 * sv);
    B.u2[i] = p;
    p += al(3 * kv);
    B.u3[i] = p;
    p += al(sv);
  }
  B.w = p;
  p += al(sv);
  B.pq = p;
  return B;
}

size_t r3_ws_bytes(const psoam_plan* P) {
  const size_t sv = P->c_elems();
  return sizeof(float) * (3 * r3_set_floats(P) + (sv + 63) / 64 * 64 + (6 * sv + 63) / 64 * 64) +
         256;
}

// x = prox of the full regulariser (TV of c, TV of S c, l1, then the final
// clamp) by n_inner steps of the stacked dual iteration from zero duals;
// th = {theta_tv, theta_tvs, theta_l1}.  Per-block steps theta_b^2 / sum_b'
// theta_b'^2 m_b' with m = {mu, mu max_v |S_v|^2, 1} (an upper bound of
// eig_max(L^T L)).
int r3_prox_core(const psoam_plan* P, float* x, const float* z, const float th[3], int n_inner,
                 const R3Bufs& B, bool literal, hipStream_t s) {
  const double mu = mu_tv(P->g);
  const double m[3] = {mu, mu * P->smax2, 1.0};
  double bsum = 0.0;
  for (int b = 0; b < 3; ++b) bsum += (double)th[b] * th[b] * m[b];
  if (n_inner <= 0 || bsum == 0.0) {
    PSOAM_HIP(launch_r3_w(P, x, z, nullptr, nullptr, nullptr, nullptr, nullptr, 0.0f, 1, s));
    return PSOAM_OK;
  }
  float step[3];
  for (int b = 0; b < 3; ++b) step[b] = (float)((double)th[b] * th[b] / bsum);
  double t = 1.0, beta_prev = 0.0;
  int cur = -1, prev = -1;
  for (int j = 0; j < n_inner; ++j) {
    int nxt = 0;
    while (nxt == cur || nxt == prev) ++nxt;
    auto U1 = [&](int i) -> const float* { return i < 0 ? nullptr : B.u1[i]; };
    auto U2 = [&](int i) -> const float* { return i < 0 ? nullptr : B.u2[i]; };
    auto U3 = [&](int i) -> const float* { return i < 0 ? nullptr : B.u3[i]; };
    // the momentum of the next step: its eta2 is projected by this step's update
    double t_next = t, beta;
    momentum_step(t_next, beta, literal);
    const bool last = j == n_inner - 1;
    PSOAM_HIP(launch_r3_w(P, B.w, z, U1(cur), U1(prev), cur < 0 ? nullptr : B.pq, U3(cur),
                          U3(prev), (float)beta_prev, 0, s));
    PSOAM_HIP(launch_r3_u(P, B.u1[nxt], B.u2[nxt], B.u3[nxt], B.pq, B.w, U1(cur), U1(prev),
                          U2(cur), U2(prev), U3(cur), U3(prev), (float)beta_prev,
                          last ? 0.0f : (float)beta, step, th, s));
    t = t_next;
    beta_prev = beta;
    prev = cur;
    cur = nxt;
  }
  // the last update projected u2 itself (no momentum)
  PSOAM_HIP(launch_r3_w(P, x, z, B.u1[cur], nullptr, B.pq, B.u3[cur], nullptr, 0.0f, 1, s));
  return PSOAM_OK;
}

int ensure_r3_ws(psoam_plan* P, R3Bufs& B) {
  const size_t need = r3_ws_bytes(P);
  if (P->r3_ws.bytes < need) {
    if (P->r3_ws.base) PSOAM_HIP(hipFree(P->r3_ws.base));
    P->r3_ws.base = nullptr;
    P->r3_ws.bytes = 0;
    PSOAM_HIP(hipMalloc(&P->r3_ws.base, need));
    P->r3_ws.bytes = need;
  }
  B = r3_carve(P, (void*)(((uintptr_t)P->r3_ws.base + 255) & ~(uintptr_t)255));
  return PSOAM_OK;
}

int check_plan(const psoam_plan* P) {
  if (!P) return fail(PSOAM_EINVAL, "plan is NULL");
  return PSOAM_OK;
}

int copy_scalars(const psoam_plan* P, double* host, int n, hipStream_t s) {
  PSOAM_HIP(hipMemcpyAsync(host, P->d_scalars, sizeof(double) * n, hipMemcpyDeviceToHost, s));
  PSOAM_HIP(hipStreamSynchronize(s));
  return PSOAM_OK;
}

// Per-solve preparation of the measurements: the separable form works with
// q = T^T p (d_q) and |p|^2 (d_scalars[9]) instead of p itself.
// Operator of a solve: the forward model A = H S (eq. one-step) or, for the
// unmixing step of the two-step method, the per-voxel switching S alone
// (eq. unmixing).
enum Op { kOpA = 0, kOpUnmix = 1 };

int prepare_p(psoam_plan* P, int op, const float* p, hipStream_t s) {
  if (op != kOpA) return PSOAM_OK;
  // FP16 residual operand: its bound takes max |p| of this solve
  PSOAM_HIP(launch_f16_pmax(P, p, s));
  if (!P->inner) return PSOAM_OK;
  PSOAM_HIP(launch_sep_contract(P, P->d_q, p, s));
  PSOAM_HIP(launch_dot(p, p, (int64_t)P->y_elems(), P->d_partial, P->d_scalars + 9, s));
  return PSOAM_OK;
}

// g = A^T (A x - p), or A^T A x when p is null.  General form: S and H with
// the residual in H's epilogue, then H^T with S^T.  Factorised form: the
// shell sums q = Lambda S x, then V^T (V q - p) written straight into the
// 16-bit H^T operand (or, for rows too long for that kernel's LDS and for
// FP32, in place row by row and then packed), then Lambda^T with S^T.  Separable form: h = H of
// phi x_s over the S species, A^T (A x - p) = phi H^T(G h - T^T p) with
// G = T^T T (prepare_p has put T^T p in d_q), never forming A x itself.
int enqueue_grad(psoam_plan* P, int op, const float* x, const float* p, float* g, hipStream_t s) {
  if (op == kOpUnmix) {
    PSOAM_HIP(launch_unmix_grad(P, g, x, p, nullptr, s));
  } else if (P->inner) {
    PSOAM_HIP(launch_switch_fwd(P->inner, x, s));
    PSOAM_HIP(launch_band(P->inner, 0, P->d_h, nullptr, nullptr, s));
    PSOAM_HIP(launch_sep_residual(P, P->d_rt, P->d_h, p ? P->d_q : nullptr, nullptr, s));
    PSOAM_HIP(launch_pack_r(P->inner, P->d_rt, s));
    PSOAM_HIP(launch_band(P->inner, 2, g, nullptr, nullptr, s));
  } else if (P->fact) {
    PSOAM_HIP(launch_switch_fwd(P, x, s));
    PSOAM_HIP(launch_band(P, 0, P->d_fq, nullptr, nullptr, s));
    if (eir_pack_fits(P, true)) {
      PSOAM_HIP(launch_eir_pack(P, P->d_fq, p, true, s));
    } else {
      PSOAM_HIP(launch_eir_rows(P, 2, P->d_fq, P->d_fq, p, nullptr, s));
      PSOAM_HIP(launch_pack_r(P, P->d_fq, s));
    }
    PSOAM_HIP(launch_band(P, 2, g, nullptr, nullptr, s));
  } else {
    PSOAM_HIP(launch_switch_fwd(P, x, s));
    PSOAM_HIP(launch_band(P, 1, nullptr, p, P->d_partial, s));
    PSOAM_HIP(launch_band(P, 2, g, nullptr, nullptr, s));
  }
  return PSOAM_OK;
}

// data term |A c - p|^2 into d_scalars[4] (separable: h^T G h - 2 h^T q, to
// which |p|^2 in d_scalars[9] is added on the host), TV and l1 sums of c into
// d_scalars[5..6], TV(S c) into d_scalars[7]
int objective_terms(psoam_plan* P, int op, const float* c, const float* p, bool with_tvs,
                    float* scratch, hipStream_t s) {
  if (op == kOpUnmix) {
    PSOAM_HIP(launch_unmix_grad(P, scratch, c, p, P->d_partial, s));
    PSOAM_HIP(launch_sum_partials(P->d_partial, unmix_blocks(P), P->d_scalars + 4, s));
  } else if (P->inner) {
    PSOAM_HIP(launch_switch_fwd(P->inner, c, s));
    PSOAM_HIP(launch_band(P->inner, 0, P->d_h, nullptr, nullptr, s));
    PSOAM_HIP(launch_sep_residual(P, P->d_rt, P->d_h, P->d_q, P->d_partial, s));
    PSOAM_HIP(launch_sum_partials(P->d_partial, sep_blocks(P), P->d_scalars + 4, s));
  } else if (P->fact) {
    PSOAM_HIP(launch_switch_fwd(P, c, s));
    PSOAM_HIP(launch_band(P, 0, P->d_fq, nullptr, nullptr, s));
    PSOAM_HIP(launch_eir_rows(P, 3, nullptr, P->d_fq, p, P->d_partial, s));
    PSOAM_HIP(launch_sum_partials(P->d_partial, eir_blocks(P), P->d_scalars + 4, s));
  } else {
    PSOAM_HIP(launch_switch_fwd(P, c, s));
    PSOAM_HIP(launch_band(P, 1, nullptr, p, P->d_partial, s));
    PSOAM_HIP(launch_sum_partials(P->d_partial, band_partials(P, 1), P->d_scalars + 4, s));
  }
  PSOAM_HIP(launch_tv_l1_sums(P, c, P->d_partial, P->d_scalars + 5, s));
  if (with_tvs) PSOAM_HIP(launch_tvs_sum(P, c, P->d_partial, P->d_scalars + 7, s));
  return PSOAM_OK;
}

// A c of the solve's iterate, y-sized (the objective by the momentum recurrence)
int ensure_yc_ws(psoam_plan* P, float*& yc) {
  const size_t need = sizeof(float) * P->y_elems() + 256;
  if (P->yc_ws.bytes < need) {
    if (P->yc_ws.base) PSOAM_HIP(hipFree(P->yc_ws.base));
    P->yc_ws.base = nullptr;
    P->yc_ws.bytes = 0;
    PSOAM_HIP(hipMalloc(&P->yc_ws.base, need));
    P->yc_ws.bytes = need;
  }
  yc = (float*)(((uintptr_t)P->yc_ws.base + 255) & ~(uintptr_t)255);
  return PSOAM_OK;
}

// The objective terms of c_{k+1} for the general operator without a second
// H: A is linear and xi_{k+1} = c_{k+1} + beta_k (c_{k+1} - c_k), so A c_{k+1}
// = (A xi_{k+1} + beta_k A c_k) / (1 + beta_k).  H's residual form at
// xi_{k+1} (the next iteration's, enqueued here) forms it from the stored
// A c_k and sums (A c_{k+1} - p)^2 into d_scalars[4]; TV, l1 (and TV(S c))
// of c_{k+1} as in objective_terms.
int objective_terms_rec(psoam_plan* P, const float* xi_next, const float* c_next,
                        const float* p, float* yc, double beta, bool with_tvs, hipStream_t s) {
  PSOAM_HIP(launch_switch_fwd(P, xi_next, s));
  PSOAM_HIP(launch_band(P, 1, nullptr, p, P->d_partial, s, yc, beta, 0));
  PSOAM_HIP(launch_sum_partials(P->d_partial, band_partials(P, 1), P->d_scalars + 4, s));
  PSOAM_HIP(launch_tv_l1_sums(P, c_next, P->d_partial, P->d_scalars + 5, s));
  if (with_tvs) PSOAM_HIP(launch_tvs_sum(P, c_next, P->d_partial, P->d_scalars + 7, s));
  return PSOAM_OK;
}

int check_opts(const float* p, const float* c, const psoam_solve_opts* o) {
  if (!p || !c || !o) return fail(PSOAM_EINVAL, "solve: NULL argument");
  if (o->k1 < 0 || o->k2 < 0 || !(o->lambda_tv >= 0.0) || !(o->lambda_l1 >= 0.0) ||
      !std::isfinite(o->lambda_tv) || !std::isfinite(o->lambda_l1) || !(o->eps1 >= 0.0) ||
      !(o->eps2 >= 0.0) || !std::isfinite(o->alpha1))
    return fail(PSOAM_EINVAL, "solve: invalid options (negative or non-finite)");
  if (o->alpha1 <= 0.0 && o->n_power < 1)
    return fail(PSOAM_EINVAL, "solve: n_power must be >= 1 when alpha1 is not given");
  if (!(o->lambda_tvs >= 0.0) || !std::isfinite(o->lambda_tvs))
    return fail(PSOAM_EINVAL, "solve: lambda_tvs must be finite and >= 0");
  return PSOAM_OK;
}

// power iteration on A^T A with FP64 norms, enqueued only: v <- v0/|v0|;
// n_power times [w = A^T A v; lam = <v, w>; v = w/|w|]; lam in d_scalars[0]
int enqueue_power(psoam_plan* P, int op, SolveBufs& B, const psoam_solve_opts* o, hipStream_t s) {
  const int64_t sv = (int64_t)P->c_elems();
  float* v = B.zb;
  float* w = B.g;
  // the power iteration's residual form of H has no measurements (max |p| = 0)
  if (op == kOpA) PSOAM_HIP(launch_f16_pmax(P, nullptr, s));
  if (o->v0) {
    PSOAM_HIP(hipMemcpyAsync(w, o->v0, sizeof(float) * sv, hipMemcpyDeviceToDevice, s));
  } else {
    PSOAM_HIP(launch_fill(w, 1.0f, sv, s));
  }
  PSOAM_HIP(launch_dot(w, w, sv, P->d_partial, P->d_scalars + 1, s));
  PSOAM_HIP(launch_scale_by_rnorm(v, w, P->d_scalars + 1, sv, s));
  for (int i = 0; i < o->n_power; ++i) {
    if (int rc = enqueue_grad(P, op, v, nullptr, w, s)) return rc;
    PSOAM_HIP(launch_dot(v, w, sv, P->d_partial, P->d_scalars + 0, s));
    PSOAM_HIP(launch_dot(w, w, sv, P->d_partial, P->d_scalars + 1, s));
    PSOAM_HIP(launch_scale_by_rnorm(v, w, P->d_scalars + 1, sv, s));
  }
  return PSOAM_OK;
}

// reads the estimate (synchronises s) and sets alpha1 = 1 / (1.01 lam)
int finish_power(psoam_plan* P, psoam_solve_stats& stats, psoam_solve_stats* st, double& alpha1,
                 hipStream_t s) {
  double hs[2];
  if (int rc = copy_scalars(P, hs, 2, s)) return rc;
  stats.lambda_max = hs[0];
  if (!std::isfinite(hs[0]) || !(hs[0] > 0.0) || !std::isfinite(hs[1])) {
    stats.status = PSOAM_EDIVERGED;
    if (st) *st = stats;
    return fail(PSOAM_EDIVERGED, "solve: power iteration gave a non-finite or non-positive estimate");
  }
  alpha1 = 1.0 / (1.01 * hs[0]);
  return PSOAM_OK;
}

psoam_solve_stats fresh_stats() {
  psoam_solve_stats stats;
  stats.iterations = 0;
  stats.status = PSOAM_OK;
  stats.alpha1 = 0.0;
  stats.lambda_max = 0.0;
  stats.objective = std::numeric_limits<double>::quiet_NaN();
  return stats;
}

int solve_one(psoam_plan* P, int op, const float* p, float* c, const psoam_solve_opts* o,
              psoam_solve_stats* st, hipStream_t s) {
  if (int rc = check_opts(p, c, o)) return rc;
  if (op == kOpUnmix && o->lambda_tvs != 0.0)
    return fail(PSOAM_EINVAL, "unmix: the unmixing regulariser has no TV(S c) term (lambda_tvs must be 0)");
  SolveBufs B;
  int rc = ensure_solve_ws(P, B);
  if (rc) return rc;
  const int64_t sv = (int64_t)P->c_elems();
  double hs[16];
  psoam_solve_stats stats = fresh_stats();
  double alpha1 = o->alpha1;
  if (alpha1 <= 0.0) {
    if ((rc = enqueue_power(P, op, B, o, s))) return rc;
    if ((rc = finish_power(P, stats, st, alpha1, s))) return rc;
  }
  stats.alpha1 = alpha1;
  const bool literal = o->literal_momentum != 0;
  const float th_tv = (float)(alpha1 * o->lambda_tv);
  const float th_l1 = (float)(alpha1 * o->lambda_l1);
  PSOAM_HIP(hipMemcpyAsync(B.cprev, c, sizeof(float) * sv, hipMemcpyDeviceToDevice, s));
  PSOAM_HIP(hipMemcpyAsync(B.xi, c, sizeof(float) * sv, hipMemcpyDeviceToDevice, s));
  const bool need_obj = o->eps1 > 0.0 || o->trace != nullptr;
  const bool r3 = o->lambda_tvs > 0.0;
  R3Bufs RB{};
  if (r3 && (rc = ensure_r3_ws(P, RB))) return rc;
  // general operator with objective evaluations: F(c_{k+1})'s data term by
  // the momentum recurrence inside the next iteration's H (enqueued at the
  // end of iteration k), not by a second H apply; PSOAM_OBJ_DIRECT=1 keeps
  // the direct evaluation (tests and timing compare both)
  const char* obj_direct = std::getenv("PSOAM_OBJ_DIRECT");
  const bool rec = need_obj && op == kOpA && !P->inner && !P->fact && o->k1 > 0 &&
                   !(obj_direct && obj_direct[0] == '1');
  float* yc = nullptr;
  if (rec && (rc = ensure_yc_ws(P, yc))) return rc;
  const float th3[3] = {th_tv, (float)(alpha1 * o->lambda_tvs), th_l1};
  double t = 1.0, f_prev = 0.0;
  bool have_f = false;
  const float* u_warm = nullptr;
  float* uw[3] = {B.u[0], B.u[1], B.u[2]};
  if ((rc = prepare_p(P, op, p, s))) return rc;
  // device stopping tests: no host read inside the loop; every kernel of
  // an iteration after the one whose test fires returns at once
  const bool dev = o->device_stop != 0;
  float* const a0 = B.cprev;
  float* const a1 = B.cnext;
  StopTest tst{o->eps1, o->eps2, o->lambda_tv, o->lambda_l1, o->lambda_tvs, need_obj ? 1 : 0,
               (op == kOpA && P->inner) ? 1 : 0, r3 ? 1 : 0};
  if (dev) {
    if (o->trace && (rc = ensure_trace(P, (size_t)std::max(o->k1, 1)))) return rc;
    PSOAM_HIP(launch_stop_init(P->d_ctl, P->d_scalars, s));
  }
  std::unique_ptr<GateGuard> gate(dev ? new GateGuard(P->d_ctl) : nullptr);
  if (rec) {
    // H's residual form at xi_0 = c_0, which also stores A c_0
    PSOAM_HIP(launch_switch_fwd(P, B.xi, s));
    PSOAM_HIP(launch_band(P, 1, nullptr, p, P->d_partial, s, yc, 0.0, 1));
  }
  for (int k = 0; k < o->k1; ++k) {
    // gradient A^T (A xi - p); with the recurrence H at xi_k ran at the end
    // of the previous iteration (its residual is H^T's operand)
    if (rec) {
      PSOAM_HIP(launch_band(P, 2, B.g, nullptr, nullptr, s));
    } else if ((rc = enqueue_grad(P, op, B.xi, p, B.g, s))) {
      return rc;
    }
    PSOAM_HIP(launch_axpby(B.zb, B.xi, B.g, 1.0f, (float)(-alpha1), sv, s));
    // prox: TV dual iteration, then max(. - alpha1 lambda_l1, 0); with the
    // TV(S c) term the stacked dual iteration of the full regulariser
    const float* u_last = nullptr;
    if (r3)
      rc = r3_prox_core(P, B.cnext, B.zb, th3, o->k2, RB, literal, s);
    else
      rc = tv_prox_core(P, B.cnext, B.zb, th_tv, o->k2, 2, th_l1, uw, B.w,
                        o->warm_inner ? u_warm : nullptr, literal, &u_last, s);
    if (rc) return rc;
    if (o->warm_inner && u_last) {
      // keep the last dual iterate out of the next call's rotation
      u_warm = u_last;
      int keep = 0;
      for (int i = 0; i < 3; ++i)
        if (uw[i] == u_last) keep = i;
      std::swap(uw[keep], uw[2]);
      // uw[2] is now the warm start; the next call writes uw[0], uw[1] and may
      // reuse uw[2] only after it stops being needed.
    }
    double beta;
    momentum_step(t, beta, literal);
    PSOAM_HIP(launch_momentum(B.xi, B.cnext, B.cprev, (float)beta, sv, P->d_partial, s));
    const size_t nb = reduce_blocks(sv);
    if (o->eps2 > 0.0) {
      PSOAM_HIP(launch_sum_partials(P->d_partial, nb, P->d_scalars + 2, s));
      PSOAM_HIP(launch_sum_partials(P->d_partial + nb, nb, P->d_scalars + 3, s));
    }
    std::swap(B.cprev, B.cnext);  // cprev = c_{k+1}
    stats.iterations = k + 1;
    // the momentum kernel's beta, as the recurrence must use it
    const double beta_f = (double)(float)beta;
    if (dev) {
      if (need_obj) {
        rc = rec ? objective_terms_rec(P, B.xi, B.cprev, p, yc, beta_f, r3, s)
                 : objective_terms(P, op, B.cprev, p, r3, B.w, s);
        if (rc) return rc;
      }
      PSOAM_HIP(launch_stop_test(P->d_ctl, P->d_scalars, o->trace ? P->d_trace : nullptr, tst, s));
      continue;
    }
    bool stop = false;
    if (need_obj || o->eps2 > 0.0) {
      if (need_obj) {
        rc = rec ? objective_terms_rec(P, B.xi, B.cprev, p, yc, beta_f, r3, s)
                 : objective_terms(P, op, B.cprev, p, r3, B.w, s);
        if (rc) return rc;
      }
      rc = copy_scalars(P, hs, 10, s);
      if (rc) return rc;
      double f_now = 0.0;
      if (need_obj) {
        const double data = (op == kOpA && P->inner) ? hs[4] + hs[9] : hs[4];
        f_now = 0.5 * data + o->lambda_tv * hs[5] + o->lambda_l1 * hs[6];
        if (r3) f_now += o->lambda_tvs * hs[7];
        if (!std::isfinite(f_now)) {
          stats.status = PSOAM_EDIVERGED;
          break;
        }
        if (o->trace) o->trace[k] = f_now;
        stats.objective = f_now;
      }
      if (k > 1) {
        if (o->eps1 > 0.0 && have_f && std::fabs(f_now - f_prev) < o->eps1 * std::fabs(f_prev))
          stop = true;
        if (o->eps2 > 0.0 && hs[3] > 0.0 && std::sqrt(hs[2]) < o->eps2 * std::sqrt(hs[3]))
          stop = true;
      }
      if (need_obj) {
        f_prev = f_now;
        have_f = true;
      }
    }
    if (stop) break;
  }
  gate.reset();
  if (dev) {
    PSOAM_HIP(launch_select_copy(c, a0, a1, P->d_ctl, sv, s));
  } else {
    PSOAM_HIP(hipMemcpyAsync(c, B.cprev, sizeof(float) * sv, hipMemcpyDeviceToDevice, s));
  }
  PSOAM_HIP(launch_dot(c, c, sv, P->d_partial, P->d_scalars + 0, s));
  rc = copy_scalars(P, hs, 13, s);
  if (rc) return rc;
  if (dev) {
    int ctl[4];
    PSOAM_HIP(hipMemcpy(ctl, P->d_ctl, sizeof(ctl), hipMemcpyDeviceToHost));
    stats.iterations = o->k1 > 0 ? ctl[1] : 0;
    if (ctl[2]) stats.status = PSOAM_EDIVERGED;
    if (need_obj && stats.iterations > 0) stats.objective = hs[12];
    if (o->trace && stats.iterations > 0)
      PSOAM_HIP(hipMemcpy(o->trace, P->d_trace, sizeof(double) * stats.iterations,
                          hipMemcpyDeviceToHost));
  }
  if (!std::isfinite(hs[0])) stats.status = PSOAM_EDIVERGED;
  if (st) *st = stats;
  if (stats.status != PSOAM_OK) return fail(PSOAM_EDIVERGED, "solve: iterate became non-finite");
  return PSOAM_OK;
}

// ---- batched solves (several plans, captured iterations) -------------------

struct BatchItem {
  psoam_plan* P;
  const float* p;
  float* c;
  const psoam_solve_opts* o;
  psoam_solve_stats* st;
  psoam_solve_stats stats;
  SolveBufs B;
  R3Bufs RB;
  double alpha1;
  int remaining;
  // device stopping tests (device_stop with eps1, eps2 or a trace)
  bool dev = false;
  bool need_obj = false;
  float* a0 = nullptr;  // the iterate buffers' initial roles (c_k, c_{k+1})
  float* a1 = nullptr;
  StopTest tst{};
};

// One outer iteration with the step state t_k on the device (d_scalars[8])
// and no host reads: the form solve_batch captures.  Same launches and the
// same arithmetic as solve_one's loop without stopping tests.
int enqueue_iteration(BatchItem& it, hipStream_t s) {
  psoam_plan* P = it.P;
  const int64_t sv = (int64_t)P->c_elems();
  SolveBufs& B = it.B;
  const psoam_solve_opts* o = it.o;
  std::unique_ptr<GateGuard> gate(it.dev ? new GateGuard(P->d_ctl) : nullptr);
  const bool literal = o->literal_momentum != 0;
  const float th_tv = (float)(it.alpha1 * o->lambda_tv);
  const float th_l1 = (float)(it.alpha1 * o->lambda_l1);
  if (int rc = enqueue_grad(P, kOpA, B.xi, it.p, B.g, s)) return rc;
  PSOAM_HIP(launch_axpby(B.zb, B.xi, B.g, 1.0f, (float)(-it.alpha1), sv, s));
  float* uw[3] = {B.u[0], B.u[1], B.u[2]};
  if (o->lambda_tvs > 0.0) {
    const float th3[3] = {th_tv, (float)(it.alpha1 * o->lambda_tvs), th_l1};
    if (int rc = r3_prox_core(P, B.cnext, B.zb, th3, o->k2, it.RB, literal, s)) return rc;
  } else if (int rc = tv_prox_core(P, B.cnext, B.zb, th_tv, o->k2, 2, th_l1, uw, B.w, nullptr,
                                   literal, nullptr, s)) {
    return rc;
  }
  const bool eps2 = it.dev && o->eps2 > 0.0;
  PSOAM_HIP(launch_momentum_dev(B.xi, B.cnext, B.cprev, P->d_scalars + 8, literal ? 1 : 0, sv,
                                eps2 ? P->d_partial : nullptr, s));
  if (eps2) {
    const size_t nb = reduce_blocks(sv);
    PSOAM_HIP(launch_sum_partials(P->d_partial, nb, P->d_scalars + 2, s));
    PSOAM_HIP(launch_sum_partials(P->d_partial + nb, nb, P->d_scalars + 3, s));
  }
  std::swap(B.cprev, B.cnext);  // cprev = c_{k+1}
  if (it.dev) {
    if (it.need_obj)
      if (int rc = objective_terms(P, kOpA, B.cprev, it.p, o->lambda_tvs > 0.0, B.w, s)) return rc;
    PSOAM_HIP(launch_stop_test(P->d_ctl, P->d_scalars, o->trace ? P->d_trace : nullptr, it.tst, s));
  }
  return PSOAM_OK;
}

// Streams and events of one batch call, released on every exit path.
struct BatchStreams {
  std::vector<hipStream_t> ss;
  std::vector<hipEvent_t> ev;
  hipEvent_t e_main = nullptr;
  ~BatchStreams() {
    for (hipStream_t x : ss)
      if (x) (void)hipStreamDestroy(x);
    for (hipEvent_t e : ev)
      if (e) (void)hipEventDestroy(e);
    if (e_main) (void)hipEventDestroy(e_main);
  }
};

// Problems on their own streams (default priority): the power iterations run
// concurrently; then each problem's pair of outer iterations is captured into
// a graph on its stream and replayed there — a pair brings the c_k / c_{k+1}
// buffers back to their roles, so one graph serves every replay; a final odd
// iteration runs eagerly.
int solve_batch_graph(std::vector<BatchItem>& items, hipStream_t caller) {
  const int n = (int)items.size();
  BatchStreams bs;
  bs.ss.assign(n, nullptr);
  bs.ev.assign(n, nullptr);
  for (int i = 0; i < n; ++i) {
    PSOAM_HIP(hipStreamCreateWithFlags(&bs.ss[i], hipStreamNonBlocking));
    PSOAM_HIP(hipEventCreateWithFlags(&bs.ev[i], hipEventDisableTiming));
  }
  PSOAM_HIP(hipEventCreateWithFlags(&bs.e_main, hipEventDisableTiming));
  PSOAM_HIP(hipEventRecord(bs.e_main, caller));
  for (int i = 0; i < n; ++i) PSOAM_HIP(hipStreamWaitEvent(bs.ss[i], bs.e_main, 0));
  // phase 1: step sizes
  for (int i = 0; i < n; ++i) {
    BatchItem& it = items[i];
    it.alpha1 = it.o->alpha1;
    if (it.alpha1 <= 0.0)
      if (int rc = enqueue_power(it.P, kOpA, it.B, it.o, bs.ss[i])) return rc;
  }
  for (int i = 0; i < n; ++i) {
    BatchItem& it = items[i];
    if (it.o->alpha1 <= 0.0)
      if (int rc = finish_power(it.P, it.stats, it.st, it.alpha1, bs.ss[i])) return rc;
    it.stats.alpha1 = it.alpha1;
    const int64_t sv = (int64_t)it.P->c_elems();
    PSOAM_HIP(hipMemcpyAsync(it.B.cprev, it.c, sizeof(float) * sv, hipMemcpyDeviceToDevice, bs.ss[i]));
    PSOAM_HIP(hipMemcpyAsync(it.B.xi, it.c, sizeof(float) * sv, hipMemcpyDeviceToDevice, bs.ss[i]));
    PSOAM_HIP(launch_set_double(it.P->d_scalars + 8, 1.0, bs.ss[i]));
    if (int rc = prepare_p(it.P, kOpA, it.p, bs.ss[i])) return rc;
    it.remaining = it.o->k1;
    it.a0 = it.B.cprev;
    it.a1 = it.B.cnext;
    if (it.dev) {
      if (it.o->trace)
        if (int rc = ensure_trace(it.P, (size_t)std::max(it.o->k1, 1))) return rc;
      PSOAM_HIP(launch_stop_init(it.P->d_ctl, it.P->d_scalars, bs.ss[i]));
    }
  }
  // phase 2: each problem's pairs of iterations captured into a graph of its
  // own and replayed on its own stream, so the problems' kernels can overlap
  // (one's HBM-bound TV steps beside another's matrix-core contractions)
  for (int i = 0; i < n; ++i) {
    BatchItem& it = items[i];
    const int pairs = it.remaining / 2;
    if (pairs == 0) continue;
    hipGraph_t graph = nullptr;
    PSOAM_HIP(hipStreamBeginCapture(bs.ss[i], hipStreamCaptureModeRelaxed));
    int rc = enqueue_iteration(it, bs.ss[i]);
    if (rc == PSOAM_OK) rc = enqueue_iteration(it, bs.ss[i]);
    const hipError_t he_end = hipStreamEndCapture(bs.ss[i], &graph);
    if (rc != PSOAM_OK || he_end != hipSuccess) {
      if (graph) (void)hipGraphDestroy(graph);
      if (rc != PSOAM_OK) return rc;
      return fail(PSOAM_EHIP, std::string("solve_batch: graph capture: ") + hipGetErrorString(he_end));
    }
    hipGraphExec_t exec = nullptr;
    const hipError_t hi = hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0);
    (void)hipGraphDestroy(graph);
    if (hi != hipSuccess) return fail(PSOAM_EHIP, std::string("solve_batch: graph instantiate: ") + hipGetErrorString(hi));
    hipError_t hl = hipSuccess;
    for (int k = 0; k < pairs && hl == hipSuccess; ++k) hl = hipGraphLaunch(exec, bs.ss[i]);
    // the executable graph may be destroyed once its launches are enqueued
    (void)hipGraphExecDestroy(exec);
    if (hl != hipSuccess) return fail(PSOAM_EHIP, std::string("solve_batch: graph launch: ") + hipGetErrorString(hl));
    it.remaining -= 2 * pairs;
  }
  // odd last iterations, results, join the caller's stream
  for (int i = 0; i < n; ++i) {
    BatchItem& it = items[i];
    if (it.remaining == 1)
      if (int rc = enqueue_iteration(it, bs.ss[i])) return rc;
    it.stats.iterations = it.o->k1;
    const int64_t sv = (int64_t)it.P->c_elems();
    if (it.dev) {
      PSOAM_HIP(launch_select_copy(it.c, it.a0, it.a1, it.P->d_ctl, sv, bs.ss[i]));
    } else {
      PSOAM_HIP(hipMemcpyAsync(it.c, it.B.cprev, sizeof(float) * sv, hipMemcpyDeviceToDevice, bs.ss[i]));
    }
    PSOAM_HIP(launch_dot(it.c, it.c, sv, it.P->d_partial, it.P->d_scalars + 0, bs.ss[i]));
  }
  int status = PSOAM_OK;
  for (int i = 0; i < n; ++i) {
    BatchItem& it = items[i];
    double h[13];
    if (int rc = copy_scalars(it.P, h, 13, bs.ss[i])) return rc;
    if (it.dev) {
      int ctl[4];
      PSOAM_HIP(hipMemcpy(ctl, it.P->d_ctl, sizeof(ctl), hipMemcpyDeviceToHost));
      it.stats.iterations = ctl[1];
      if (ctl[2]) it.stats.status = PSOAM_EDIVERGED;
      if (it.need_obj && ctl[1] > 0) it.stats.objective = h[12];
      if (it.o->trace && ctl[1] > 0)
        PSOAM_HIP(hipMemcpy(it.o->trace, it.P->d_trace, sizeof(double) * ctl[1],
                            hipMemcpyDeviceToHost));
    }
    if (!std::isfinite(h[0])) it.stats.status = PSOAM_EDIVERGED;
    if (it.st) *it.st = it.stats;
    if (it.stats.status != PSOAM_OK) status = PSOAM_EDIVERGED;
    PSOAM_HIP(hipEventRecord(bs.ev[i], bs.ss[i]));
    PSOAM_HIP(hipStreamWaitEvent(caller, bs.ev[i], 0));
  }
  if (status != PSOAM_OK) return fail(PSOAM_EDIVERGED, "solve_batch: an iterate became non-finite");
  return PSOAM_OK;
}

}  // namespace
}  // namespace psoam

// ---- the TV prox without a workspace (for callers that cannot allocate) ----
namespace psoam {
namespace {
// Dual buffers of psoam_prox_tv_noalloc: three sets of [3][S][Ny][Nx][Nz]
// floats, each set 256-byte aligned.  Every GPU the library runs on holds
// this array (128 MiB) until the process ends.  In host code its name is a
// host-side stand-in: the device address comes from hipGetSymbolAddress,
// taken once per device (noalloc_scratch) and used everywhere instead.
constexpr size_t kNoAllocFloats = (size_t)32 << 20;
static __device__ __align__(256) float scratch[kNoAllocFloats];
constexpr int kNoAllocDevices = 64;
std::mutex g_noalloc_mu;
float* g_noalloc_ptr[kNoAllocDevices] = {};

inline size_t noalloc_set_floats(size_t sv) { return (3 * sv + 63) / 64 * 64; }

// device address of `scratch` on the current device (looked up on the
// device's first call; hipGetSymbolAddress allocates nothing)
int noalloc_scratch(int plan_device, float** out) {
  int dev = -1;
  PSOAM_HIP(hipGetDevice(&dev));
  if (dev != plan_device)
    return fail(PSOAM_EINVAL, "prox_tv_noalloc: the current device is not the plan's device");
  if (dev < 0 || dev >= kNoAllocDevices)
    return fail(PSOAM_EUNSUPPORTED, "prox_tv_noalloc: device index beyond 63");
  std::lock_guard<std::mutex> lock(g_noalloc_mu);
  if (!g_noalloc_ptr[dev]) {
    void* p = nullptr;
    PSOAM_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(PSOAM_EHIP, "prox_tv_noalloc: no device address for the dual buffer");
    g_noalloc_ptr[dev] = (float*)p;
  }
  *out = g_noalloc_ptr[dev];
  return PSOAM_OK;
}
}  // namespace
}  // namespace psoam

using namespace psoam;

namespace psoam {
namespace {

// ---- launch-shape autotuner (psoam_plan_create_tuned) ---------------------
// The choice: rows per staged workgroup of H and of H^T, the H^T operand
// shift, H's loader waves, and the tile of the TV dual step.  Measured per
// process and cached in memory and on disk by device, geometry, precision
// and a hash of the impulse-response table.
constexpr int kTuneVersion = 4;  // bump when the kernels or the choices change meaning

struct Shape {
  int h_rows = 0, ht_rows = 0, tsh = 0, h_loadw = 0, tv = 0;
  int runs_h = 0, runs_ht = 0;  // FP32: run-packed (1) or per-tile (0) kernel
  bool operator==(const Shape& o) const {
    return h_rows == o.h_rows && ht_rows == o.ht_rows && tsh == o.tsh && h_loadw == o.h_loadw &&
           tv == o.tv && runs_h == o.runs_h && runs_ht == o.runs_ht;
  }
};

std::mutex g_tune_mu;
std::map<std::string, Shape> g_tune_cache;

std::string tune_key(const psoam_geom& g, int32_t sir_w, int32_t prec, const int32_t* t0,
                     const float* taps) {
  uint64_t h = 1469598103934665603ull;  // FNV-1a over the table bytes
  auto mix = [&h](const void* p, size_t n) {
    const unsigned char* b = (const unsigned char*)p;
    for (size_t i = 0; i < n; ++i) h = (h ^ b[i]) * 1099511628211ull;
  };
  const size_t ntab = (size_t)g.nz * g.f * g.f;
  mix(t0, ntab * sizeof(int32_t));
  mix(taps, ntab * (size_t)sir_w * sizeof(float));
  // the device: architecture and compute units
  int dev = 0;
  hipDeviceProp_t prop{};
  char arch[64] = "unknown";
  int cus = 0;
  if (hipGetDevice(&dev) == hipSuccess && hipGetDeviceProperties(&prop, dev) == hipSuccess) {
    std::snprintf(arch, sizeof arch, "%s", prop.gcnArchName);
    for (char* c = arch; *c; ++c)
      if (*c == ' ' || *c == '\t') *c = '_';
    cus = prop.multiProcessorCount;
  }
  char buf[320];
  std::snprintf(buf, sizeof buf, "v%d %s %d %d %d %d %d %d %d %d %d %d %d %016llx", kTuneVersion,
                arch, cus, g.nx, g.ny, g.nz, g.n_species, g.n_pulses, g.nt, g.f, g.phi_per_voxel,
                sir_w, prec, (unsigned long long)h);
  return buf;
}

// the disk cache: PSOAM_TUNE_CACHE (empty: none), else $HOME/.cache/psoam/tune.txt
std::string tune_file() {
  if (const char* e = std::getenv("PSOAM_TUNE_CACHE")) return e;
  const char* home = std::getenv("HOME");
  if (!home || !home[0]) return "";
  return std::string(home) + "/.cache/psoam/tune.txt";
}

// the last line "key<TAB>h_rows ht_rows tsh h_loadw tv runs_h runs_ht" of the file for key
bool disk_lookup(const std::string& key, Shape& out) {
  const std::string path = tune_file();
  if (path.empty()) return false;
  std::FILE* f = std::fopen(path.c_str(), "r");
  if (!f) return false;
  bool found = false;
  char line[512];
  while (std::fgets(line, sizeof line, f)) {
    char* tab = std::strchr(line, '\t');
    if (!tab || (size_t)(tab - line) != key.size() || key.compare(0, key.size(), line, key.size()))
      continue;
    Shape s;
    if (std::sscanf(tab + 1, "%d %d %d %d %d %d %d", &s.h_rows, &s.ht_rows, &s.tsh, &s.h_loadw,
                    &s.tv, &s.runs_h, &s.runs_ht) == 7 &&
        s.tv >= 0 && s.tv < tv_tile_count()) {
      out = s;
      found = true;
    }
  }
  std::fclose(f);
  return found;
}

void disk_store(const std::string& key, const Shape& s) {
  const std::string path = tune_file();
  if (path.empty()) return;
  // make the parent folders (best effort)
  for (size_t i = 1; i < path.size(); ++i)
    if (path[i] == '/') (void)::mkdir(path.substr(0, i).c_str(), 0755);
  std::FILE* f = std::fopen(path.c_str(), "a");
  if (!f) return;
  std::fprintf(f, "%s\t%d %d %d %d %d %d %d\n", key.c_str(), s.h_rows, s.ht_rows, s.tsh,
               s.h_loadw, s.tv, s.runs_h, s.runs_ht);
  std::fclose(f);
}

Shape shape_of(const psoam_plan* P) {
  Shape s;
  s.h_rows = P->fwd.lds_ok ? P->fwd.rows : 0;
  s.ht_rows = P->adj.lds_ok ? P->adj.rows : 0;
  s.tsh = P->tsh;
  s.h_loadw = P->fwd.lds_ok && P->fwd.loadw > 0 ? 1 : 0;
  s.tv = P->tv_tile;
  s.runs_h = P->fwd.runs32 ? 1 : 0;
  s.runs_ht = P->adj.runs32 ? 1 : 0;
  return s;
}

// average ms of `launch` over kReps launches after one warm-up
template <class F>
int time_launches(F&& launch, int reps, hipStream_t s, double* ms) {
  hipEvent_t e0 = nullptr, e1 = nullptr;
  hipError_t e = hipEventCreate(&e0);
  if (e == hipSuccess) e = hipEventCreate(&e1);
  if (e == hipSuccess) e = launch(0);
  if (e == hipSuccess) e = hipEventRecord(e0, s);
  for (int i = 0; i < reps && e == hipSuccess; ++i) e = launch(i + 1);
  if (e == hipSuccess) e = hipEventRecord(e1, s);
  if (e == hipSuccess) e = hipEventSynchronize(e1);
  float t = 0.0f;
  if (e == hipSuccess) e = hipEventElapsedTime(&t, e0, e1);
  if (e0) (void)hipEventDestroy(e0);
  if (e1) (void)hipEventDestroy(e1);
  if (e != hipSuccess) return hip_fail(e, "autotune: timing launch");
  *ms = (double)t / reps;
  return PSOAM_OK;
}

// average ms of the band kernel of direction dir in the solver's form
// (dir 0: H with the residual epilogue, dir 1: S^T H^T), one warm-up launch
int time_band(psoam_plan* P, int dir, hipStream_t s, double* ms) {
  SolveBufs B;
  if (int rc = ensure_solve_ws(P, B)) return rc;
  return time_launches(
      [&](int) {
        return dir == 0 ? launch_band(P, 1, nullptr, nullptr, P->d_partial, s)
                        : launch_band(P, 2, B.g, nullptr, nullptr, s);
      },
      3, s, ms);
}

// average ms of one TV dual step with the plan's tile, on zeroed duals
int time_tv(psoam_plan* P, hipStream_t s, double* ms) {
  SolveBufs B;
  if (int rc = ensure_solve_ws(P, B)) return rc;
  const size_t sv = P->c_elems();
  for (float* b : {B.u[0], B.u[1], B.u[2]}) PSOAM_HIP(hipMemsetAsync(b, 0, sizeof(float) * 3 * sv, s));
  PSOAM_HIP(hipMemsetAsync(B.zb, 0, sizeof(float) * sv, s));
  return time_launches(
      [&](int i) {
        float* nxt = B.u[i % 3];
        const float* cur = B.u[(i + 2) % 3];
        const float* prev = B.u[(i + 1) % 3];
        return launch_tv_step(P, nxt, B.zb, cur, prev, 0.5f, 0.08f, 1.0f, s);
      },
      10, s, ms);
}

// a plan built with the given launch shape (0 entries: the plan's own rules)
int build_shaped(const psoam_geom* g, const psoam_species* sp, const float* phi,
                 const int32_t* t0, const float* taps, int32_t sir_w, int32_t prec,
                 hipStream_t s, const Shape& want, psoam_plan** out) {
  const bool fp32 = prec == PSOAM_FP32;
  set_tune_choice(want.h_rows, want.ht_rows, want.tsh, want.h_rows ? want.h_loadw : -1,
                  fp32 ? want.runs_h : -1, fp32 ? want.runs_ht : -1);
  const int rc = create_plan(g, sp, phi, t0, taps, sir_w, prec, s, out);
  clear_tune_choice();
  if (rc == PSOAM_OK) (*out)->tv_tile = want.tv;
  return rc;
}

int create_tuned(const psoam_geom* g, const psoam_species* sp, const float* phi,
                 const int32_t* t0, const float* taps, int32_t sir_w, int32_t prec,
                 hipStream_t s, psoam_plan** out, psoam_tune_report* rep) {
  psoam_tune_report r{};
  auto done = [&](psoam_plan* P) {
    const Shape got = shape_of(P);
    r.h_rows = got.h_rows;
    r.ht_rows = got.ht_rows;
    r.ht_shift = got.tsh;
    r.h_loaders = got.h_loadw ? 4 : 0;
    tv_tile_dims(got.tv, r.tv_tile);
    r.fp32_runs[0] = got.runs_h;
    r.fp32_runs[1] = got.runs_ht;
    if (rep) *rep = r;
    *out = P;
    return PSOAM_OK;
  };
  if (!out) return fail(PSOAM_EINVAL, "plan_create_tuned: out is NULL");
  *out = nullptr;
  if (!g || !sp || !phi || !t0 || !taps) return fail(PSOAM_EINVAL, "plan_create_tuned: NULL argument");
  psoam_plan* P = nullptr;
  if (g->separable != 0) {
    if (int rc = create_plan(g, sp, phi, t0, taps, sir_w, prec, s, &P)) return rc;
    return done(P);
  }
  if (sir_w < 1 || sir_w > 64 || g->nz <= 0 || g->f <= 0)
    return create_plan(g, sp, phi, t0, taps, sir_w, prec, s, out);  // its own errors
  const std::string key = tune_key(*g, sir_w, prec, t0, taps);
  {
    Shape want;
    int from = 0;
    {
      std::lock_guard<std::mutex> lk(g_tune_mu);
      // PSOAM_TUNE_MEMO=0 skips this process's cache (tests read the disk's)
      const char* memo = std::getenv("PSOAM_TUNE_MEMO");
      auto it = memo && memo[0] == '0' ? g_tune_cache.end() : g_tune_cache.find(key);
      if (it != g_tune_cache.end()) {
        want = it->second;
        from = 1;
      } else if (disk_lookup(key, want)) {
        g_tune_cache[key] = want;
        from = 2;
      }
    }
    if (from) {
      if (int rc = build_shaped(g, sp, phi, t0, taps, sir_w, prec, s, want, &P)) return rc;
      r.from_cache = from;
      return done(P);
    }
  }
  // the plan's own choice, timed
  if (int rc = create_plan(g, sp, phi, t0, taps, sir_w, prec, s, &P)) return rc;
  const Shape base = shape_of(P);
  double h_best = 0.0, ht_best = 0.0, tv_best = 0.0;
  int rc = PSOAM_OK;
  const bool fp32 = prec == PSOAM_FP32;
  if (base.h_rows || fp32) rc = time_band(P, 0, s, &h_best);
  if (rc == PSOAM_OK && (base.ht_rows || fp32)) rc = time_band(P, 1, s, &ht_best);
  if (rc == PSOAM_OK) rc = time_tv(P, s, &tv_best);  // the default tile
  r.tv_ms_default = tv_best;
  Shape best = base;
  // TV tiles: the same plan, another tile
  for (int t = 1; t < tv_tile_count() && rc == PSOAM_OK; ++t) {
    P->tv_tile = t;
    double ms = 0.0;
    rc = time_tv(P, s, &ms);
    if (rc == PSOAM_OK && ms < tv_best * 0.995) {
      tv_best = ms;
      best.tv = t;
    }
  }
  P->tv_tile = base.tv;
  if (rc != PSOAM_OK) {
    free_plan(P);
    return rc;
  }
  r.candidates = 1;
  r.h_ms_default = h_best;
  r.ht_ms_default = ht_best;
  // alternatives: the other row counts and loader-wave settings for H; the
  // other row counts and shifts for H^T (each timed on the direction it changes)
  std::vector<std::pair<Shape, int>> alts;
  if (base.h_rows)
    for (int rows : {4, 8, 12})
      for (int lw : {0, 1})
        if ((rows != base.h_rows || lw != base.h_loadw) && !(rows != 8 && lw == 1))
          alts.push_back({Shape{rows, base.ht_rows, base.tsh, lw, base.tv}, 0});
  if (base.ht_rows)
    for (int rows : {4, 8, 12})
      for (int tsh : {0, 4})
        if (rows != base.ht_rows || tsh != base.tsh)
          alts.push_back({Shape{base.h_rows, rows, tsh, base.h_loadw, base.tv}, 1});
  if (fp32 && (base.runs_h || base.runs_ht)) {
    // the other FP32 kernel, for both directions at once (timed on each)
    Shape o = base;
    o.runs_h = base.runs_h ? 0 : 1;
    o.runs_ht = base.runs_ht ? 0 : 1;
    alts.push_back({o, 2});
  }
  for (const auto& a : alts) {
    psoam_plan* Q = nullptr;
    if ((rc = build_shaped(g, sp, phi, t0, taps, sir_w, prec, s, a.first, &Q))) break;
    const Shape got = shape_of(Q);
    double ms = 0.0, ms2 = 0.0;
    if (got == a.first) {  // it fitted
      rc = time_band(Q, a.second == 2 ? 0 : a.second, s, &ms);
      if (rc == PSOAM_OK && a.second == 2) rc = time_band(Q, 1, s, &ms2);
      ++r.candidates;
    }
    free_plan(Q);
    if (rc != PSOAM_OK) break;
    if (!(got == a.first)) continue;
    if (a.second == 2) {
      if (ms < h_best) {
        h_best = ms;
        best.runs_h = a.first.runs_h;
      }
      if (ms2 < ht_best) {
        ht_best = ms2;
        best.runs_ht = a.first.runs_ht;
      }
      continue;
    }
    if (a.second == 0 && ms < h_best) {
      h_best = ms;
      best.h_rows = a.first.h_rows;
      best.h_loadw = a.first.h_loadw;
    }
    if (a.second == 1 && ms < ht_best) {
      ht_best = ms;
      best.ht_rows = a.first.ht_rows;
      best.tsh = a.first.tsh;
    }
  }
  if (rc != PSOAM_OK) {
    free_plan(P);
    return rc;
  }
  r.candidates += tv_tile_count() - 1;
  r.h_ms = h_best;
  r.ht_ms = ht_best;
  r.tv_ms = tv_best;
  {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_tune_cache[key] = best;
    disk_store(key, best);
  }
  if (best.h_rows == base.h_rows && best.ht_rows == base.ht_rows && best.tsh == base.tsh &&
      best.h_loadw == base.h_loadw && best.runs_h == base.runs_h && best.runs_ht == base.runs_ht) {
    P->tv_tile = best.tv;
    return done(P);
  }
  free_plan(P);
  P = nullptr;
  if ((rc = build_shaped(g, sp, phi, t0, taps, sir_w, prec, s, best, &P))) return rc;
  return done(P);
}

}  // namespace
}  // namespace psoam

extern "C" {

int psoam_plan_create(const psoam_geom* g, const psoam_species* sp, const float* phi,
                      const int32_t* sir_t0, const float* sir_taps, int32_t sir_w,
                      int32_t prec, void* stream, psoam_plan** out) {
  return create_plan(g, sp, phi, sir_t0, sir_taps, sir_w, prec, S(stream), out);
}

int psoam_plan_create_tuned(const psoam_geom* g, const psoam_species* sp, const float* phi,
                            const int32_t* sir_t0, const float* sir_taps, int32_t sir_w,
                            int32_t prec, void* stream, psoam_plan** out,
                            psoam_tune_report* report) {
  return create_tuned(g, sp, phi, sir_t0, sir_taps, sir_w, prec, S(stream), out, report);
}

int psoam_plan_destroy(psoam_plan* plan) {
  free_plan(plan);
  return PSOAM_OK;
}

int psoam_plan_geom(const psoam_plan* plan, psoam_geom* g) {
  if (!plan || !g) return fail(PSOAM_EINVAL, "plan_geom: NULL argument");
  *g = plan->g;
  return PSOAM_OK;
}

int psoam_apply_A(const psoam_plan* plan, const float* c, float* y, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!c || !y) return fail(PSOAM_EINVAL, "apply_A: NULL argument");
  if (((uintptr_t)y & 15) != 0) return fail(PSOAM_EINVAL, "apply_A: y must be 16-byte aligned");
  if (plan->inner) {
    PSOAM_HIP(launch_switch_fwd(plan->inner, c, S(stream)));
    PSOAM_HIP(launch_band(plan->inner, 0, plan->d_h, nullptr, nullptr, S(stream)));
    PSOAM_HIP(launch_sep_expand(plan, y, plan->d_h, S(stream)));
    return PSOAM_OK;
  }
  if (plan->fact) {
    PSOAM_HIP(launch_switch_fwd(plan, c, S(stream)));
    PSOAM_HIP(launch_band(plan, 0, plan->d_fq, nullptr, nullptr, S(stream)));
    PSOAM_HIP(launch_eir_rows(plan, 0, y, plan->d_fq, nullptr, nullptr, S(stream)));
    return PSOAM_OK;
  }
  PSOAM_HIP(launch_switch_fwd(plan, c, S(stream)));
  PSOAM_HIP(launch_band(plan, 0, y, nullptr, nullptr, S(stream)));
  return PSOAM_OK;
}

int psoam_apply_AT(const psoam_plan* plan, const float* y, float* c, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!c || !y) return fail(PSOAM_EINVAL, "apply_AT: NULL argument");
  if (plan->inner) {
    PSOAM_HIP(launch_sep_contract(plan, plan->d_rt, y, S(stream)));
    PSOAM_HIP(launch_pack_r(plan->inner, plan->d_rt, S(stream)));
    PSOAM_HIP(launch_band(plan->inner, 2, c, nullptr, nullptr, S(stream)));
    return PSOAM_OK;
  }
  if (plan->fact) {
    if (eir_pack_fits(plan, false)) {
      PSOAM_HIP(launch_eir_pack(plan, y, nullptr, false, S(stream)));
    } else {
      PSOAM_HIP(launch_eir_rows(plan, 1, plan->d_fq, y, nullptr, nullptr, S(stream)));
      PSOAM_HIP(launch_pack_r(plan, plan->d_fq, S(stream)));
    }
    PSOAM_HIP(launch_band(plan, 2, c, nullptr, nullptr, S(stream)));
    return PSOAM_OK;
  }
  PSOAM_HIP(launch_pack_r(plan, y, S(stream)));
  PSOAM_HIP(launch_band(plan, 2, c, nullptr, nullptr, S(stream)));
  return PSOAM_OK;
}

int psoam_prox_l1(float* x, const float* z, int64_t n, float thresh, int32_t nonneg,
                  void* stream) {
  if (n < 0) return fail(PSOAM_EINVAL, "prox_l1: n < 0");
  if (!(thresh >= 0.0f) || !std::isfinite(thresh))
    return fail(PSOAM_EINVAL, "prox_l1: thresh must be finite and >= 0");
  if (n > 0 && (!x || !z)) return fail(PSOAM_EINVAL, "prox_l1: NULL argument");
  PSOAM_HIP(launch_prox_l1(x, z, n, thresh, nonneg, S(stream)));
  return PSOAM_OK;
}

size_t psoam_prox_tv_ws_bytes(const psoam_plan* plan) {
  if (!plan) return 0;
  return sizeof(float) * plan->c_elems() * 10 + 4 * 256;
}

int psoam_prox_tv(const psoam_plan* plan, float* x, const float* z, float theta,
                  int32_t n_inner, int32_t nonneg, void* ws, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!x || !z || !ws) return fail(PSOAM_EINVAL, "prox_tv: NULL argument");
  if (!(theta >= 0.0f) || !std::isfinite(theta))
    return fail(PSOAM_EINVAL, "prox_tv: theta must be finite and >= 0");
  if (n_inner < 0) return fail(PSOAM_EINVAL, "prox_tv: n_inner < 0");
  if (((uintptr_t)ws & 255) != 0) return fail(PSOAM_EINVAL, "prox_tv: ws must be 256-byte aligned");
  const size_t sv = plan->c_elems();
  auto align = [](float* p) { return (float*)(((uintptr_t)p + 255) & ~(uintptr_t)255); };
  float* u0 = (float*)ws;
  float* u1 = align(u0 + 3 * sv);
  float* u2 = align(u1 + 3 * sv);
  float* w = align(u2 + 3 * sv);
  float* u[3] = {u0, u1, u2};
  // z and x may alias: keep z intact until the final map, which reads z[v] only at v
  return tv_prox_core(plan, x, z, theta, n_inner, nonneg ? 1 : 0, 0.0f, u, w, nullptr, false,
                      nullptr, S(stream));
}

size_t psoam_prox_r3_ws_bytes(const psoam_plan* plan) {
  if (!plan) return 0;
  return r3_ws_bytes(plan);
}

int psoam_prox_r3(const psoam_plan* plan, float* x, const float* z, float theta_tv,
                  float theta_tvs, float theta_l1, int32_t n_inner, void* ws, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!x || !z || !ws) return fail(PSOAM_EINVAL, "prox_r3: NULL argument");
  const float th[3] = {theta_tv, theta_tvs, theta_l1};
  for (float t : th)
    if (!(t >= 0.0f) || !std::isfinite(t))
      return fail(PSOAM_EINVAL, "prox_r3: thresholds must be finite and >= 0");
  if (n_inner < 0) return fail(PSOAM_EINVAL, "prox_r3: n_inner < 0");
  if (((uintptr_t)ws & 255) != 0) return fail(PSOAM_EINVAL, "prox_r3: ws must be 256-byte aligned");
  return r3_prox_core(plan, x, z, th, n_inner, r3_carve(plan, ws), false, S(stream));
}

int psoam_plan_create_acoustic(const psoam_geom* g, const int32_t* sir_t0, const float* sir_taps,
                               int32_t sir_w, int32_t prec, void* stream, psoam_plan** out) {
  return create_plan_acoustic(g, sir_t0, sir_taps, sir_w, prec, S(stream), out);
}

int psoam_plan_create_factorised(const psoam_geom* g, const psoam_species* sp, const float* phi,
                                 const float* spr, const float* eir, const psoam_shell* sh,
                                 int32_t prec, void* stream, psoam_plan** out) {
  return create_plan_factorised(g, sp, phi, spr, eir, sh, prec, S(stream), out);
}

int psoam_unmix(const psoam_plan* plan, const float* b, float* c, const psoam_solve_opts* o,
                psoam_solve_stats* st, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  return solve_one(const_cast<psoam_plan*>(plan), kOpUnmix, b, c, o, st, S(stream));
}

int psoam_solve(const psoam_plan* plan, const float* p, float* c, const psoam_solve_opts* o,
                psoam_solve_stats* st, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  return solve_one(const_cast<psoam_plan*>(plan), kOpA, p, c, o, st, S(stream));
}

int psoam_solve_batch(int32_t n, const psoam_plan* const* plans, const float* const* p,
                      float* const* c, const psoam_solve_opts* o, psoam_solve_stats* st,
                      void* stream) {
  if (n < 0) return fail(PSOAM_EINVAL, "solve_batch: n < 0");
  if (n == 0) return PSOAM_OK;
  if (!plans || !p || !c || !o) return fail(PSOAM_EINVAL, "solve_batch: NULL argument");
  for (int i = 0; i < n; ++i) {
    if (!plans[i]) return fail(PSOAM_EINVAL, "solve_batch: NULL plan");
    if (int rc = check_opts(p[i], c[i], &o[i])) return rc;
  }
  // Captured iterations need distinct plans (each owns its operand buffers and
  // scalars) and no host decisions inside the loop; other problems are solved
  // one after another on the caller's stream.
  bool distinct = true;
  for (int i = 0; i < n && distinct; ++i)
    for (int j = 0; j < i; ++j)
      if (plans[i] == plans[j]) distinct = false;
  std::vector<BatchItem> items;
  for (int i = 0; i < n; ++i) {
    const psoam_solve_opts* oi = &o[i];
    // host decisions inside the loop (stopping tests, a trace) are needed
    // unless the tests run on the device (device_stop)
    const bool host_tests = oi->eps1 > 0.0 || oi->eps2 > 0.0 || oi->trace;
    const bool graphable = distinct && (!host_tests || oi->device_stop) && !oi->warm_inner &&
                           oi->k1 >= 2;
    if (!graphable) {
      const int rc = solve_one(const_cast<psoam_plan*>(plans[i]), kOpA, p[i], c[i], oi,
                               st ? &st[i] : nullptr, S(stream));
      if (rc) return rc;
      continue;
    }
    BatchItem it;
    it.P = const_cast<psoam_plan*>(plans[i]);
    it.p = p[i];
    it.c = c[i];
    it.o = oi;
    it.st = st ? &st[i] : nullptr;
    it.stats = fresh_stats();
    it.alpha1 = 0.0;
    it.remaining = 0;
    it.dev = oi->device_stop != 0 && host_tests;
    it.need_obj = oi->eps1 > 0.0 || oi->trace != nullptr;
    it.tst = StopTest{oi->eps1, oi->eps2, oi->lambda_tv, oi->lambda_l1, oi->lambda_tvs,
                      it.need_obj ? 1 : 0, it.P->inner ? 1 : 0, oi->lambda_tvs > 0.0 ? 1 : 0};
    if (int rc = ensure_solve_ws(it.P, it.B)) return rc;
    it.RB = R3Bufs{};
    if (oi->lambda_tvs > 0.0)
      if (int rc = ensure_r3_ws(it.P, it.RB)) return rc;
    items.push_back(it);
  }
  if (items.empty()) return PSOAM_OK;
  return solve_batch_graph(items, S(stream));
}

int psoam_plan_stats(const psoam_plan* plan, psoam_plan_info* info) {
  if (!plan || !info) return fail(PSOAM_EINVAL, "plan_stats: NULL argument");
  if (plan->inner) plan = plan->inner;  // the contraction of the separable form
  const bool half = plan->prec != PSOAM_FP32;
  const int64_t tile = half ? 16 * 32 : 16 * 4;
  const BandTable* T[2] = {&plan->fwd, &plan->adj};
  for (int d = 0; d < 2; ++d) {
    info->useful_macs[d] = (int64_t)T[d]->useful_macs;
    const bool staged = half && T[d]->lds_ok;
    info->chunks[d] = staged ? T[d]->l_chunks : T[d]->n_chunks;
    info->executed_macs[d] = (int64_t)info->chunks[d] * tile;
    info->lds_bytes[d] = staged ? (int64_t)T[d]->lds_bytes : 0;
    info->lds_rows[d] = staged ? T[d]->rows : 0;
  }
  info->operand_bytes[0] = (int64_t)plan->bq_bytes;
  info->operand_bytes[1] = (int64_t)plan->rq_bytes;
  return PSOAM_OK;
}

int psoam_band_only(const psoam_plan* plan, int32_t dir, float* out, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!out || (dir != 0 && dir != 1)) return fail(PSOAM_EINVAL, "band_only: bad argument");
  if (dir == 0 && ((uintptr_t)out & 15) != 0)
    return fail(PSOAM_EINVAL, "band_only: y must be 16-byte aligned");
  if (plan->inner) plan = plan->inner;  // the contraction of the separable form (S columns)
  PSOAM_HIP(launch_band(plan, dir == 0 ? 0 : 2, out, nullptr, nullptr, S(stream)));
  return PSOAM_OK;
}

int psoam_prox_tv_noalloc(const psoam_plan* plan, float* x, const float* z, float theta,
                          int32_t n_inner, int32_t nonneg, void* stream) {
  if (int rc = check_plan(plan)) return rc;
  if (!x || !z) return fail(PSOAM_EINVAL, "prox_tv_noalloc: NULL argument");
  if (!(theta >= 0.0f) || !std::isfinite(theta))
    return fail(PSOAM_EINVAL, "prox_tv_noalloc: theta must be finite and >= 0");
  if (n_inner < 0) return fail(PSOAM_EINVAL, "prox_tv_noalloc: n_inner < 0");
  const size_t sv = plan->c_elems();
  const size_t set = noalloc_set_floats(sv);
  if (3 * set > kNoAllocFloats)
    return fail(PSOAM_EINVAL, "prox_tv_noalloc: S*Ny*Nx*Nz = " + std::to_string(sv) +
                                  " exceeds the static dual buffer (at most 3728256 "
                                  "species-voxels); use psoam_prox_tv with a workspace");
  float* base = nullptr;
  if (int rc = noalloc_scratch(plan->device, &base)) return rc;
  float* u[3] = {base, base + set, base + 2 * set};
  // the dual iteration writes every dual it reads (the first step starts from
  // u = 0 without reading memory), so the buffer needs no clearing
  return tv_prox_core(plan, x, z, theta, n_inner, nonneg ? 1 : 0, 0.0f, u, nullptr, nullptr,
                      false, nullptr, S(stream));
}

const char* psoam_last_error(void) { return last_error_cstr(); }

}  // extern "C"
