// Internal declarations of the psoam library (not part of the C ABI).
//
// Data layout in HBM (all padded operands have zeroed borders that are never
// written, so the band kernels need no bounds checks on their reads):
//   16-bit operands (BF16/FP16):  Q[Yp][Xp][Lo][Kp][8]   (8 consecutive
//       samples of the contracted axis -- depth z for H, time t for H^T --
//       form one 16-byte "octet"; the Kp pulses of one octet are adjacent so
//       16 pulses x 16 bytes of one octet are 256 contiguous bytes)
//   FP32 operands:                Q[Yp][Xp][L][Kp]       (pulses adjacent)
// Yp = Ny + 2R, Xp = roundup(Nx, 16) + 2R: a scan/voxel position (iy, ix)
// reads its whole F x F footprint at padded rows iy..iy+F-1, columns
// ix..ix+F-1.  Kp = K rounded up to 16 (one matrix-core column block).
#pragma once

#include <hip/hip_runtime.h>

#include <cstddef>
#include <cstdint>
#include <string>
#include <vector>

#include "psoam.h"

namespace psoam {

constexpr int kMaxSpecies = 8;
constexpr int kWaveLanes = 64;
constexpr int kPosPerWave = 8;       // scan/voxel positions owned by one wave
constexpr int kPadX = 16;            // Nx is padded up to a multiple of this
constexpr int kWavesPerBlock = 4;    // consecutive output tiles of one position block
constexpr float kFp16Scale = 256.0f; // FP16 operand scale when no per-call scale is given
constexpr int kLdsPos = 16;          // staged kernel: positions per wave
constexpr int kLdsMaxBytes = 160 * 1024;
constexpr int kRunMax = 4;           // longest sliding run (chunks) of the staged kernel
constexpr int kMaxEir = 32;          // taps of the electrical impulse response (factorised form)
constexpr int kMaxEirNt = 4096;      // longest A-scan of the factorised form (LDS row buffer)

// electrical impulse response of the factorised form: y[t] = sum_j v[j] q[t - j + origin]
struct EirParams {
  int n, origin;
  float v[kMaxEir];
  const int* gate = nullptr;  // device stop flag of the solve (set per launch), or null
};

// Photo-switching coefficients in the form the kernels evaluate:
//   S_v[k][s] = phi_v * (a[s] + b[s] * exp(-k * phi_v^gamma * inv_tau[s]))
struct SwitchParams {
  int ns;
  int nk;
  int per_voxel;
  int diag;        // 1: S_v[k][s] = phi_v if k == s else 0 (inner plan of the separable form)
  float gamma;
  float a[kMaxSpecies];
  float b[kMaxSpecies];
  float inv_tau[kMaxSpecies];
};

// One direction of the band contraction (H, or H^T viewed as a correlation
// with flipped offsets): for every output tile of 16 rows, a list of chunks;
// a chunk is 4 "groups", each naming one octet (16-bit) or one sample (FP32)
// of the contracted axis at one lateral offset, plus the matching 16 x 32
// (16-bit) or 16 x 4 (FP32) block of the band matrix, pre-packed in the
// lane order of the matrix-core instruction.
struct BandTable {
  int n_mtiles = 0;          // output tiles of 16 rows
  int m_rows = 0;            // valid output rows (Nt for H, Nz for H^T)
  int n_chunks = 0;
  std::vector<int> h_start;  // [n_mtiles + 1]
  int* d_start = nullptr;
  int* d_off = nullptr;      // [n_chunks * 4] element offsets from the position base
  void* d_a = nullptr;       // packed band values (hi part)
  void* d_a_lo = nullptr;    // low-order parts for the split precisions
  size_t useful_macs = 0;    // nonzero band entries covered (per position and pulse)
  // staged (LDS) variant, 16-bit operands: chunks listed per (tile, dy)
  bool lds_ok = false;
  int rows = 4;                // output rows (waves) per workgroup: 4, 8 or 12
  int l_chunks = 0;
  int max_oct = 0;             // widest staged octet window
  size_t lds_bytes = 0;        // dynamic LDS per workgroup
  int* d_lstart = nullptr;     // [n_mtiles * F + 1] first run of each (tile, dy)
  uint32_t* d_lgrp = nullptr;  // [n_runs * 4]  octet << 16 | dx at the run's first chunk
  uint32_t* d_win = nullptr;   // [n_mtiles * (F + rows - 1)]  obase << 16 | ocnt
  void* d_la = nullptr;
  void* d_la_lo = nullptr;
  int* d_order = nullptr;      // [n_mtiles] tiles by decreasing chunk count
  int n_runs = 0;
  int max_runs = 0;            // most runs of one output tile (LDS run table)
  int* d_rinfo = nullptr;      // [n_runs * 2] run length, first chunk
  int loadw = 0;               // > 0: loader waves beside the contracting ones (staged H)
  // 1: the last 16-pulse block holds at most 8 pulses and the staged kernel
  // runs it as 8 pulses x pairs of positions (half the products and staging)
  int half = 0;
  // FP32 plans: the run tables (no windows) feed the global-operand run kernel
  bool runs32 = false;
};

// LDS bytes of the staged kernel's per-tile tables: row windows (F + rows - 1),
// run bounds (F + 1), run records (4 group words + 2 ints each)
inline size_t lds_meta_bytes(int F, int rows, int max_runs) {
  return sizeof(uint32_t) * ((size_t)(F + rows - 1) + (F + 1) + 6 * (size_t)max_runs) + 16;
}

struct Workspace {
  size_t bytes = 0;
  void* base = nullptr;
};

}  // namespace psoam

struct psoam_plan {
  psoam_geom g;
  psoam_species sp_in;
  psoam::SwitchParams sw;
  int prec;
  int R, F, W;
  int Kp, NB;       // padded pulses, 16-pulse column blocks
  int Yp, Xp;
  int Lz, Lt;       // contracted lengths of the H operand (z) and H^T operand (t), in samples
  int tsh = 0;      // 16-bit H^T operand: sample t is stored at t + tsh (0 or 4)
  int tv_tile = 0;  // tile shape of the TV dual step (index into the kernel's shape list)
  size_t ps_b, ps_r;  // elements per padded position of the H / H^T operands
  int device;
  float* d_phi = nullptr;
  float* d_stab = nullptr;   // [Nz][Kp][S] when phi is per depth
  float* d_stab_t = nullptr; // [K][S][Nz]: the same table with depth fastest (per-voxel kernels)
  float* d_stab_o = nullptr; // [Lz/8][S][Kp][8]: per depth octet, pulses then depths (16-bit S)
  void* d_bq = nullptr;      // H operand (hi)
  void* d_bq_lo = nullptr;
  void* d_rq = nullptr;      // H^T operand (hi)
  void* d_rq_lo = nullptr;
  size_t bq_bytes = 0, rq_bytes = 0;
  psoam::BandTable fwd, adj;
  // solver scratch (allocated on first use, grown as needed)
  psoam::Workspace solve_ws;
  double* d_partial = nullptr;  // per-wave / per-block FP64 partial sums
  size_t n_partial = 0;
  double* d_scalars = nullptr;  // small FP64 results (reductions)
  int* d_ctl = nullptr;         // device stopping tests: stopped, iterations, diverged, index
  double* d_trace = nullptr;    // objective per iteration under device stopping tests
  size_t n_trace = 0;
  // duals of the full regulariser's prox (TV(S c) term), allocated on first use
  psoam::Workspace r3_ws;
  psoam::Workspace yc_ws;  // A c of the solve's iterate (objective by the momentum recurrence)
  // max over voxels of the largest eigenvalue of S_v^T S_v (FP64, at creation)
  double smax2 = 0.0;
  // separable switching (fluence-independent rate): S_v[k][s] = phi_v T[k][s].
  // The contraction runs in `inner`, a plan over the S species with
  // S'_v = phi_v I; this plan keeps the true switching data for the prox
  // steps and owns the small pulse-expansion buffers.
  psoam_plan* inner = nullptr;
  float* d_T = nullptr;       // [K][S]
  float sep_g[psoam::kMaxSpecies * psoam::kMaxSpecies] = {};  // G = T^T T, [S][S]
  float* d_h = nullptr;       // [S][Ny][Nx][Nt]: H of phi c_s
  float* d_rt = nullptr;      // [S][Ny][Nx][Nt]: T^T r, the adjoint's input
  float* d_q = nullptr;       // [S][Ny][Nx][Nt]: T^T p of the current solve
  // factorised acoustic operator: the band holds the shell sums Lambda, the
  // impulse response runs as a separate pass over the A-scans
  int fact = 0;
  psoam::EirParams eir{};
  float* d_fq = nullptr;      // [K][Ny][Nx][Nt]: shell sums q = Lambda S c (and V^T r)
  // FP16 operands (FP16 plans with operands, else null): power-of-two scales
  // chosen on the device for every operand written, from FP32 max-abs
  // reductions and bounds that hold for every element, so no operand
  // overflows FP16 whatever the units of c and p:
  //   [0] s_b, [1] 1/s_b (H operand), [2] s_r, [3] 1/s_r (H^T operand),
  //   [4] max |x| of the last switching input, [5] max |p| of the solve
  float* d_f16 = nullptr;
  unsigned* d_f16acc = nullptr;  // [2] float bits of running maxima, zero between uses
  double srow = 0.0;  // max over voxels and pulses of sum_s |S_v[k][s]|
  double hrow = 0.0;  // max over output samples of the sum of |h| over (z, dy, dx)
  double eir_l1 = 0.0;  // sum_j |v[j]| (factorised form)
  size_t h_elems() const { return (size_t)g.n_species * g.ny * g.nx * g.nt; }
  size_t y_elems() const { return (size_t)g.n_pulses * g.ny * g.nx * g.nt; }
  size_t c_elems() const { return (size_t)g.n_species * g.ny * g.nx * g.nz; }
  size_t v_elems() const { return (size_t)g.ny * g.nx * g.nz; }
};

namespace psoam {

// Launch-shape choice for the next plan built on this thread (the
// autotuner's lever): output rows per staged workgroup for H (rows_fwd) and
// H^T (rows_adj), 4, 8 or 12, the H^T operand shift, 0 or 4, H's loader
// waves, 0 (off) or 1 (on where they can run), and for FP32 plans the kernel
// of H and of H^T, 0 (per-tile) or 1 (run-packed); any other value leaves
// that choice to the plan's own rules.  A choice that does not fit is ignored.
void set_tune_choice(int rows_fwd, int rows_adj, int tsh, int loadw_fwd, int runs_fwd = -1,
                     int runs_adj = -1);
void clear_tune_choice();

// Device stop gate of the calling thread: while a solve with device-side
// stopping tests enqueues its iterations, every kernel launched on this
// thread receives the solve's stop flag and returns at once when it is set.
void set_gate(const int* g);
const int* gate_now();

// thread-local error message
void set_error(const std::string& msg);
int fail(int code, const std::string& msg);
int hip_fail(hipError_t e, const char* what);
#define PSOAM_HIP(call)                                   \
  do {                                                    \
    hipError_t _e = (call);                               \
    if (_e != hipSuccess) return psoam::hip_fail(_e, #call); \
  } while (0)

// kernel launchers (psoam_kernels.hip); all return hipError_t of the launch
hipError_t launch_switch_fwd(const psoam_plan* P, const float* c, hipStream_t s);
hipError_t launch_pack_r(const psoam_plan* P, const float* y, hipStream_t s);
// mode 0: y = H b (writes y);  mode 1: r = H b - p (p may be null), written into the
// H^T operand, sum r^2 into partial[]; mode 2: c = S^T H^T r (writes c).
// Mode 1 with yc: also A c = (H b + yc_beta yc) / (1 + yc_beta) (H b alone
// when yc_first) written back to yc, and the partials sum (A c - p)^2
hipError_t launch_band(const psoam_plan* P, int mode, float* out, const float* pmeas,
                       double* partial, hipStream_t s, float* yc = nullptr, double yc_beta = 0.0,
                       int yc_first = 0);
size_t band_partials(const psoam_plan* P, int mode);

hipError_t launch_prox_l1(float* x, const float* z, int64_t n, float thresh, int nonneg,
                          hipStream_t s);
// one inner step of the TV dual iteration:
//   w = z - grad^T eta ; u_next = clip(eta + inv_mu * grad w, -theta, theta),
//   eta = u_cur + beta (u_cur - u_prev)  (u_cur == null: eta = 0; u_prev == null: eta = u_cur)
hipError_t launch_tv_step(const psoam_plan* P, float* u_next, const float* z, const float* u_cur,
                          const float* u_prev, float beta, float inv_mu, float theta,
                          hipStream_t s);
// tile shapes of the TV dual step: count, and (y, x, z, threads) of shape i
int tv_tile_count();
void tv_tile_dims(int i, int* d);
// x = z - grad^T u (u may be null: x = z); then mode 0: as is, 1: max(x,0), 2: max(x - t1, 0)
hipError_t launch_tv_final(const psoam_plan* P, float* x, const float* z, const float* u,
                           int mode, float thresh1, hipStream_t s);
// x = a*x + b*y  elementwise (n floats)
hipError_t launch_axpby(float* out, const float* x, const float* y, float a, float b,
                        int64_t n, hipStream_t s);
// FP64 reductions, deterministic two-stage: results written to out[0..]
//   dot: out[0] = <x, y>   (y == x allowed)
hipError_t launch_dot(const float* x, const float* y, int64_t n, double* partial,
                      double* out, hipStream_t s);
hipError_t launch_sum_partials(const double* partial, size_t n, double* out, hipStream_t s);
//   out[0] = sum |grad c| (TV), out[1] = sum |c|
hipError_t launch_tv_l1_sums(const psoam_plan* P, const float* c, double* partial,
                             double* out, hipStream_t s);
// v = w / sqrt(*norm2)  (norm2 on device)
hipError_t launch_scale_by_rnorm(float* v, const float* w, const double* norm2, int64_t n,
                                 hipStream_t s);
hipError_t launch_fill(float* x, float v, int64_t n, hipStream_t s);
// xi_next = c_next + beta (c_next - c_prev); partial sums of |xi_next - xi|^2 and |xi|^2
hipError_t launch_momentum(float* xi, const float* c_next, const float* c_prev, float beta,
                           int64_t n, double* partial, hipStream_t s);
size_t reduce_blocks(int64_t n);
// xi = c_next + beta (c_next - c_prev) with beta from the device step state
// tst[0] = t_k, which is then advanced to t_{k+1} (captured iterations);
// partial (may be null): the partial sums of launch_momentum
hipError_t launch_momentum_dev(float* xi, const float* c_next, const float* c_prev, double* tst,
                               int literal, int64_t n, double* partial, hipStream_t s);
hipError_t launch_set_double(double* p, double v, hipStream_t s);
// device-side stopping tests of a solve (device_stop): ctl [4] ints, sc the
// plan's FP64 scalars; launch_select_copy copies the last iterate (a0 after
// an even number of iterations, a1 after an odd one) into out
struct StopTest {
  double eps1, eps2, lam_tv, lam_l1, lam_tvs;
  int need_obj;  // evaluate the objective (eps1 > 0 or a trace)
  int add_p2;    // data term = sc[4] + sc[9] (separable form)
  int tvs;       // add the TV(S c) term
};
hipError_t launch_stop_init(int* ctl, double* sc, hipStream_t s);
hipError_t launch_stop_test(int* ctl, double* sc, double* trace, const StopTest& t, hipStream_t s);
hipError_t launch_select_copy(float* out, const float* a0, const float* a1, const int* ctl,
                              int64_t n, hipStream_t s);
// FP16 operand scales (no-ops for other plans).  launch_f16_pmax records
// max |p| of a solve's measurements (p null: 0) for the residual operand's
// bound; the switching and pack launchers and the residual form of H set
// their own scales.
hipError_t launch_f16_pmax(const psoam_plan* P, const float* p, hipStream_t s);
// full regulariser with the TV(S c) term (stacked dual iteration):
//   w = z - (grad^T eta1 + S^T grad^T eta2 + eta3)   [clamp_out: max(., 0)]
//   u1' = clip(eta1 + step0 grad w), u2' = clip(eta2 + step1 grad S w),
//   u3' = clip(eta3 + step2 w)  at radii theta[0..2]
// duals u1 [3][S][V], u2 [3][ceil(K/4)][V][4] (four pulses per 16-byte
// word), u3 [S][V]; eta from (current, previous).  eta2 reaches w through
// its projections pq [6][S][V] (null: eta2 = 0), which launch_r3_u writes
// for the next step's eta2 (beta_next; 0 gives those of u2' itself).
hipError_t launch_r3_w(const psoam_plan* P, float* out, const float* z, const float* u1c,
                       const float* u1p, const float* pq, const float* u3c, const float* u3p,
                       float beta, int clamp_out, hipStream_t s);
hipError_t launch_r3_u(const psoam_plan* P, float* n1, float* n2, float* n3, float* pq,
                       const float* w, const float* u1c, const float* u1p, const float* u2c,
                       const float* u2p, const float* u3c, const float* u3p, float beta,
                       float beta_next, const float step[3], const float theta[3],
                       hipStream_t s);
// separable form (n = Ny*Nx*Nt elements per volume; T [K][S] on the device):
//   y[k] = sum_s T[k][s] h[s]           (expand)
//   out[s] = sum_k T[k][s] y[k]         (contract)
//   rt[s] = sum_s' G[s][s'] h[s'] - q[s] (q may be null); with partial, the
//           FP64 block sums of sum_s h[s] (rt[s] - q[s]) = h^T G h - 2 h^T q
hipError_t launch_sep_expand(const psoam_plan* P, float* y, const float* h, hipStream_t s);
hipError_t launch_sep_contract(const psoam_plan* P, float* out, const float* y, hipStream_t s);
hipError_t launch_sep_residual(const psoam_plan* P, float* rt, const float* h, const float* q,
                               double* partial, hipStream_t s);
size_t sep_blocks(const psoam_plan* P);
// per-voxel unmixing gradient g = S^T (S x - b) (b may be null), optional FP64
// partial sums of |S x - b|^2 over unmix_blocks(P) blocks
hipError_t launch_unmix_grad(const psoam_plan* P, float* g, const float* x, const float* b,
                             double* partial, hipStream_t s);
size_t unmix_blocks(const psoam_plan* P);
// factorised form, one pass over the K*Ny*Nx A-scans of Nt samples:
//   mode 0: out = V in;  mode 1: out = V^T in;
//   mode 2: r = V in - p (p may be null), out = V^T r (out may alias in);
//   mode 3: r = V in - p, FP64 sums of r^2 only.
// Modes 2 and 3 write eir_blocks(P) partial sums when partial is not null.
hipError_t launch_eir_rows(const psoam_plan* P, int mode, float* out, const float* in,
                           const float* p, double* partial, hipStream_t s);
size_t eir_blocks(const psoam_plan* P);
// factorised form, the H^T operand in one pass: V^T (V q - p) when resid
// (p may be null), else V^T q, rounded straight into the 16-bit octet
// operand (what launch_eir_rows followed by launch_pack_r would leave there).
// Only for 16-bit plans whose rows fit the kernel's LDS: eir_pack_fits.
bool eir_pack_fits(const psoam_plan* P, bool resid);
hipError_t launch_eir_pack(const psoam_plan* P, const float* q, const float* p, bool resid,
                           hipStream_t s);
// sum over pulses of the anisotropic TV of (S c)^k into out[0] (FP64)
hipError_t launch_tvs_sum(const psoam_plan* P, const float* c, double* partial, double* out,
                          hipStream_t s);

}  // namespace psoam
