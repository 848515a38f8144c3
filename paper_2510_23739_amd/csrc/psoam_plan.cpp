// Plan construction: validation, photo-switching table, padded operand
// buffers and the packing of the banded impulse response into matrix-core
// tiles for H (output tiles over samples t) and H^T (output tiles over
// depths z).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "psoam_internal.h"

namespace psoam {

namespace {

thread_local std::string g_last_error;

// launch-shape choice of the autotuner for the plan being built (0: the
// plan's own rules)
struct TuneChoice {
  int rows[2] = {0, 0};
  int tsh = -1;
  int loadw = -1;  // H's loader waves: 0 off, 1 on where they can run, else the rules
  int runs[2] = {-1, -1};  // FP32: 0 per-tile kernel, 1 run kernel, else the rules
};
thread_local TuneChoice g_tune;

inline uint16_t to_bf16(float f) {
  // round to nearest even, NaN preserved
  uint32_t u;
  std::memcpy(&u, &f, 4);
  if ((u & 0x7fffffffu) > 0x7f800000u) return (uint16_t)((u >> 16) | 0x40);
  const uint32_t lsb = (u >> 16) & 1u;
  u += 0x7fffu + lsb;
  return (uint16_t)(u >> 16);
}

inline float from_bf16(uint16_t h) {
  uint32_t u = (uint32_t)h << 16;
  float f;
  std::memcpy(&f, &u, 4);
  return f;
}

inline uint16_t to_f16(float f) {
  _Float16 h = (_Float16)f;  // host conversion rounds to nearest even
  uint16_t u;
  std::memcpy(&u, &h, 2);
  return u;
}

inline float from_f16(uint16_t u) {
  _Float16 h;
  std::memcpy(&h, &u, 2);
  return (float)h;
}

struct Group {
  int jy, jx, l;  // lateral offset indices (already flipped for H^T) and contracted index
  int layer = 0;  // 0: the band values; 1: their low-order BF16 parts (refined BF16)
};

}  // namespace

void set_error(const std::string& msg) { g_last_error = msg; }

void set_tune_choice(int rows_fwd, int rows_adj, int tsh, int loadw_fwd, int runs_fwd,
                     int runs_adj) {
  g_tune.rows[0] = rows_fwd;
  g_tune.rows[1] = rows_adj;
  g_tune.tsh = tsh;
  g_tune.loadw = loadw_fwd;
  g_tune.runs[0] = runs_fwd;
  g_tune.runs[1] = runs_adj;
}

void clear_tune_choice() { g_tune = TuneChoice(); }

int fail(int code, const std::string& msg) {
  g_last_error = msg;
  return code;
}

int hip_fail(hipError_t e, const char* what) {
  g_last_error = std::string(what) + ": " + hipGetErrorString(e);
  return e == hipErrorOutOfMemory ? PSOAM_ENOMEM : PSOAM_EHIP;
}

const char* last_error_cstr() { return g_last_error.c_str(); }

// Build the tables of one direction.
//  dir 0 (H):   output rows t (tiles of 16 over Nt), contracted axis z
//  dir 1 (H^T): output rows z (tiles of 16 over Nz), contracted axis t, offsets flipped
// Two packings of the same band blocks: chunks per output tile (global-operand
// kernel, offsets relative to the position base) and, for 16-bit operands,
// chunks per (tile, dy) for the LDS-staged kernel (groups as octet << 16 | dx).
// refine: per column (z, jdy, jdx), 1 where the refined BF16 form adds the
// low-order part of the column's band values as a second layer of groups
// (null for every other precision).
static int build_table(psoam_plan* P, int dir, const int32_t* t0, const float* taps,
                       const uint8_t* refine, BandTable& T) {
  const auto& g = P->g;
  const int F = P->F, W = P->W;
  const bool half = P->prec != PSOAM_FP32;
  const bool split = P->prec == PSOAM_BF16_SPLIT || P->prec == PSOAM_FP16_SPLIT;
  const bool fp16 = P->prec == PSOAM_FP16 || P->prec == PSOAM_FP16_SPLIT;
  const int out_len = dir == 0 ? g.nt : g.nz;
  const int n_mt = (out_len + 15) / 16;
  const int gw = half ? 8 : 1;                     // samples per group
  const int lc = dir == 0 ? P->Lz : P->Lt;         // padded contracted length
  const int n_l = lc / gw;                         // groups along the contracted axis
  const size_t ps = dir == 0 ? P->ps_b : P->ps_r;
  // mark[layer][(tile*F + jy)*F + jx][l]
  const size_t n_off = (size_t)F * F;
  const size_t layer_sz = (size_t)n_mt * n_off * n_l;
  const int n_layers = refine ? 2 : 1;
  std::vector<uint8_t> mark(layer_sz * n_layers, 0);
  // low-order BF16 part of a band value (second layer of the refined form)
  auto low = [](float v) { return v - from_bf16(to_bf16(v)); };
  size_t useful = 0;
  std::vector<double> rowsum(dir == 0 ? g.nt : 0, 0.0);  // sum of |h| per output sample
  for (int z = 0; z < g.nz; ++z)
    for (int jdy = 0; jdy < F; ++jdy)
      for (int jdx = 0; jdx < F; ++jdx) {
        const size_t col = ((size_t)z * F + jdy) * F + jdx;
        for (int j = 0; j < W; ++j) {
          const float v = taps[col * W + j];
          const int t = t0[col] + j;
          if (v == 0.0f || t < 0 || t >= g.nt) continue;
          ++useful;
          if (dir == 0) rowsum[t] += std::fabs((double)v);
          int tile, jy, jx, l;
          if (dir == 0) {
            tile = t / 16; jy = jdy; jx = jdx; l = z / gw;
          } else {
            tile = z / 16; jy = F - 1 - jdy; jx = F - 1 - jdx; l = (t + P->tsh) / gw;
          }
          mark[((size_t)tile * n_off + (size_t)jy * F + jx) * n_l + l] = 1;
          if (refine && refine[col] && low(v) != 0.0f)
            mark[layer_sz + ((size_t)tile * n_off + (size_t)jy * F + jx) * n_l + l] = 1;
        }
      }
  T.n_mtiles = n_mt;
  T.m_rows = out_len;
  T.useful_macs = useful;
  if (dir == 0) {
    // largest row sum of |h| (FP16 rounding of the table can add 2^-11 of it;
    // the operand scales keep a factor of four of headroom)
    double m = 0.0;
    for (double r : rowsum) m = std::max(m, r);
    P->hrow = m;
  }

  // band values of one group into lane-major chunk storage
  auto fill = [&](std::vector<float>& vals, int c, int gi, const Group& G, int tile) {
    const int jdy = dir == 0 ? G.jy : F - 1 - G.jy;
    const int jdx = dir == 0 ? G.jx : F - 1 - G.jx;
    if (dir == 0) {
      for (int e = 0; e < gw; ++e) {
        const int z = G.l * gw + e;
        if (z >= g.nz) continue;
        const size_t col = ((size_t)z * F + jdy) * F + jdx;
        for (int j = 0; j < W; ++j) {
          const int t = t0[col] + j;
          if (t < tile * 16 || t >= tile * 16 + 16 || t >= g.nt) continue;
          const int lane = 16 * gi + (t - tile * 16);
          const float v = taps[col * W + j];
          vals[((size_t)c * 64 + lane) * gw + e] = G.layer ? low(v) : v;
        }
      }
    } else {
      for (int zi = 0; zi < 16; ++zi) {
        const int z = tile * 16 + zi;
        if (z >= g.nz) continue;
        const size_t col = ((size_t)z * F + jdy) * F + jdx;
        for (int j = 0; j < W; ++j) {
          const int t = t0[col] + j;
          if (t < 0 || t >= g.nt || (t + P->tsh) / gw != G.l) continue;
          const int lane = 16 * gi + zi;
          const float v = taps[col * W + j];
          vals[((size_t)c * 64 + lane) * gw + (t + P->tsh - G.l * gw)] = G.layer ? low(v) : v;
        }
      }
    }
  };
  // `pad` zero chunks follow the table (read, unused, by the staged kernel's
  // fixed-width run loads)
  auto upload_vals = [&](const std::vector<float>& vals, int n_chunks, void** hi_out,
                         void** lo_out, int pad) -> int {
    const size_t nc = (n_chunks > 0 ? (size_t)n_chunks : 1) + (size_t)pad;
    if (!half) {
      PSOAM_HIP(hipMalloc(hi_out, sizeof(float) * 64 * nc));
      PSOAM_HIP(hipMemset(*hi_out, 0, sizeof(float) * 64 * nc));
      if (n_chunks)
        PSOAM_HIP(hipMemcpy(*hi_out, vals.data(), sizeof(float) * 64 * n_chunks, hipMemcpyHostToDevice));
      return PSOAM_OK;
    }
    std::vector<uint16_t> hi(vals.size()), lo(vals.size());
    for (size_t i = 0; i < vals.size(); ++i) {
      if (fp16) {
        hi[i] = to_f16(vals[i]);
        lo[i] = to_f16(vals[i] - from_f16(hi[i]));
      } else {
        hi[i] = to_bf16(vals[i]);
        lo[i] = to_bf16(vals[i] - from_bf16(hi[i]));
      }
    }
    PSOAM_HIP(hipMalloc(hi_out, sizeof(uint16_t) * 512 * nc));
    PSOAM_HIP(hipMemset(*hi_out, 0, sizeof(uint16_t) * 512 * nc));
    if (n_chunks)
      PSOAM_HIP(hipMemcpy(*hi_out, hi.data(), sizeof(uint16_t) * 512 * n_chunks, hipMemcpyHostToDevice));
    if (split) {
      PSOAM_HIP(hipMalloc(lo_out, sizeof(uint16_t) * 512 * nc));
      PSOAM_HIP(hipMemset(*lo_out, 0, sizeof(uint16_t) * 512 * nc));
      if (n_chunks)
        PSOAM_HIP(hipMemcpy(*lo_out, lo.data(), sizeof(uint16_t) * 512 * n_chunks, hipMemcpyHostToDevice));
    }
    return PSOAM_OK;
  };

  // ---- packing 1: per output tile (all offsets mixed)
  T.h_start.assign(n_mt + 1, 0);
  std::vector<Group> groups;
  std::vector<Group> chunk_groups;  // 4 per chunk
  for (int tile = 0; tile < n_mt; ++tile) {
    groups.clear();
    for (int layer = 0; layer < n_layers; ++layer)
      for (int jy = 0; jy < F; ++jy)
        for (int jx = 0; jx < F; ++jx)
          for (int l = 0; l < n_l; ++l)
            if (mark[layer * layer_sz + ((size_t)tile * n_off + (size_t)jy * F + jx) * n_l + l])
              groups.push_back({jy, jx, l, layer});
    const int nch = (int)((groups.size() + 3) / 4);
    T.h_start[tile + 1] = T.h_start[tile] + nch;
    for (int i = 0; i < nch * 4; ++i)
      chunk_groups.push_back(i < (int)groups.size() ? groups[i] : Group{-1, -1, -1});
  }
  const int n_chunks = T.h_start[n_mt];
  T.n_chunks = n_chunks;
  {
    std::vector<int> off((size_t)n_chunks * 4, 0);
    std::vector<float> vals((size_t)n_chunks * 64 * gw, 0.0f);
    for (int tile = 0; tile < n_mt; ++tile)
      for (int c = T.h_start[tile]; c < T.h_start[tile + 1]; ++c)
        for (int gi = 0; gi < 4; ++gi) {
          const Group& G = chunk_groups[(size_t)c * 4 + gi];
          if (G.jy < 0) continue;  // padding group: offset 0, zero band values
          off[(size_t)c * 4 + gi] =
              (int)(((size_t)G.jy * P->Xp + G.jx) * ps + (size_t)G.l * gw * P->Kp);
          fill(vals, c, gi, G, tile);
        }
    PSOAM_HIP(hipMalloc(&T.d_start, sizeof(int) * (n_mt + 1)));
    PSOAM_HIP(hipMemcpy(T.d_start, T.h_start.data(), sizeof(int) * (n_mt + 1), hipMemcpyHostToDevice));
    const size_t nc = n_chunks > 0 ? (size_t)n_chunks : 1;
    PSOAM_HIP(hipMalloc(&T.d_off, sizeof(int) * 4 * nc));
    if (n_chunks) PSOAM_HIP(hipMemcpy(T.d_off, off.data(), sizeof(int) * 4 * n_chunks, hipMemcpyHostToDevice));
    if (int rc = upload_vals(vals, n_chunks, &T.d_a, &T.d_a_lo, 0)) return rc;
  }
  // FP32 plans use the runs below with the global-operand run kernel
  // (PSOAM_FP32_RUNS=0 or PSOAM_BAND_GLOBAL=1 keeps them on the per-tile kernel)
  if (!half) {
    const char* e = std::getenv("PSOAM_FP32_RUNS");
    const char* gl = std::getenv("PSOAM_BAND_GLOBAL");
    if ((e && e[0] == '0') || (gl && gl[0] == '1')) return PSOAM_OK;
    if (g_tune.runs[dir] == 0) return PSOAM_OK;  // the autotuner's choice
  }

  // ---- packing 2: runs per (tile, dy) for the LDS-staged kernel.
  // A run holds m consecutive chunks whose 4 groups keep their octet while
  // their offset steps dx_g, dx_g - 1, ..., dx_g - m + 1: the operand of
  // position p at chunk i is then the one of position p - 1 at chunk i - 1,
  // so the kernel slides a register window and reads one new column per
  // chunk.  The marked (dx, octet) pairs of each octet are split into
  // pieces of at most kRunMax consecutive dx, grouped four per run (longest
  // first); a lane shorter than the run is placed so that its idle chunks
  // still address columns inside [0, F) (with zero band values).
  const int run_max = std::max(1, std::min(kRunMax, (F + 1) / 2));
  struct Piece { int l, lo, len, layer; };
  std::vector<int> rstart((size_t)n_mt * F + 1, 0);
  std::vector<uint32_t> rgrp;   // 4 per run: octet << 16 | dx at the run's first chunk
  std::vector<int> rlen, rcb;   // run length, first chunk index
  std::vector<Group> lgroups;   // 4 per chunk (active groups; jy < 0 for idle lanes)
  std::vector<int> lo_l((size_t)n_mt * F, 1 << 30), hi_l((size_t)n_mt * F, -1);
  int l_chunks = 0;
  std::vector<Piece> pieces;
  for (int tile = 0; tile < n_mt; ++tile)
    for (int jy = 0; jy < F; ++jy) {
      const size_t key = (size_t)tile * F + jy;
      pieces.clear();
      for (int layer = 0; layer < n_layers; ++layer) {
        const uint8_t* mk = mark.data() + layer * layer_sz;
        for (int l = 0; l < n_l; ++l) {
          int jx = 0;
          while (jx < F) {
            if (!mk[((size_t)tile * n_off + (size_t)jy * F + jx) * n_l + l]) { ++jx; continue; }
            int e = jx;
            while (e + 1 < F && mk[((size_t)tile * n_off + (size_t)jy * F + e + 1) * n_l + l]) ++e;
            for (int lo = jx; lo <= e; lo += run_max)
              pieces.push_back({l, lo, std::min(run_max, e - lo + 1), layer});
            lo_l[key] = std::min(lo_l[key], l);
            hi_l[key] = std::max(hi_l[key], l);
            jx = e + 1;
          }
        }
      }
      std::stable_sort(pieces.begin(), pieces.end(),
                       [](const Piece& x, const Piece& y) { return x.len > y.len; });
      for (size_t i = 0; i < pieces.size(); i += 4) {
        const int m = pieces[i].len;
        rlen.push_back(m);
        rcb.push_back(l_chunks);
        int dstart[4], lane_l[4], first[4], len[4], lane_layer[4];
        for (int gi = 0; gi < 4; ++gi) {
          if (i + gi < pieces.size()) {
            const Piece& pc = pieces[i + gi];
            lane_l[gi] = pc.l;
            lane_layer[gi] = pc.layer;
            len[gi] = pc.len;
            if (pc.lo + m - 1 <= F - 1) {        // piece at the end of the run
              dstart[gi] = pc.lo + m - 1;
              first[gi] = m - pc.len;
            } else {                             // piece at the start
              dstart[gi] = pc.lo + pc.len - 1;
              first[gi] = 0;
              if (dstart[gi] - (m - 1) < 0) return fail(PSOAM_EINVAL, "plan: run placement");
            }
          } else {                               // idle lane: zero band, valid columns
            lane_l[gi] = pieces[i].l;
            lane_layer[gi] = 0;
            len[gi] = 0;
            dstart[gi] = m - 1;
            first[gi] = 0;
          }
          rgrp.push_back(((uint32_t)lane_l[gi] << 16) | (uint32_t)dstart[gi]);
        }
        for (int c = 0; c < m; ++c) {
          for (int gi = 0; gi < 4; ++gi) {
            const bool on = c >= first[gi] && c < first[gi] + len[gi];
            lgroups.push_back(on ? Group{jy, dstart[gi] - c, lane_l[gi], lane_layer[gi]} : Group{-1, -1, -1});
          }
          ++l_chunks;
        }
      }
      rstart[key + 1] = (int)rlen.size();
    }
  T.l_chunks = l_chunks;
  T.n_runs = (int)rlen.size();
  T.max_runs = 0;
  for (int tile = 0; tile < n_mt; ++tile)
    T.max_runs = std::max(T.max_runs, rstart[(size_t)(tile + 1) * F] - rstart[(size_t)tile * F]);
  // the run tables on the device: per (tile, dy) first run, per run its four
  // group words and (length, first chunk), the tile order, the band values
  auto upload_runs = [&]() -> int {
    std::vector<float> lvals((size_t)l_chunks * 64 * gw, 0.0f);
    {
      // chunk -> tile for the band fill
      std::vector<int> chunk_tile(l_chunks, 0);
      for (int tile = 0; tile < n_mt; ++tile)
        for (int jy = 0; jy < F; ++jy) {
          const size_t key = (size_t)tile * F + jy;
          for (int r = rstart[key]; r < rstart[key + 1]; ++r)
            for (int c = rcb[r]; c < rcb[r] + rlen[r]; ++c) chunk_tile[c] = tile;
        }
      for (int c = 0; c < l_chunks; ++c)
        for (int gi = 0; gi < 4; ++gi) {
          const Group& G = lgroups[(size_t)c * 4 + gi];
          if (G.jy >= 0) fill(lvals, c, gi, G, chunk_tile[c]);
        }
    }
    const size_t nr = std::max<size_t>(rlen.size(), 1);
    PSOAM_HIP(hipMalloc(&T.d_lstart, sizeof(int) * rstart.size()));
    PSOAM_HIP(hipMemcpy(T.d_lstart, rstart.data(), sizeof(int) * rstart.size(), hipMemcpyHostToDevice));
    PSOAM_HIP(hipMalloc(&T.d_lgrp, sizeof(uint32_t) * 4 * nr));
    if (!rgrp.empty())
      PSOAM_HIP(hipMemcpy(T.d_lgrp, rgrp.data(), sizeof(uint32_t) * rgrp.size(), hipMemcpyHostToDevice));
    {
      std::vector<int> rinfo(2 * nr, 0);  // (length, first chunk) per run
      for (size_t r = 0; r < rlen.size(); ++r) {
        rinfo[2 * r] = rlen[r];
        rinfo[2 * r + 1] = rcb[r];
      }
      PSOAM_HIP(hipMalloc(&T.d_rinfo, sizeof(int) * rinfo.size()));
      PSOAM_HIP(hipMemcpy(T.d_rinfo, rinfo.data(), sizeof(int) * rinfo.size(), hipMemcpyHostToDevice));
    }
    {
      std::vector<int> order(n_mt);
      for (int i = 0; i < n_mt; ++i) order[i] = i;
      std::vector<long> work(n_mt, 0);
      for (int t = 0; t < n_mt; ++t)
        for (int r = rstart[(size_t)t * F]; r < rstart[(size_t)(t + 1) * F]; ++r) work[t] += rlen[r];
      std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return work[x] > work[y]; });
      PSOAM_HIP(hipMalloc(&T.d_order, sizeof(int) * n_mt));
      PSOAM_HIP(hipMemcpy(T.d_order, order.data(), sizeof(int) * n_mt, hipMemcpyHostToDevice));
    }
    return upload_vals(lvals, l_chunks, &T.d_la, &T.d_la_lo, kRunMax);
  };
  if (!half) {
    if (n_l >= 0xffff || F >= 0xffff) return PSOAM_OK;
    T.runs32 = true;
    return upload_runs();
  }
  // staged row windows for a workgroup of `rows` output rows (waves): the
  // union of the octet ranges of the dy values j - r, r < rows
  auto windows = [&](int rows, std::vector<uint32_t>& win, int& max_oct) {
    const int nwin = F + rows - 1;
    win.assign((size_t)n_mt * nwin, 0);
    max_oct = 0;
    for (int tile = 0; tile < n_mt; ++tile)
      for (int j = 0; j < nwin; ++j) {
        int lo = 1 << 30, hi = -1;
        for (int r = 0; r < rows; ++r) {
          const int dy = j - r;
          if (dy < 0 || dy >= F) continue;
          const size_t key = (size_t)tile * F + dy;
          if (hi_l[key] < 0) continue;
          lo = std::min(lo, lo_l[key]);
          hi = std::max(hi, hi_l[key]);
        }
        if (hi >= 0) {
          const int cnt = hi - lo + 1;
          max_oct = std::max(max_oct, cnt);
          win[(size_t)tile * nwin + j] = ((uint32_t)lo << 16) | (uint32_t)cnt;
        }
      }
  };
  const int XW = kLdsPos + F - 1;
  auto lds_of = [&](int rows, int max_oct) {
    return (size_t)max_oct * XW * 16 * 8 * sizeof(uint16_t) +
           lds_meta_bytes(F, rows, T.max_runs) + 16;
  };
  std::vector<uint32_t> win4, win8, win12;
  int mo4 = 0, mo8 = 0, mo12 = 0;
  windows(4, win4, mo4);
  windows(8, win8, mo8);
  windows(12, win12, mo12);
  const size_t lds4 = lds_of(4, mo4), lds8 = lds_of(8, mo8), lds12 = lds_of(12, mo12);
  // 12 rows (three waves per SIMD, one-part operands): a staged row serves
  // twelve output rows instead of eight
  // Rows per workgroup: four while at least two such workgroups fit in one
  // CU's LDS (eight waves per CU); when only one fits, eight rows keep two
  // waves per SIMD resident (measured: H^T at 31 x 31 footprint 2.48 ms with
  // eight rows vs 4.44 ms with four; H 2.55 ms with four vs 2.64 with eight)
  int rows = 4;
  if (lds4 > (size_t)kLdsMaxBytes / 2 && lds8 <= (size_t)kLdsMaxBytes) rows = 8;
  if (lds4 > (size_t)kLdsMaxBytes && lds8 <= (size_t)kLdsMaxBytes) rows = 8;
  // split-operand H^T needs more registers than two waves per SIMD allow, so
  // a second 4-row workgroup could not share the CU: eight rows instead
  if (dir == 1 && split && lds8 <= (size_t)kLdsMaxBytes) rows = 8;
  const bool fit12 = !split && lds12 <= (size_t)kLdsMaxBytes;
  // where one workgroup holds the CU anyway, twelve rows stage a row for
  // twelve output rows instead of eight, at three waves per SIMD: H at 320 x
  // 320 x 128 (footprint 51) 66.6 -> 63.1 ms, at 256 x 256 x 96 16.6 -> 16.0
  // ms.  H^T, whose S^T epilogue spills more at three waves per SIMD, keeps
  // eight rows (63.8 -> 62.3 ms at the first, 15.8 -> 17.0 ms at the second);
  // the autotuner times both
  if (dir == 0 && rows == 8 && fit12) rows = 12;
  // PSOAM_LDS_ROWS=4, 8 or 12 overrides the choice when it fits (tests cover all)
  if (const char* fr = std::getenv("PSOAM_LDS_ROWS")) {
    if (fr[0] == '8' && lds8 <= (size_t)kLdsMaxBytes) rows = 8;
    if (fr[0] == '4' && lds4 <= (size_t)kLdsMaxBytes) rows = 4;
    if (fr[0] == '1' && fr[1] == '2' && fit12) rows = 12;
  }
  // the autotuner's choice, when it fits
  if (g_tune.rows[dir] == 8 && lds8 <= (size_t)kLdsMaxBytes) rows = 8;
  if (g_tune.rows[dir] == 4 && lds4 <= (size_t)kLdsMaxBytes) rows = 4;
  if (g_tune.rows[dir] == 12 && fit12) rows = 12;
  std::vector<uint32_t>& win = rows == 12 ? win12 : rows == 8 ? win8 : win4;
  T.rows = rows;
  T.max_oct = rows == 12 ? mo12 : rows == 8 ? mo8 : mo4;
  T.lds_bytes = (size_t)T.max_oct * XW * 16 * 8 * sizeof(uint16_t);
  // Loader waves: four more waves that load the next staged row into
  // registers during the current row's contractions (H and its residual
  // form, one 8-row workgroup per CU, one-part operands; 25 items per loader
  // thread must cover the widest window).  Off by default: staging straight
  // into LDS (buffer loads with the LDS destination, every item in flight at
  // once) is faster on every workload measured; the autotuner still times
  // them.
  T.loadw = 0;
  {
    const size_t items = (size_t)T.max_oct * XW * 16;
    const bool able = rows == 8 && !split && dir == 0 && items <= (size_t)25 * 256;
    // PSOAM_LDS_LOADW=0 keeps the plain staging, =1 takes the loader waves
    // wherever they can run (tests and A/B timing run both)
    if (const char* e = std::getenv("PSOAM_LDS_LOADW")) {
      if (e[0] == '0') T.loadw = 0;
      if (e[0] == '1' && able) T.loadw = 4;
    }
    // the autotuner's choice
    if (dir == 0 && g_tune.loadw == 0) T.loadw = 0;
    if (dir == 0 && g_tune.loadw == 1 && able) T.loadw = 4;
  }
  // Half last block: with K mod 16 in 1..8 the last 16-pulse block is at
  // least half padding; the staged kernel then stages 8 pulses per column and
  // fills the matrix cores' 16 columns with 8 pulses of two positions.
  // PSOAM_HALF_BLOCK=0 keeps the padded block (tests compare both).
  T.half = P->g.n_pulses <= P->Kp - 8 ? 1 : 0;
  if (const char* e = std::getenv("PSOAM_HALF_BLOCK"))
    if (e[0] == '0') T.half = 0;
  // PSOAM_BAND_GLOBAL=1 keeps the plan on the global-operand kernel (tests cover both)
  const char* force_global = std::getenv("PSOAM_BAND_GLOBAL");
  T.lds_ok = n_l < 0xffff && F < 0xffff &&
             (rows == 12 ? lds12 : rows == 8 ? lds8 : lds4) <= (size_t)kLdsMaxBytes &&
             !(force_global && force_global[0] == '1');
  if (!T.lds_ok) return PSOAM_OK;
  PSOAM_HIP(hipMalloc(&T.d_win, sizeof(uint32_t) * win.size()));
  PSOAM_HIP(hipMemcpy(T.d_win, win.data(), sizeof(uint32_t) * win.size(), hipMemcpyHostToDevice));
  return upload_runs();
}

static void free_table(BandTable& T) {
  void* ptrs[] = {T.d_start, T.d_off, T.d_a, T.d_a_lo, T.d_lstart, T.d_lgrp, T.d_win, T.d_la,
                  T.d_la_lo, T.d_order, T.d_rinfo};
  for (void* p : ptrs)
    if (p) (void)hipFree(p);
  T.d_start = nullptr;
  T.d_off = nullptr;
  T.d_a = T.d_a_lo = nullptr;
  T.d_lstart = nullptr;
  T.d_lgrp = nullptr;
  T.d_win = nullptr;
  T.d_la = T.d_la_lo = nullptr;
  T.d_order = nullptr;
  T.d_rinfo = nullptr;
}

// Largest eigenvalue of a symmetric n x n matrix (n <= kMaxSpecies), cyclic
// Jacobi rotations in FP64 until the off-diagonal part vanishes.
static double sym_eig_max(double (&m)[kMaxSpecies][kMaxSpecies], int n) {
  for (int sweep = 0; sweep < 64; ++sweep) {
    double off = 0.0, tot = 0.0;
    for (int i = 0; i < n; ++i)
      for (int j = 0; j < n; ++j) {
        tot += m[i][j] * m[i][j];
        if (i != j) off += m[i][j] * m[i][j];
      }
    if (off <= 1e-30 * tot) break;
    for (int p = 0; p < n - 1; ++p)
      for (int q = p + 1; q < n; ++q) {
        if (m[p][q] == 0.0) continue;
        const double th = (m[q][q] - m[p][p]) / (2.0 * m[p][q]);
        const double t = (th >= 0.0 ? 1.0 : -1.0) / (std::fabs(th) + std::sqrt(th * th + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), sn = t * c;
        for (int k = 0; k < n; ++k) {  // columns p, q
          const double a = m[k][p], b = m[k][q];
          m[k][p] = c * a - sn * b;
          m[k][q] = sn * a + c * b;
        }
        for (int k = 0; k < n; ++k) {  // rows p, q
          const double a = m[p][k], b = m[q][k];
          m[p][k] = c * a - sn * b;
          m[q][k] = sn * a + c * b;
        }
      }
  }
  double e = m[0][0];
  for (int i = 1; i < n; ++i) e = std::max(e, m[i][i]);
  return e;
}

// max over the fluence values phi of eig_max(S^T S) for the switching block
// S[k][s] = phi (a_s + b_s exp(-k phi^gamma / tau_s)) (FP64)
static double switching_norm2(const psoam_geom& g, const psoam_species* sp, const float* phi,
                              size_t nphi) {
  const int ns = g.n_species, nk = g.n_pulses;
  double best = 0.0;
  std::vector<double> col((size_t)nk * ns);
  float last = -1.0f;
  for (size_t i = 0; i < nphi; ++i) {
    if (phi[i] == last) continue;  // runs of equal fluence give the same block
    last = phi[i];
    const double ph = phi[i];
    const double pg = sp->gamma == 0.0 ? 1.0 : std::pow(ph, sp->gamma);
    for (int k = 0; k < nk; ++k)
      for (int s = 0; s < ns; ++s)
        col[(size_t)k * ns + s] = ph * (sp->a[s] + sp->b[s] * std::exp(-(double)k * pg / sp->tau[s]));
    double m[kMaxSpecies][kMaxSpecies] = {};
    for (int a = 0; a < ns; ++a)
      for (int b = 0; b < ns; ++b) {
        double acc = 0.0;
        for (int k = 0; k < nk; ++k) acc += col[(size_t)k * ns + a] * col[(size_t)k * ns + b];
        m[a][b] = acc;
      }
    best = std::max(best, sym_eig_max(m, ns));
  }
  return best;
}

void free_plan(psoam_plan* P) {
  if (!P) return;
  (void)hipSetDevice(P->device);
  (void)hipDeviceSynchronize();
  if (P->inner) free_plan(P->inner);
  P->inner = nullptr;
  for (void* b : {(void*)P->d_T, (void*)P->d_h, (void*)P->d_rt, (void*)P->d_q, (void*)P->d_fq})
    if (b) (void)hipFree(b);
  free_table(P->fwd);
  free_table(P->adj);
  void* bufs[] = {P->d_phi, P->d_stab, P->d_stab_t, P->d_stab_o, P->d_bq, P->d_bq_lo, P->d_rq, P->d_rq_lo,
                  P->solve_ws.base, P->r3_ws.base, P->yc_ws.base, P->d_partial, P->d_scalars, P->d_f16,
                  P->d_f16acc, P->d_ctl, P->d_trace};
  for (void* b : bufs)
    if (b) (void)hipFree(b);
  delete P;
}

// diag: switching S'_v = phi_v I over the species (inner plan of the
// separable form); build_op = false skips the contraction tables and operand
// buffers (outer plan of the separable form).
// Widest octet window (8-sample groups of the H^T operand, samples shifted
// by tsh) that a workgroup of `rows` output rows of H^T stages: per output
// tile of 16 depths and lateral offset dy, the octet range of the band; per
// staged row, the union over the rows' dy values.
static int adj_window_octets(const psoam_geom& g, const int32_t* t0, const float* taps, int W,
                             int tsh, int rows) {
  const int F = g.f, n_mt = (g.nz + 15) / 16;
  std::vector<int> lo((size_t)n_mt * F, 1 << 30), hi((size_t)n_mt * F, -1);
  for (int z = 0; z < g.nz; ++z)
    for (int jdy = 0; jdy < F; ++jdy)
      for (int jdx = 0; jdx < F; ++jdx) {
        const size_t col = ((size_t)z * F + jdy) * F + jdx;
        for (int j = 0; j < W; ++j) {
          const int t = t0[col] + j;
          if (taps[col * W + j] == 0.0f || t < 0 || t >= g.nt) continue;
          const size_t key = (size_t)(z / 16) * F + (F - 1 - jdy);
          lo[key] = std::min(lo[key], (t + tsh) / 8);
          hi[key] = std::max(hi[key], (t + tsh) / 8);
        }
      }
  int best = 0;
  for (int tile = 0; tile < n_mt; ++tile)
    for (int j = 0; j < F + rows - 1; ++j) {
      int l = 1 << 30, h = -1;
      for (int r = 0; r < rows; ++r) {
        const int dy = j - r;
        if (dy < 0 || dy >= F) continue;
        const size_t key = (size_t)tile * F + dy;
        if (hi[key] < 0) continue;
        l = std::min(l, lo[key]);
        h = std::max(h, hi[key]);
      }
      if (h >= 0) best = std::max(best, h - l + 1);
    }
  return best;
}

static int create_plan_impl(const psoam_geom* gp, const psoam_species* sp, const float* phi,
                            const int32_t* t0, const float* taps, int32_t sir_w, int32_t prec,
                            hipStream_t stream, int diag, bool build_op, psoam_plan** out) {
  if (!out) return fail(PSOAM_EINVAL, "plan_create: out is NULL");
  *out = nullptr;
  if (!gp || !sp || !phi || !t0 || !taps) return fail(PSOAM_EINVAL, "plan_create: NULL argument");
  const psoam_geom g = *gp;
  if (g.nx <= 0 || g.ny <= 0 || g.nz <= 0 || g.nt <= 0 || g.n_pulses <= 0)
    return fail(PSOAM_EINVAL, "plan_create: sizes must be positive");
  if (g.f <= 0 || (g.f % 2) == 0) return fail(PSOAM_EINVAL, "plan_create: footprint f must be odd and positive");
  // diagonal switching (pulse volumes as "species") allows one volume per pulse
  if (g.n_species < 1 || g.n_species > (diag ? 64 : kMaxSpecies))
    return fail(PSOAM_EINVAL, "plan_create: n_species must be in 1..8");
  if (sir_w < 1 || sir_w > 64) return fail(PSOAM_EINVAL, "plan_create: sir_w must be in 1..64");
  if (g.phi_per_voxel != 0 && g.phi_per_voxel != 1)
    return fail(PSOAM_EINVAL, "plan_create: phi_per_voxel must be 0 or 1");
  if (prec < PSOAM_FP32 || prec > PSOAM_BF16_REFINED)
    return fail(PSOAM_EUNSUPPORTED, "plan_create: unknown precision");
  if (g.n_pulses > 64) return fail(PSOAM_EUNSUPPORTED, "plan_create: at most 64 pulses");
  for (int s = 0; s < (diag ? 0 : g.n_species); ++s) {
    if (!std::isfinite(sp->a[s]) || !std::isfinite(sp->b[s]) || !(sp->tau[s] > 0.0) ||
        !std::isfinite(sp->tau[s]))
      return fail(PSOAM_EINVAL, "plan_create: species constants must be finite, tau > 0");
  }
  if (!std::isfinite(sp->gamma)) return fail(PSOAM_EINVAL, "plan_create: gamma not finite");
  const size_t nphi = g.phi_per_voxel ? (size_t)g.ny * g.nx * g.nz : (size_t)g.nz;
  for (size_t i = 0; i < nphi; ++i)
    if (!(phi[i] > 0.0f) || !std::isfinite(phi[i])) return fail(PSOAM_EINVAL, "plan_create: phi must be finite and > 0");
  const size_t ntab = (size_t)g.nz * g.f * g.f;
  for (size_t i = 0; i < ntab * sir_w; ++i)
    if (!std::isfinite(taps[i])) return fail(PSOAM_EINVAL, "plan_create: non-finite impulse-response tap");
  for (size_t i = 0; i < ntab; ++i)
    if (t0[i] < -(1 << 28) || t0[i] > (1 << 28)) return fail(PSOAM_EINVAL, "plan_create: band start out of range");

  psoam_plan* P = new (std::nothrow) psoam_plan();
  if (!P) return fail(PSOAM_ENOMEM, "plan_create: host allocation failed");
  P->g = g;
  P->sp_in = *sp;
  P->prec = prec;
  P->F = g.f;
  P->R = (g.f - 1) / 2;
  P->W = sir_w;
  P->Kp = (g.n_pulses + 15) / 16 * 16;
  P->NB = P->Kp / 16;
  P->Yp = g.ny + 2 * P->R;
  P->Xp = (g.nx + kPadX - 1) / kPadX * kPadX + 2 * P->R;
  const bool half = prec != PSOAM_FP32;
  const bool split = prec == PSOAM_BF16_SPLIT || prec == PSOAM_FP16_SPLIT;
  P->Lz = half ? (g.nz + 7) / 8 * 8 : g.nz;
  // 16-bit H^T operand: shifting its samples by 4 (the residual epilogue
  // writes aligned quarters of 8-sample octets, so only 0 and 4 keep them
  // aligned) can narrow the widest staged octet window of the H^T kernel by
  // one octet.  Per shift, the row count the staged kernel's LDS rule would
  // pick is predicted (two 4-row workgroups per CU, else one 8-row, else one
  // 4-row); the shift with the better outcome, then the narrower window, wins.
  if (half) {
    const size_t row_bytes = (size_t)(kLdsPos + g.f - 1) * 16 * 8 * sizeof(uint16_t);
    const size_t meta = 8192;  // generous bound of the per-tile tables
    auto outcome = [&](int sh, int& width) {
      const int o4 = adj_window_octets(g, t0, taps, sir_w, sh, 4);
      const int o8 = adj_window_octets(g, t0, taps, sir_w, sh, 8);
      const size_t l4 = o4 * row_bytes + meta, l8 = o8 * row_bytes + meta;
      if (!split && l4 <= (size_t)kLdsMaxBytes / 2) { width = o4; return 3; }
      if (l8 <= (size_t)kLdsMaxBytes) { width = o8; return 2; }
      width = o4;
      return l4 <= (size_t)kLdsMaxBytes ? 1 : 0;
    };
    int w0 = 0, w4 = 0;
    const int s0 = outcome(0, w0), s4 = outcome(4, w4);
    P->tsh = (s4 > s0 || (s4 == s0 && w4 < w0)) ? 4 : 0;
    // PSOAM_ADJ_SHIFT=0 or 4 overrides the choice (tests cover both)
    if (const char* e = std::getenv("PSOAM_ADJ_SHIFT")) P->tsh = e[0] == '4' ? 4 : 0;
    if (g_tune.tsh == 0 || g_tune.tsh == 4) P->tsh = g_tune.tsh;  // the autotuner's choice
  }
  // PSOAM_TV_TILE=i takes tile shape i of the TV dual step (tests run each)
  if (const char* e = std::getenv("PSOAM_TV_TILE")) {
    const int t = std::atoi(e);
    if (t >= 0 && t < tv_tile_count()) P->tv_tile = t;
  }
  P->Lt = (g.nt + 15) / 16 * 16 + (P->tsh ? 16 : 0);
  P->ps_b = (size_t)P->Lz * P->Kp;
  P->ps_r = (size_t)P->Lt * P->Kp;
  (void)hipGetDevice(&P->device);
  auto& sw = P->sw;
  sw.ns = g.n_species;
  sw.nk = g.n_pulses;
  sw.per_voxel = g.phi_per_voxel;
  sw.diag = diag;
  sw.gamma = (float)sp->gamma;
  for (int s = 0; s < kMaxSpecies; ++s) {
    sw.a[s] = s < g.n_species ? (float)sp->a[s] : 0.0f;
    sw.b[s] = s < g.n_species ? (float)sp->b[s] : 0.0f;
    sw.inv_tau[s] = (!diag && s < g.n_species) ? (float)(1.0 / sp->tau[s]) : 0.0f;
  }
  int rc = PSOAM_OK;
  auto bail = [&](int code) {
    free_plan(P);
    return code;
  };
#define PLAN_HIP(call)                                  \
  do {                                                  \
    hipError_t _e = (call);                             \
    if (_e != hipSuccess) return bail(hip_fail(_e, #call)); \
  } while (0)
  if (diag) {
    double m = 0.0;  // S'_v = phi_v I
    for (size_t i = 0; i < nphi; ++i) m = std::max(m, (double)phi[i] * (double)phi[i]);
    P->smax2 = m;
    P->srow = std::sqrt(m);
  } else {
    P->smax2 = switching_norm2(g, sp, phi, nphi);
    // largest row sum of |S_v| (bound of the switched operand per unit of c)
    double m = 0.0;
    for (size_t i = 0; i < nphi; ++i) {
      const double ph = phi[i];
      const double pg = sp->gamma == 0.0 ? 1.0 : std::pow(ph, sp->gamma);
      for (int k = 0; k < g.n_pulses; ++k) {
        double row = 0.0;
        for (int sidx = 0; sidx < g.n_species; ++sidx)
          row += std::fabs(ph * (sp->a[sidx] + sp->b[sidx] * std::exp(-(double)k * pg / sp->tau[sidx])));
        m = std::max(m, row);
      }
    }
    P->srow = m;
  }
  PLAN_HIP(hipMalloc(&P->d_phi, sizeof(float) * nphi));
  PLAN_HIP(hipMemcpy(P->d_phi, phi, sizeof(float) * nphi, hipMemcpyHostToDevice));
  if (!g.phi_per_voxel) {
    // per-depth switching table S[z][k][s] (zero for padded pulses), computed in double
    std::vector<float> st((size_t)g.nz * P->Kp * g.n_species, 0.0f);
    for (int z = 0; z < g.nz; ++z)
      for (int k = 0; k < g.n_pulses; ++k)
        for (int s = 0; s < g.n_species; ++s) {
          const double ph = phi[z];
          const double pg = sp->gamma == 0.0 ? 1.0 : std::pow(ph, sp->gamma);
          st[((size_t)z * P->Kp + k) * g.n_species + s] =
              diag ? (k == s ? (float)ph : 0.0f)
                   : (float)(ph * (sp->a[s] + sp->b[s] * std::exp(-(double)k * pg / sp->tau[s])));
        }
    PLAN_HIP(hipMalloc(&P->d_stab, sizeof(float) * st.size()));
    PLAN_HIP(hipMemcpy(P->d_stab, st.data(), sizeof(float) * st.size(), hipMemcpyHostToDevice));
    std::vector<float> stt((size_t)g.n_pulses * g.n_species * g.nz);
    for (int z = 0; z < g.nz; ++z)
      for (int k = 0; k < g.n_pulses; ++k)
        for (int s = 0; s < g.n_species; ++s)
          stt[((size_t)k * g.n_species + s) * g.nz + z] = st[((size_t)z * P->Kp + k) * g.n_species + s];
    PLAN_HIP(hipMalloc(&P->d_stab_t, sizeof(float) * stt.size()));
    PLAN_HIP(hipMemcpy(P->d_stab_t, stt.data(), sizeof(float) * stt.size(), hipMemcpyHostToDevice));
    if (half) {
      // the 16-bit S kernel's lanes are pulses of one depth octet: each reads
      // its octet's eight coefficients per species as 32 contiguous bytes
      const int zo_n = P->Lz / 8;
      std::vector<float> sto((size_t)zo_n * g.n_species * P->Kp * 8, 0.0f);
      for (int z = 0; z < g.nz; ++z)
        for (int k = 0; k < P->Kp; ++k)
          for (int s = 0; s < g.n_species; ++s)
            sto[(((size_t)(z / 8) * g.n_species + s) * P->Kp + k) * 8 + (z & 7)] =
                st[((size_t)z * P->Kp + k) * g.n_species + s];
      PLAN_HIP(hipMalloc(&P->d_stab_o, sizeof(float) * sto.size()));
      PLAN_HIP(hipMemcpy(P->d_stab_o, sto.data(), sizeof(float) * sto.size(), hipMemcpyHostToDevice));
    }
  }
  if (!build_op) {
    PLAN_HIP(hipStreamSynchronize(stream));
    *out = P;
    return PSOAM_OK;
  }
  const size_t esz = half ? 2 : 4;
  P->bq_bytes = (size_t)P->Yp * P->Xp * P->ps_b * esz;
  P->rq_bytes = (size_t)P->Yp * P->Xp * P->ps_r * esz;
  PLAN_HIP(hipMalloc(&P->d_bq, P->bq_bytes));
  PLAN_HIP(hipMalloc(&P->d_rq, P->rq_bytes));
  PLAN_HIP(hipMemsetAsync(P->d_bq, 0, P->bq_bytes, stream));
  PLAN_HIP(hipMemsetAsync(P->d_rq, 0, P->rq_bytes, stream));
  if (prec == PSOAM_FP16 || prec == PSOAM_FP16_SPLIT) {
    const float init[8] = {kFp16Scale, 1.0f / kFp16Scale, kFp16Scale, 1.0f / kFp16Scale, 0, 0, 0, 0};
    PLAN_HIP(hipMalloc(&P->d_f16, sizeof(init)));
    PLAN_HIP(hipMemcpy(P->d_f16, init, sizeof(init), hipMemcpyHostToDevice));
    PLAN_HIP(hipMalloc(&P->d_f16acc, 4 * sizeof(unsigned)));
    PLAN_HIP(hipMemset(P->d_f16acc, 0, 4 * sizeof(unsigned)));
  }
  if (split) {
    PLAN_HIP(hipMalloc(&P->d_bq_lo, P->bq_bytes));
    PLAN_HIP(hipMalloc(&P->d_rq_lo, P->rq_bytes));
    PLAN_HIP(hipMemsetAsync(P->d_bq_lo, 0, P->bq_bytes, stream));
    PLAN_HIP(hipMemsetAsync(P->d_rq_lo, 0, P->rq_bytes, stream));
  }
  // refined BF16: the fewest columns, by decreasing squared rounding error of
  // their band values, that hold 90% of the table's squared rounding error
  std::vector<uint8_t> refine;
  if (prec == PSOAM_BF16_REFINED) {
    const size_t ncol = (size_t)g.nz * g.f * g.f;
    std::vector<double> err(ncol, 0.0);
    double tot = 0.0;
    for (size_t col = 0; col < ncol; ++col) {
      for (int j = 0; j < sir_w; ++j) {
        const int t = t0[col] + j;
        if (t < 0 || t >= g.nt) continue;
        const double e = (double)taps[col * sir_w + j] - (double)from_bf16(to_bf16(taps[col * sir_w + j]));
        err[col] += e * e;
      }
      tot += err[col];
    }
    std::vector<size_t> idx(ncol);
    for (size_t i = 0; i < ncol; ++i) idx[i] = i;
    std::stable_sort(idx.begin(), idx.end(), [&](size_t a, size_t b) { return err[a] > err[b]; });
    refine.assign(ncol, 0);
    double acc = 0.0;
    for (size_t i = 0; i < ncol && acc < 0.9 * tot; ++i) {
      refine[idx[i]] = 1;
      acc += err[idx[i]];
    }
  }
  const uint8_t* rf = refine.empty() ? nullptr : refine.data();
  // BF16: the band values are rounded with error feedback along dy.  For each
  // (dx, t, z), walking dy = -R .. R over the entries inside the band, every
  // entry is rounded (to nearest) after adding the rounding error carried
  // from the previous one, so the table's errors cancel in sums over nearby
  // lateral offsets, which is how they reach images that are smooth on the
  // scale of the beam.  Every entry stays a BF16 value within about one unit
  // in the last place of the exact one; H and H^T read the same table.
  std::vector<float> tq;
  const float* tab = taps;
  if (prec == PSOAM_BF16) {
    const int F = g.f;
    tq.assign(taps, taps + (size_t)g.nz * F * F * sir_w);
    for (int z = 0; z < g.nz; ++z)
      for (int jx = 0; jx < F; ++jx)
        for (int t = 0; t < g.nt; ++t) {
          double e = 0.0;
          for (int jy = 0; jy < F; ++jy) {
            const size_t col = ((size_t)z * F + jy) * F + jx;
            const int j = t - t0[col];
            if (j < 0 || j >= sir_w) continue;
            const float v = taps[col * sir_w + j];
            if (v == 0.0f) continue;
            const double w = (double)v + e;
            const float r = from_bf16(to_bf16((float)w));
            // an entry that rounds to zero (values near the float32 underflow)
            // keeps its place in the band, as without the feedback
            tq[col * sir_w + j] = r != 0.0f ? r : v;
            e = w - (double)r;
          }
        }
    tab = tq.data();
  }
  rc = build_table(P, 0, t0, tab, rf, P->fwd);
  if (rc != PSOAM_OK) return bail(rc);
  rc = build_table(P, 1, t0, tab, rf, P->adj);
  if (rc != PSOAM_OK) return bail(rc);
  PLAN_HIP(hipStreamSynchronize(stream));
#undef PLAN_HIP
  *out = P;
  return PSOAM_OK;
}

int create_plan_acoustic(const psoam_geom* gp, const int32_t* t0, const float* taps,
                         int32_t sir_w, int32_t prec, hipStream_t stream, psoam_plan** out) {
  if (!out) return fail(PSOAM_EINVAL, "plan_create_acoustic: out is NULL");
  *out = nullptr;
  if (!gp) return fail(PSOAM_EINVAL, "plan_create_acoustic: NULL argument");
  if (gp->nz <= 0 || gp->n_pulses <= 0) return fail(PSOAM_EINVAL, "plan_create_acoustic: sizes must be positive");
  psoam_geom g = *gp;
  g.n_species = g.n_pulses;  // one volume per pulse
  g.phi_per_voxel = 0;
  g.separable = 0;
  psoam_species sp{};
  std::vector<float> ones((size_t)g.nz, 1.0f);  // S_v = I
  return create_plan_impl(&g, &sp, ones.data(), t0, taps, sir_w, prec, stream, 1, true, out);
}

int create_plan(const psoam_geom* gp, const psoam_species* sp, const float* phi,
                const int32_t* t0, const float* taps, int32_t sir_w, int32_t prec,
                hipStream_t stream, psoam_plan** out) {
  if (!out) return fail(PSOAM_EINVAL, "plan_create: out is NULL");
  *out = nullptr;
  if (!gp || !sp) return fail(PSOAM_EINVAL, "plan_create: NULL argument");
  if (gp->separable != 0 && gp->separable != 1)
    return fail(PSOAM_EINVAL, "plan_create: separable must be 0 or 1");
  if (!gp->separable) return create_plan_impl(gp, sp, phi, t0, taps, sir_w, prec, stream, 0, true, out);
  if (sp->gamma != 0.0)
    return fail(PSOAM_EINVAL, "plan_create: the separable form needs a fluence-independent rate (gamma = 0)");
  // outer plan: geometry with K pulses and the true switching data (prox steps)
  psoam_plan* P = nullptr;
  if (int rc = create_plan_impl(gp, sp, phi, t0, taps, sir_w, prec, stream, 0, false, &P)) return rc;
  // inner plan: the contraction over the S species with S'_v = phi_v I
  psoam_geom gi = *gp;
  gi.n_pulses = gp->n_species;
  gi.separable = 0;
  if (int rc = create_plan_impl(&gi, sp, phi, t0, taps, sir_w, prec, stream, 1, true, &P->inner)) {
    free_plan(P);
    return rc;
  }
  const int K = gp->n_pulses, ns = gp->n_species;
  std::vector<double> T((size_t)K * ns);
  for (int k = 0; k < K; ++k)
    for (int s = 0; s < ns; ++s) T[(size_t)k * ns + s] = sp->a[s] + sp->b[s] * std::exp(-(double)k / sp->tau[s]);
  std::vector<float> Tf(T.begin(), T.end());
  for (int a = 0; a < ns; ++a)
    for (int b = 0; b < ns; ++b) {
      double acc = 0.0;
      for (int k = 0; k < K; ++k) acc += T[(size_t)k * ns + a] * T[(size_t)k * ns + b];
      P->sep_g[a * kMaxSpecies + b] = (float)acc;
    }
  auto bail = [&](hipError_t e, const char* what) {
    free_plan(P);
    return hip_fail(e, what);
  };
  hipError_t e;
  if ((e = hipMalloc(&P->d_T, sizeof(float) * Tf.size())) != hipSuccess) return bail(e, "hipMalloc T");
  if ((e = hipMemcpy(P->d_T, Tf.data(), sizeof(float) * Tf.size(), hipMemcpyHostToDevice)) != hipSuccess)
    return bail(e, "hipMemcpy T");
  float** bufs[] = {&P->d_h, &P->d_rt, &P->d_q};
  for (float** b : bufs)
    if ((e = hipMalloc(b, sizeof(float) * P->h_elems())) != hipSuccess) return bail(e, "hipMalloc separable buffers");
  *out = P;
  return PSOAM_OK;
}

// Factorised acoustic operator (Sec. 2.2.3, eqs. q-above-final, q-below-final):
// the shell membership of every voxel column (z, jdy, jdx) is a run of
// consecutive samples (the radius grows with |t - t_focus| and each column
// sits on one side of the focal plane), so Lambda is a band of eta values
// and goes through the same packing as the impulse-response table; the
// impulse response v is kept for the per-A-scan convolution pass.
int create_plan_factorised(const psoam_geom* gp, const psoam_species* sp, const float* phi,
                           const float* spr, const float* eir, const psoam_shell* sh,
                           int32_t prec, hipStream_t stream, psoam_plan** out) {
  if (!out) return fail(PSOAM_EINVAL, "plan_create_factorised: out is NULL");
  *out = nullptr;
  if (!gp || !sp || !phi || !spr || !eir || !sh)
    return fail(PSOAM_EINVAL, "plan_create_factorised: NULL argument");
  const psoam_geom g = *gp;
  if (g.separable != 0)
    return fail(PSOAM_EUNSUPPORTED, "plan_create_factorised: no separable form of the factorised operator");
  if (g.nx <= 0 || g.ny <= 0 || g.nz <= 0 || g.nt <= 0 || g.n_pulses <= 0)
    return fail(PSOAM_EINVAL, "plan_create_factorised: sizes must be positive");
  if (g.f <= 0 || (g.f % 2) == 0)
    return fail(PSOAM_EINVAL, "plan_create_factorised: footprint f must be odd and positive");
  if (g.nt > kMaxEirNt) return fail(PSOAM_EUNSUPPORTED, "plan_create_factorised: nt above 4096");
  if (!(sh->dr > 0.0) || !std::isfinite(sh->dr))
    return fail(PSOAM_EINVAL, "plan_create_factorised: dr must be finite and > 0");
  if (!std::isfinite(sh->z_focus)) return fail(PSOAM_EINVAL, "plan_create_factorised: z_focus not finite");
  if (sh->t_focus < -(1 << 28) || sh->t_focus > (1 << 28))
    return fail(PSOAM_EINVAL, "plan_create_factorised: t_focus out of range");
  if (sh->n_eir < 1 || sh->n_eir > kMaxEir)
    return fail(PSOAM_EINVAL, "plan_create_factorised: n_eir must be in 1..32");
  if (sh->eir_origin < 0 || sh->eir_origin >= sh->n_eir)
    return fail(PSOAM_EINVAL, "plan_create_factorised: eir_origin outside 0..n_eir-1");
  for (int j = 0; j < sh->n_eir; ++j)
    if (!std::isfinite(eir[j])) return fail(PSOAM_EINVAL, "plan_create_factorised: non-finite eir tap");
  const int F = g.f, R = (F - 1) / 2;
  const size_t ncol = (size_t)g.nz * F * F;
  for (size_t i = 0; i < ncol; ++i)
    if (!std::isfinite(spr[i])) return fail(PSOAM_EINVAL, "plan_create_factorised: non-finite spr entry");
  // nearest and farthest coordinate of the unit box around offset o
  auto near = [](double o) { return std::max(std::fabs(o) - 0.5, 0.0); };
  auto far = [](double o) { return std::fabs(o) + 0.5; };
  std::vector<int32_t> first(ncol, -1), count(ncol, 0);
  int width = 1;
  for (int z = 0; z < g.nz; ++z) {
    const double dz = (double)z - sh->z_focus;
    const double nz2 = near(dz) * near(dz), fz2 = far(dz) * far(dz);
    const bool below = dz >= 0.0;
    for (int jy = 0; jy < F; ++jy) {
      const double oy = (double)(jy - R);
      for (int jx = 0; jx < F; ++jx) {
        const double ox = (double)(jx - R);
        const double dmin2 = (near(oy) * near(oy) + near(ox) * near(ox)) + nz2;
        const double dmax2 = (far(oy) * far(oy) + far(ox) * far(ox)) + fz2;
        const size_t col = ((size_t)z * F + jy) * F + jx;
        for (int t = 0; t < g.nt; ++t) {
          if ((t >= sh->t_focus) != below) continue;
          const double rho = (double)std::abs(t - sh->t_focus) * sh->dr;
          const double rho2 = rho * rho;
          if (!(dmin2 <= rho2 && rho2 <= dmax2)) continue;
          if (first[col] < 0) first[col] = t;
          if (t != first[col] + count[col])
            return fail(PSOAM_EINVAL, "plan_create_factorised: shell samples of a column not consecutive");
          ++count[col];
        }
        width = std::max(width, (int)count[col]);
      }
    }
  }
  if (width > 64)
    return fail(PSOAM_EUNSUPPORTED, "plan_create_factorised: shell band wider than 64 samples (dr too small)");
  std::vector<int32_t> t0(ncol, 0);
  std::vector<float> taps(ncol * (size_t)width, 0.0f);
  for (size_t col = 0; col < ncol; ++col) {
    if (count[col] == 0) continue;
    t0[col] = first[col];
    for (int j = 0; j < count[col]; ++j) taps[col * width + j] = spr[col];
  }
  psoam_plan* P = nullptr;
  if (int rc = create_plan_impl(&g, sp, phi, t0.data(), taps.data(), width, prec, stream, 0, true, &P))
    return rc;
  P->fact = 1;
  P->eir.n = sh->n_eir;
  P->eir.origin = sh->eir_origin;
  for (int j = 0; j < sh->n_eir; ++j) P->eir.v[j] = eir[j];
  P->eir_l1 = 0.0;
  for (int j = 0; j < sh->n_eir; ++j) P->eir_l1 += std::fabs((double)eir[j]);
  hipError_t e = hipMalloc(&P->d_fq, sizeof(float) * P->y_elems());
  if (e != hipSuccess) {
    free_plan(P);
    return hip_fail(e, "hipMalloc factorised buffer");
  }
  *out = P;
  return PSOAM_OK;
}

}  // namespace psoam
