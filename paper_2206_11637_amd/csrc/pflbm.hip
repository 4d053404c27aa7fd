// C ABI of the coupled phase-field LBM step (see include/pflbm.h).
//
// Host side: argument checking, workspace carving, kernel dispatch over the
// compile-time variants (storage type x collision x mask), the bookkeeping of
// the two population buffers and phase-field buffers, and the adjoint.  Every launch goes to the context's stream; the
// library never allocates device memory.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "../../include/pflbm.h"
#include "adjoint.hpp"
#include "kernels.hpp"
#include "probe.hpp"

using namespace pflbm;

namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t v) { return (v + kAlign - 1) / kAlign * kAlign; }

size_t store_size(int precision) { return precision == PFLBM_FP64 ? 8 : precision == PFLBM_FP32 ? 4 : 2; }
size_t real_size(int precision) { return precision == PFLBM_FP64 ? 8 : 4; }

// Tile width of the one-thread-per-cell kernels (bx * by = 256) and the
// number of blocks the step kernel aims for when it splits z into chunks
// (each chunk re-derives two extra phi planes, so fewer, longer chunks cost
// less; enough blocks keep all 256 CUs busy through the tail).
#ifndef PFLBM_TILE_X
#define PFLBM_TILE_X 64
#endif
// each thread of a 256-thread block derives at most one cell of the tile's
// one-cell ring, 2 (bx + 2) + 2 by cells
static_assert(PFLBM_TILE_X >= 16 && PFLBM_TILE_X <= 64 && 256 % PFLBM_TILE_X == 0 &&
                  2 * (PFLBM_TILE_X + 2) + 2 * (256 / PFLBM_TILE_X) <= 256,
              "unsupported tile width");
// the pipelined step keeps the raw h of at most kRingMax ring cells in LDS;
// every tile the host picks (bx = PFLBM_TILE_X, 32 or 16) stays within it
static_assert(2 * (PFLBM_TILE_X + 2) + 2 * (256 / PFLBM_TILE_X) <= kRingMax &&
                  2 * (32 + 2) + 2 * 8 <= kRingMax && 2 * (16 + 2) + 2 * 16 <= kRingMax,
              "ring larger than the pipelined step's LDS slots");
#ifndef PFLBM_STEP_BLOCKS
#define PFLBM_STEP_BLOCKS 2048
#endif
#ifndef PFLBM_MIN_ZC
#define PFLBM_MIN_ZC 4
#endif

// Tile of the one-thread-per-cell kernels (bx * by = 256); narrow grids use
// narrower tiles.
void tile_shape(int nx, int& bx, int& by) {
  bx = nx > 32 ? PFLBM_TILE_X : (nx > 16 ? 32 : 16);
  by = 256 / bx;
}

bool desc_ok(const pflbm_desc* d) {
  if (!d) return false;
  if (d->nx < 1 || d->ny < 1 || d->nz < 1) return false;
  if (d->precision < 0 || d->precision > 2) return false;
  if (d->collision < 0 || d->collision > 1) return false;
  if (d->periodic > 7u) return false;
  if (d->streaming < 0 || d->streaming > 1) return false;
  if (d->forcing < 0 || d->forcing > 1) return false;
  // population addressing uses 32-bit byte offsets within each opposite pair
  // of populations (and within the FP32/FP64 adjoint arrays of one population):
  // 2 N bytes-per-value < 2^32.  The product is bounded factor by factor so
  // that it cannot overflow.
  const long long limit = (1ll << 31) / (d->precision == PFLBM_FP64 ? 8 : 4);
  const long long nxy = (long long)d->nx * d->ny;
  if (nxy >= limit || nxy * d->nz >= limit) return false;
  // one-plane kernels launch a block per (tile, plane): the grid's work-items
  // along x must stay below 2^32 (reached only by thin, heavily padded shapes)
  int bx, by;
  tile_shape(d->nx, bx, by);
  const long long tiles = (long long)((d->nx + bx - 1) / bx) * ((d->ny + by - 1) / by);
  if (tiles * d->nz * 256 >= (1ll << 32)) return false;
  return true;
}

struct Layout {
  int bx, by, tiles_x, tiles_y;
  int zc, nchunks;          // z-chunks of the marching step kernel
  unsigned nblocks;         // one-plane kernels: tiles x nz
  unsigned nblocks_step;    // step kernel: tiles x nchunks
  long long N;
  size_t off_h[2], off_g[2], off_phi[2], off_mask, off_nbr, off_part, off_red, total;
  size_t bytes_h, bytes_g, bytes_phi;
};

Layout make_layout(const pflbm_desc* d) {
  Layout L{};
  tile_shape(d->nx, L.bx, L.by);
  L.tiles_x = (d->nx + L.bx - 1) / L.bx;
  L.tiles_y = (d->ny + L.by - 1) / L.by;
  L.nblocks = (unsigned)L.tiles_x * (unsigned)L.tiles_y * (unsigned)d->nz;
  const long long tiles = (long long)L.tiles_x * L.tiles_y;
  long long nch = (PFLBM_STEP_BLOCKS + tiles - 1) / tiles;
  nch = nch < 1 ? 1 : (nch > d->nz ? d->nz : nch);
  L.zc = (int)((d->nz + nch - 1) / nch);
  if (L.zc < PFLBM_MIN_ZC) L.zc = PFLBM_MIN_ZC < d->nz ? PFLBM_MIN_ZC : d->nz;
  L.nchunks = (d->nz + L.zc - 1) / L.zc;
  L.nblocks_step = (unsigned)(tiles * L.nchunks);
  L.N = (long long)d->nx * d->ny * d->nz;
  const size_t ss = store_size(d->precision), rs = real_size(d->precision);
  L.bytes_h = (size_t)Q_H * L.N * ss;
  L.bytes_g = (size_t)Q_G * L.N * ss;
  L.bytes_phi = (size_t)L.N * rs;
  size_t o = 0;
  const int nbuf = d->streaming == PFLBM_STREAM_AA ? 1 : 2;
  for (int k = 0; k < nbuf; ++k) {
    L.off_h[k] = o; o = align_up(o + L.bytes_h);
    L.off_g[k] = o; o = align_up(o + L.bytes_g);
  }
  if (nbuf == 1) { L.off_h[1] = L.off_h[0]; L.off_g[1] = L.off_g[0]; }
  L.off_phi[0] = o; o = align_up(o + L.bytes_phi);
  L.off_phi[1] = o; o = align_up(o + L.bytes_phi);
  L.off_mask = o; if (d->has_mask) o = align_up(o + (size_t)L.N);
  L.off_nbr = o; if (d->has_mask) o = align_up(o + (size_t)L.N * sizeof(unsigned));
  L.off_part = o; o = align_up(o + (size_t)L.nblocks * 8 * sizeof(double));
  L.off_red = o; o = align_up(o + 8 * sizeof(double));
  L.total = o;
  return L;
}

struct AdjLayout {
  size_t off_lh[2], off_lg[2], off_aphi[2], off_as, off_part, off_gsum, off_red, total;
  size_t bytes_lh, bytes_lg, bytes_aphi, bytes_as;
};

AdjLayout make_adj_layout(const pflbm_desc* d, const Layout& L) {
  AdjLayout A{};
  const size_t rs = real_size(d->precision);
  A.bytes_lh = (size_t)Q_H * L.N * rs;
  A.bytes_lg = (size_t)Q_G * L.N * rs;
  A.bytes_aphi = (size_t)L.N * rs;
  A.bytes_as = (size_t)4 * L.N * rs;
  size_t o = 0;
  for (int k = 0; k < 2; ++k) { A.off_lh[k] = o; o = align_up(o + A.bytes_lh); }
  for (int k = 0; k < 2; ++k) { A.off_lg[k] = o; o = align_up(o + A.bytes_lg); }
  for (int k = 0; k < 2; ++k) { A.off_aphi[k] = o; o = align_up(o + A.bytes_aphi); }
  A.off_as = o; o = align_up(o + A.bytes_as);
  A.off_part = o; o = align_up(o + (size_t)L.nblocks * 3 * sizeof(double));
  A.off_gsum = o; o = align_up(o + (size_t)L.nblocks * 3 * sizeof(double));
  A.off_red = o; o = align_up(o + 8 * sizeof(double));
  A.total = o;
  return A;
}

}  // namespace

struct pflbm_ctx {
  pflbm_desc d;
  pflbm_params p;
  hipStream_t stream;
  Layout L;
  char* ws;
  int pcur = 0;          // population buffer holding the current state
  int iprev = 1;         // phi buffer holding phi^{n-1} (FP16 storage, AA)
  bool phi_ok = false;   // phi^n of the current state has been gathered
  int64_t steps = 0;
  int64_t check_every = 0;
  bool initialised = false;
  bool mask_set = false;
  // adjoint
  char* adj = nullptr;
  AdjLayout A{};
  int acur = 0;
  std::string err;
};

namespace {

pflbm_status fail(pflbm_ctx* c, pflbm_status s, const std::string& msg) {
  if (c) c->err = msg;
  return s;
}

pflbm_status check_hip(pflbm_ctx* c, hipError_t e, const char* where) {
  if (e == hipSuccess) return PFLBM_OK;
  return fail(c, PFLBM_ERR_HIP, std::string(where) + ": " + hipGetErrorString(e));
}

Geom make_geom(const pflbm_ctx* c) {
  Geom G;
  G.nx = c->d.nx; G.ny = c->d.ny; G.nz = c->d.nz;
  G.px = (c->d.periodic >> 0) & 1; G.py = (c->d.periodic >> 1) & 1; G.pz = (c->d.periodic >> 2) & 1;
  G.bx = c->L.bx; G.by = c->L.by;
  G.tiles_x = c->L.tiles_x; G.tiles_y = c->L.tiles_y;
  G.nblocks = c->L.nblocks;
  G.zc = c->L.zc; G.nchunks = c->L.nchunks;
  G.nblocks_step = c->L.nblocks_step;
  G.N = c->L.N;
  return G;
}

template <typename R>
Phys<R> make_phys(const pflbm_params& p, int32_t collision) {
  Phys<R> P;
  const bool inf_xi = std::isinf(p.xi);
  P.tau_L = R(p.tau_L);
  P.dtau = R(p.tau_H - p.tau_L);
  P.rho_L = R(p.rho_L);
  P.drho = R(p.rho_H - p.rho_L);
  P.theta_k = inf_xi ? R(0) : R(4.0 / p.xi);
  P.beta4 = inf_xi ? R(0) : R(48.0 * p.sigma / p.xi);
  P.kappa = inf_xi ? R(0) : R(1.5 * p.sigma * p.xi);
  P.gx = R(p.g[0]); P.gy = R(p.g[1]); P.gz = R(p.g[2]);
  P.omega_phi = R(1.0 / (3.0 * p.mobility + 0.5));
  P.s_high = R(p.s_high);
  P.eps2 = R(p.normal_eps * p.normal_eps);
  P.s_bulk = collision == PFLBM_MRT ? R(p.s_bulk) : R(0);
  P.rho_gref = R(p.rho_g_ref);
  return P;
}

template <typename R>
Codec<R> make_codec(const pflbm_ctx* c) {
  Codec<R> cd;
  const bool f16 = c->d.precision == PFLBM_FP32_FP16S;
  const double kh = f16 ? c->p.fp16_scale_log2[0] : 0.0, kg = f16 ? c->p.fp16_scale_log2[1] : 0.0;
  cd.scale_h = R(std::ldexp(1.0, (int)kh));
  cd.inv_scale_h = R(std::ldexp(1.0, -(int)kh));
  cd.scale_g = R(std::ldexp(1.0, (int)kg));
  cd.inv_scale_g = R(std::ldexp(1.0, -(int)kg));
  return cd;
}

// FP32 and FP16 storage keep h shifted by w_i times a phase field one step old
bool shifted(const pflbm_ctx* c) { return c->d.precision != PFLBM_FP64; }
bool is_aa(const pflbm_ctx* c) { return c->d.streaming == PFLBM_STREAM_AA; }

template <typename S> S* pop_h(pflbm_ctx* c, int k) { return reinterpret_cast<S*>(c->ws + c->L.off_h[k]); }
template <typename S> S* pop_g(pflbm_ctx* c, int k) { return reinterpret_cast<S*>(c->ws + c->L.off_g[k]); }
template <typename R> R* phi_buf(pflbm_ctx* c, int k) { return reinterpret_cast<R*>(c->ws + c->L.off_phi[k]); }
unsigned char* mask_ptr(pflbm_ctx* c) {
  return c->d.has_mask ? reinterpret_cast<unsigned char*>(c->ws + c->L.off_mask) : nullptr;
}
unsigned* nbr_ptr(pflbm_ctx* c) {
  return c->d.has_mask ? reinterpret_cast<unsigned*>(c->ws + c->L.off_nbr) : nullptr;
}
// phi buffer that holds (or receives) phi^n of the current state; the other
// one holds phi^{n-1} where a step needs it (FP16 shifts, and the AA step,
// which forms phi^{n+1} into it)
int phi_cur_idx(const pflbm_ctx* c) { return (shifted(c) || is_aa(c)) ? (c->iprev ^ 1) : 0; }
template <typename R> R* phi_cur(pflbm_ctx* c) { return phi_buf<R>(c, phi_cur_idx(c)); }
template <typename R> R* phi_prev(pflbm_ctx* c) { return shifted(c) ? phi_buf<R>(c, c->iprev) : nullptr; }

// A saved state: h, g, phi^n and, for FP16 storage, phi^{n-1}.
struct StateView { size_t oh, og, ophi, oprev, total; };
StateView state_view(const pflbm_ctx* c) {
  StateView v;
  v.oh = 0;
  v.og = c->L.bytes_h;
  v.ophi = c->L.bytes_h + c->L.bytes_g;
  v.oprev = v.ophi + c->L.bytes_phi;
  v.total = v.oprev + (shifted(c) ? c->L.bytes_phi : 0);
  return v;
}

// ---- launch helpers ----------------------------------------------------------
template <typename S>
StepArgs<S> step_args(pflbm_ctx* c) {
  using R = typename Store<S>::R;
  StepArgs<S> a;
  a.h_in = pop_h<S>(c, c->pcur);
  a.g_in = pop_g<S>(c, c->pcur);
  a.h_out = pop_h<S>(c, c->pcur ^ 1);
  a.g_out = pop_g<S>(c, c->pcur ^ 1);
  a.phi_prev = phi_prev<R>(c);
  a.phi_out = shifted(c) ? phi_buf<R>(c, c->iprev ^ 1) : nullptr;
  a.phi_src_out = nullptr;
  a.nbr = nbr_ptr(c);
  a.geo = make_geom(c);
  a.P = make_phys<R>(c->p, c->d.collision);
  a.cd = make_codec<R>(c);
  return a;
}

template <typename S, bool MRT, bool GUO>
void launch_step_k(pflbm_ctx* c, const StepArgs<S>& a, dim3 grd, dim3 blk, size_t sm) {
  if constexpr (DmaStep<S>::value) {
    if (c->d.has_mask) hipLaunchKernelGGL((k_step_dma<S, MRT, true, GUO>), grd, blk, sm, c->stream, a);
    else hipLaunchKernelGGL((k_step_dma<S, MRT, false, GUO>), grd, blk, sm, c->stream, a);
  } else {
    if (c->d.has_mask) hipLaunchKernelGGL((k_step<S, MRT, true, GUO>), grd, blk, sm, c->stream, a);
    else hipLaunchKernelGGL((k_step<S, MRT, false, GUO>), grd, blk, sm, c->stream, a);
  }
}

template <typename S>
void launch_step(pflbm_ctx* c, const StepArgs<S>& a) {
  using R = typename Store<S>::R;
  // 4-plane phi ring, + two planes of the threads' own h where the kernel
  // keeps them in dynamic LDS (the pipelined kernel's raw slots are static)
  const size_t ring = (size_t)4 * (c->L.bx + 2) * (c->L.by + 2);
  const size_t sm = (ring + (DmaStep<S>::value ? 0 : 2 * Q_H * 256)) * sizeof(R);
  const dim3 blk(c->L.bx, c->L.by), grd(c->L.nblocks_step);
  const bool mrt = c->d.collision == PFLBM_MRT, guo = c->d.forcing == PFLBM_FORCING_GUO;
  if (mrt) {
    if (guo) launch_step_k<S, true, true>(c, a, grd, blk, sm);
    else launch_step_k<S, true, false>(c, a, grd, blk, sm);
  } else {
    if (guo) launch_step_k<S, false, true>(c, a, grd, blk, sm);
    else launch_step_k<S, false, false>(c, a, grd, blk, sm);
  }
}

// the state advanced by one step: buffers swap, phi^n becomes the shift
// reference, phi^{n+1} is not gathered yet
void advance(pflbm_ctx* c) {
  c->pcur ^= 1;
  if (shifted(c)) c->iprev ^= 1;
  c->phi_ok = false;
  c->steps += 1;
}

template <typename S>
LightArgs<S> light_args(pflbm_ctx* c) {
  using R = typename Store<S>::R;
  LightArgs<S> a;
  a.h = pop_h<S>(c, c->pcur);
  a.g = pop_g<S>(c, c->pcur);
  a.nbr = nbr_ptr(c);
  a.phi_prev = phi_prev<R>(c);
  a.geo = make_geom(c);
  a.cd = make_codec<R>(c);
  a.phi_out = nullptr;
  a.out_h = a.out_g = nullptr;
  a.partials = nullptr;
  return a;
}

// read rule of a state after `steps` steps
int state_rule(const pflbm_ctx* c, int64_t steps) {
  return !is_aa(c) ? RULE_AB : ((steps & 1) ? RULE_AA_ODD : RULE_AA_EVEN);
}

template <typename S, int LM, int RULE>
void launch_light_r(pflbm_ctx* c, const LightArgs<S>& a) {
  const dim3 blk(c->L.bx, c->L.by), grd(c->L.nblocks);
  if (c->d.has_mask) hipLaunchKernelGGL((k_light<S, RULE, true, LM>), grd, blk, 0, c->stream, a);
  else hipLaunchKernelGGL((k_light<S, RULE, false, LM>), grd, blk, 0, c->stream, a);
}

template <typename S, int LM>
void launch_light(pflbm_ctx* c, const LightArgs<S>& a, int rule) {
  if (rule == RULE_AB) launch_light_r<S, LM, RULE_AB>(c, a);
  else if (rule == RULE_AA_ODD) launch_light_r<S, LM, RULE_AA_ODD>(c, a);
  else launch_light_r<S, LM, RULE_AA_EVEN>(c, a);
}

// phi^n of the current state (sum of the h its next step reads), gathered on
// demand
template <typename S>
void ensure_phi(pflbm_ctx* c) {
  using R = typename Store<S>::R;
  if (c->phi_ok) return;
  LightArgs<S> a = light_args<S>(c);
  a.phi_out = phi_cur<R>(c);
  launch_light<S, LM_GATHER>(c, a, state_rule(c, c->steps));
  c->phi_ok = true;
}

// ---- AA step ------------------------------------------------------------------
template <typename S>
CellArgs<S> aa_args(pflbm_ctx* c) {
  using R = typename Store<S>::R;
  CellArgs<S> a;
  a.h_in = a.h = pop_h<S>(c, 0);
  a.g_in = a.g = pop_g<S>(c, 0);
  a.phi = phi_cur<R>(c);
  a.phi_prev = phi_prev<R>(c);
  a.mask = mask_ptr(c);
  a.geo = make_geom(c);
  a.P = make_phys<R>(c->p, c->d.collision);
  a.cd = make_codec<R>(c);
  a.out_phi = a.out_u = a.out_p = nullptr;
  return a;
}

template <typename S, bool MRT, bool ODD, bool GUO>
void launch_aa_g(pflbm_ctx* c, const CellArgs<S>& a) {
  using R = typename Store<S>::R;
  const size_t sm = (size_t)(c->L.bx + 2) * (c->L.by + 2) * 3 * sizeof(R);
  const dim3 blk(c->L.bx, c->L.by), grd(c->L.nblocks);
  if (c->d.has_mask) hipLaunchKernelGGL((k_cell_aa<S, MRT, ODD, true, GUO>), grd, blk, sm, c->stream, a);
  else hipLaunchKernelGGL((k_cell_aa<S, MRT, ODD, false, GUO>), grd, blk, sm, c->stream, a);
}

template <typename S, bool MRT, bool ODD>
void launch_aa_m(pflbm_ctx* c, const CellArgs<S>& a) {
  if (c->d.forcing == PFLBM_FORCING_GUO) launch_aa_g<S, MRT, ODD, true>(c, a);
  else launch_aa_g<S, MRT, ODD, false>(c, a);
}

template <typename S>
void launch_aa(pflbm_ctx* c, const CellArgs<S>& a, bool odd) {
  if (c->d.collision == PFLBM_MRT) {
    if (odd) launch_aa_m<S, true, true>(c, a); else launch_aa_m<S, true, false>(c, a);
  } else {
    if (odd) launch_aa_m<S, false, true>(c, a); else launch_aa_m<S, false, false>(c, a);
  }
}

// phi^{n+1} after an AA step, into the buffer of phi^{n-1}; phi^n becomes the
// shift reference of the new state
template <typename S>
void aa_gather(pflbm_ctx* c) {
  using R = typename Store<S>::R;
  LightArgs<S> a = light_args<S>(c);
  a.phi_prev = phi_buf<R>(c, c->iprev ^ 1);
  a.phi_out = phi_buf<R>(c, c->iprev);
  launch_light<S, LM_GATHER>(c, a, state_rule(c, c->steps));
  c->iprev ^= 1;
  c->phi_ok = true;
}

// one step of the context's state with either scheme; the AA phi pass is
// timed separately when events are given
template <typename S>
void one_step(pflbm_ctx* c, hipEvent_t mid = nullptr) {
  if (!is_aa(c)) {
    launch_step<S>(c, step_args<S>(c));
    advance(c);
    return;
  }
  launch_aa<S>(c, aa_args<S>(c), c->steps & 1);
  if (mid) (void)hipEventRecord(mid, c->stream);
  c->steps += 1;
  aa_gather<S>(c);
}

template <typename S>
pflbm_status do_reduce(pflbm_ctx* c, double* out_host);

template <typename S>
pflbm_status do_steps(pflbm_ctx* c, int64_t n) {
  for (int64_t s = 0; s < n; ++s) {
    one_step<S>(c);
    if (c->check_every > 0 && c->steps % c->check_every == 0) {
      double r[5];
      const pflbm_status st = do_reduce<S>(c, r);
      if (st == PFLBM_ERR_UNSTABLE)
        return fail(c, st, "non-finite sum(phi) or sum(p*) after step " + std::to_string(c->steps));
      if (st) return st;
    }
  }
  return check_hip(c, hipGetLastError(), "pflbm_step");
}

// One step from a saved state (level n) into another saved-state buffer
// (level n + 1), leaving the context's own state untouched.
//   AB: the step kernel writes dst's populations (and, for FP16 storage,
//       phi^n as dst's shift reference), then phi^{n+1} is gathered into dst.
//   AA: the collide-and-stream kernel runs out of place (each slot is written
//       exactly once, so dst needs no copy of src), phi^{n+1} is gathered with
//       the writers' phi^n from src, and src's phi^n becomes dst's reference.
template <typename S>
pflbm_status do_step_states(pflbm_ctx* c, void* src, void* dst, int64_t n, int32_t flags) {
  using R = typename Store<S>::R;
  char* s = static_cast<char*>(src);
  char* d = static_cast<char*>(dst);
  const StateView v = state_view(c);
  const S* hs = reinterpret_cast<const S*>(s + v.oh);
  const S* gs = reinterpret_cast<const S*>(s + v.og);
  S* hd = reinterpret_cast<S*>(d + v.oh);
  S* gd = reinterpret_cast<S*>(d + v.og);
  LightArgs<S> b = light_args<S>(c);
  b.h = hd;
  b.g = gd;
  b.phi_out = reinterpret_cast<R*>(d + v.ophi);
  if (!is_aa(c)) {
    StepArgs<S> a = step_args<S>(c);
    a.h_in = hs;
    a.g_in = gs;
    a.h_out = hd;
    a.g_out = gd;
    a.phi_prev = shifted(c) ? reinterpret_cast<const R*>(s + v.oprev) : nullptr;
    a.phi_out = shifted(c) ? reinterpret_cast<R*>(d + v.oprev) : nullptr;
    if (flags & PFLBM_STATES_WRITE_SRC_PHI) a.phi_src_out = reinterpret_cast<R*>(s + v.ophi);
    launch_step<S>(c, a);
    b.phi_prev = a.phi_out;
    if (!(flags & PFLBM_STATES_SKIP_DST_PHI)) launch_light<S, LM_GATHER>(c, b, RULE_AB);
  } else {
    CellArgs<S> a = aa_args<S>(c);
    a.h_in = hs;
    a.g_in = gs;
    a.h = hd;
    a.g = gd;
    a.phi = reinterpret_cast<const R*>(s + v.ophi);
    a.phi_prev = shifted(c) ? reinterpret_cast<const R*>(s + v.oprev) : nullptr;
    launch_aa<S>(c, a, n & 1);
    b.phi_prev = a.phi;
    launch_light<S, LM_GATHER>(c, b, state_rule(c, n + 1));
    if (shifted(c)) {
      const hipError_t e = hipMemcpyAsync(d + v.oprev, s + v.ophi, c->L.bytes_phi, hipMemcpyDeviceToDevice,
                                          c->stream);
      if (e != hipSuccess) return check_hip(c, e, "pflbm_step_states copy");
    }
  }
  return check_hip(c, hipGetLastError(), "pflbm_step_states");
}

template <typename S>
pflbm_status do_profile(pflbm_ctx* c, int64_t n, double* out_ms) {
  // events around every launch, read back once at the end (no per-step sync)
  std::vector<hipEvent_t> ev;
  try {
    ev.resize((size_t)(2 * n + 1), nullptr);
  } catch (...) {
    return fail(c, PFLBM_ERR_ARG, "pflbm_profile_step: too many steps for the host event list");
  }
  for (size_t k = 0; k < ev.size(); ++k) {
    if (pflbm_status s = check_hip(c, hipEventCreate(&ev[k]), "pflbm_profile_step event")) {
      for (size_t j = 0; j < k; ++j) (void)hipEventDestroy(ev[j]);
      return s;
    }
  }
  (void)hipEventRecord(ev[0], c->stream);
  for (int64_t s = 0; s < n; ++s) {
    one_step<S>(c, ev[2 * s + 1]);
    if (!is_aa(c)) (void)hipEventRecord(ev[2 * s + 1], c->stream);
    (void)hipEventRecord(ev[2 * s + 2], c->stream);
  }
  pflbm_status st = check_hip(c, hipEventSynchronize(ev[2 * n]), "pflbm_profile_step");
  double acc[3] = {0.0, 0.0, 0.0};
  for (int64_t s = 0; s < n && !st; ++s) {
    float t0 = 0.f, t1 = 0.f;
    (void)hipEventElapsedTime(&t0, ev[2 * s], ev[2 * s + 1]);
    (void)hipEventElapsedTime(&t1, ev[2 * s + 1], ev[2 * s + 2]);
    acc[0] += t0;
    acc[1] += t1;
  }
  if (!st && n > 0) {
    float t = 0.f;
    (void)hipEventElapsedTime(&t, ev[0], ev[2 * n]);
    acc[2] = t;
  }
  for (auto& e : ev) (void)hipEventDestroy(e);
  for (int k = 0; k < 3; ++k) out_ms[k] = acc[k];
  if (st) return st;
  return check_hip(c, hipGetLastError(), "pflbm_profile_step");
}

template <typename S>
pflbm_status do_init(pflbm_ctx* c, const double* phi0, const double* u0, const double* p0) {
  using R = typename Store<S>::R;
  c->pcur = 0;
  c->iprev = 1;
  InitArgs<S> a;
  a.h = pop_h<S>(c, 0);
  a.g = pop_g<S>(c, 0);
  a.nbr = nbr_ptr(c);
  a.phi0 = phi0;
  a.u0 = u0;
  a.p0 = p0;
  a.phi_ref = phi_prev<R>(c);
  a.geo = make_geom(c);
  a.cd = make_codec<R>(c);
  // shifted forms: R(phi0) plays phi^{-1}, the shift reference of the initial
  // populations
  if (shifted(c)) {
    const unsigned nb = (unsigned)((c->L.N + 255) / 256);
    hipLaunchKernelGGL(k_phi_from_f64<R>, dim3(nb), dim3(256), 0, c->stream, phi0, mask_ptr(c), c->L.N,
                       phi_buf<R>(c, c->iprev));
  }
  const dim3 blk(c->L.bx, c->L.by), grd(c->L.nblocks);
  const bool m = c->d.has_mask;
  if (is_aa(c)) {
    if (m) hipLaunchKernelGGL((k_init<S, true, true>), grd, blk, 0, c->stream, a);
    else hipLaunchKernelGGL((k_init<S, true, false>), grd, blk, 0, c->stream, a);
  } else {
    if (m) hipLaunchKernelGGL((k_init<S, false, true>), grd, blk, 0, c->stream, a);
    else hipLaunchKernelGGL((k_init<S, false, false>), grd, blk, 0, c->stream, a);
  }
  c->steps = 0;
  c->phi_ok = false;
  ensure_phi<S>(c);
  const pflbm_status s = check_hip(c, hipGetLastError(), "pflbm_init_equilibrium");
  c->initialised = s == PFLBM_OK;
  return s;
}

template <typename S, int RULE>
void launch_moments(pflbm_ctx* c, const CellArgs<S>& a) {
  using R = typename Store<S>::R;
  const size_t sm = (size_t)(c->L.bx + 2) * (c->L.by + 2) * 3 * sizeof(R);
  const dim3 blk(c->L.bx, c->L.by), grd(c->L.nblocks);
  if (c->d.has_mask) hipLaunchKernelGGL((k_moments<S, RULE, true>), grd, blk, sm, c->stream, a);
  else hipLaunchKernelGGL((k_moments<S, RULE, false>), grd, blk, sm, c->stream, a);
}

template <typename S>
pflbm_status do_moments(pflbm_ctx* c, double* phi, double* u, double* p) {
  ensure_phi<S>(c);
  CellArgs<S> a = aa_args<S>(c);
  a.h_in = pop_h<S>(c, c->pcur);
  a.g_in = pop_g<S>(c, c->pcur);
  a.out_phi = phi;
  a.out_u = u;
  a.out_p = p;
  const int rule = state_rule(c, c->steps);
  if (rule == RULE_AB) launch_moments<S, RULE_AB>(c, a);
  else if (rule == RULE_AA_ODD) launch_moments<S, RULE_AA_ODD>(c, a);
  else launch_moments<S, RULE_AA_EVEN>(c, a);
  return check_hip(c, hipGetLastError(), "pflbm_read_moments");
}

template <typename S>
pflbm_status do_read_phi(pflbm_ctx* c, double* d_phi) {
  using R = typename Store<S>::R;
  ensure_phi<S>(c);
  const unsigned nb = (unsigned)((c->L.N + 255) / 256);
  hipLaunchKernelGGL(k_phi_to_f64<R>, dim3(nb), dim3(256), 0, c->stream, phi_cur<R>(c), c->L.N, d_phi);
  return check_hip(c, hipGetLastError(), "pflbm_read_phi");
}

template <typename S>
pflbm_status do_read_pops(pflbm_ctx* c, double* h, double* g) {
  LightArgs<S> a = light_args<S>(c);
  a.out_h = h;
  a.out_g = g;
  launch_light<S, LM_READ_POPS>(c, a, state_rule(c, c->steps));
  return check_hip(c, hipGetLastError(), "pflbm_read_populations");
}

template <typename S>
pflbm_status do_save_state(pflbm_ctx* c, void* dst) {
  using R = typename Store<S>::R;
  ensure_phi<S>(c);
  char* o = static_cast<char*>(dst);
  const StateView v = state_view(c);
  hipError_t e = hipMemcpyAsync(o + v.oh, pop_h<S>(c, c->pcur), c->L.bytes_h, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(o + v.og, pop_g<S>(c, c->pcur), c->L.bytes_g, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(o + v.ophi, phi_cur<R>(c), c->L.bytes_phi, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && shifted(c))
    e = hipMemcpyAsync(o + v.oprev, phi_prev<R>(c), c->L.bytes_phi, hipMemcpyDeviceToDevice, c->stream);
  return check_hip(c, e, "pflbm_save_state");
}

// FP64 sums of the current state into `red` (5 doubles) through the per-block
// partials `part` (nblocks x 5 doubles), then to the host.
template <typename S>
pflbm_status do_reduce_via(pflbm_ctx* c, double* part, double* red, double* out_host) {
  LightArgs<S> a = light_args<S>(c);
  a.partials = part;
  launch_light<S, LM_REDUCE>(c, a, state_rule(c, c->steps));
  hipLaunchKernelGGL(k_reduce_final, dim3(1), dim3(1024), 0, c->stream, part, c->L.nblocks, 5, red);
  pflbm_status s = check_hip(c, hipGetLastError(), "pflbm_reduce launch");
  if (s) return s;
  s = check_hip(c, hipMemcpyAsync(out_host, red, 5 * sizeof(double), hipMemcpyDeviceToHost, c->stream),
                "pflbm_reduce copy");
  if (s) return s;
  s = check_hip(c, hipStreamSynchronize(c->stream), "pflbm_reduce sync");
  if (s) return s;
  for (int k = 0; k < 5; ++k)
    if (!std::isfinite(out_host[k])) return fail(c, PFLBM_ERR_UNSTABLE, "non-finite reduction");
  return PFLBM_OK;
}

template <typename S>
pflbm_status do_reduce(pflbm_ctx* c, double* out_host) {
  return do_reduce_via<S>(c, reinterpret_cast<double*>(c->ws + c->L.off_part),
                          reinterpret_cast<double*>(c->ws + c->L.off_red), out_host);
}

// ---- the allocation-free reduction -------------------------------------------
// pflbm_reduce_static keeps its partial sums in this file-scope device array
// instead of the context's workspace.  Each GPU holds its own copy, whose
// address is looked up once per device (hipGetSymbolAddress, with that device
// current) and kept; in host code the array's name is not a device address.
constexpr size_t kStaticScratchBytes = size_t(16) << 20;
__device__ __align__(256) unsigned char scratch[kStaticScratchBytes];
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// bytes of scratch the reduction of a lattice with this layout needs: one
// 5-double partial per (tile, plane) block, then the 5 sums
size_t static_scratch_bytes(const Layout& L) {
  return align_up((size_t)L.nblocks * 5 * sizeof(double)) + align_up(8 * sizeof(double));
}

// device address of `scratch` on device dev
pflbm_status scratch_of(pflbm_ctx* c, int dev, char** out) {
  if (dev < 0 || dev >= kMaxDevices) return fail(c, PFLBM_ERR_STATE, "device index out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    int cur = -1;
    if (pflbm_status s = check_hip(c, hipGetDevice(&cur), "pflbm_reduce_static device")) return s;
    if (cur != dev)
      if (pflbm_status s = check_hip(c, hipSetDevice(dev), "pflbm_reduce_static set device")) return s;
    void* p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (cur != dev) (void)hipSetDevice(cur);
    if (pflbm_status s = check_hip(c, e, "pflbm_reduce_static symbol address")) return s;
    if (!p) return fail(c, PFLBM_ERR_HIP, "pflbm_reduce_static: null scratch address");
    g_scratch_ptr[dev] = p;
  }
  *out = static_cast<char*>(g_scratch_ptr[dev]);
  return PFLBM_OK;
}

#define DISPATCH(c, fn, ...)                                     \
  do {                                                           \
    switch ((c)->d.precision) {                                  \
      case PFLBM_FP64: return fn<double>(__VA_ARGS__);           \
      case PFLBM_FP32: return fn<float>(__VA_ARGS__);            \
      default: return fn<_Float16>(__VA_ARGS__);                 \
    }                                                            \
  } while (0)

pflbm_status params_ok(const pflbm_params* p, std::string& why) {
  if (!p) { why = "params is NULL"; return PFLBM_ERR_ARG; }
  auto bad = [&](bool cond, const char* m) { if (cond) why = m; return cond; };
  if (bad(!(p->tau_H > 0.5) || !(p->tau_L > 0.5), "tau must be > 1/2")) return PFLBM_ERR_ARG;
  if (bad(!(p->mobility > 0) || !std::isfinite(p->mobility), "mobility must be > 0")) return PFLBM_ERR_ARG;
  if (bad(!(p->xi > 0), "xi must be > 0")) return PFLBM_ERR_ARG;
  if (bad(!(p->sigma >= 0) || !std::isfinite(p->sigma), "sigma must be >= 0")) return PFLBM_ERR_ARG;
  if (bad(!(p->rho_H > 0) || !(p->rho_L > 0), "densities must be > 0")) return PFLBM_ERR_ARG;
  if (bad(!(p->s_high > 0 && p->s_high < 2), "s_high must lie in (0, 2)")) return PFLBM_ERR_ARG;
  if (bad(!(p->normal_eps > 0) || !std::isfinite(p->normal_eps), "normal_eps must be > 0"))
    return PFLBM_ERR_ARG;
  if (bad(!(p->s_bulk == 0 || (p->s_bulk > 0 && p->s_bulk < 2)), "s_bulk must be 0 or lie in (0, 2)"))
    return PFLBM_ERR_ARG;
  for (int k = 0; k < 3; ++k)
    if (bad(!std::isfinite(p->g[k]), "g must be finite")) return PFLBM_ERR_ARG;
  if (bad(!std::isfinite(p->rho_g_ref), "rho_g_ref must be finite")) return PFLBM_ERR_ARG;
  for (int k = 0; k < 2; ++k) {
    const double v = p->fp16_scale_log2[k];
    if (bad(!(std::fabs(v) <= 24) || v != std::floor(v), "fp16_scale_log2 must be integers in [-24, 24]"))
      return PFLBM_ERR_ARG;
  }
  return PFLBM_OK;
}

// rows of the halo pack: per face the h, then the g directions with c_z = -1
// (face 0, plane 0) or +1 (face 1, plane nz - 1), in table order
PackRows pack_rows() {
  PackRows r{};
  for (int f = 0; f < 2; ++f) {
    const int dz = f ? 1 : -1;
    int n = 0;
    for (int i = 0; i < Q_H; ++i)
      if (ch(i).z == dz) r.pop[f][n++] = i;
    r.nh = n;
    for (int i = 0; i < Q_G; ++i)
      if (cg(i).z == dz) r.pop[f][n++] = i;
    r.n = n;
  }
  return r;
}

template <typename S>
pflbm_status do_pack_faces(pflbm_ctx* c, void* dst) {
  const PackRows r = pack_rows();
  const long long nxy = (long long)c->d.nx * c->d.ny;
  const dim3 grid((unsigned)((nxy + 255) / 256), (unsigned)(2 * r.n));
  hipLaunchKernelGGL(k_pack_faces<S>, grid, dim3(256), 0, c->stream, pop_h<S>(c, c->pcur), pop_g<S>(c, c->pcur),
                     static_cast<S*>(dst), c->L.N, nxy, c->d.nz, r);
  return check_hip(c, hipGetLastError(), "pflbm_pack_faces");
}

}  // namespace

// ============================================================================
extern "C" {

size_t pflbm_workspace_bytes(const pflbm_desc* desc) {
  if (!desc_ok(desc)) return 0;
  return make_layout(desc).total;
}

pflbm_status pflbm_create(const pflbm_desc* desc, void* d_workspace, size_t bytes,
                          void* hip_stream, pflbm_ctx** out) {
  if (!out) return PFLBM_ERR_ARG;
  *out = nullptr;
  if (!desc_ok(desc) || !d_workspace) return PFLBM_ERR_ARG;
  const Layout L = make_layout(desc);
  if (bytes < L.total || (reinterpret_cast<uintptr_t>(d_workspace) % kAlign) != 0) return PFLBM_ERR_ARG;
  pflbm_ctx* c = new (std::nothrow) pflbm_ctx();
  if (!c) return PFLBM_ERR_ARG;
  c->d = *desc;
  c->L = L;
  c->ws = static_cast<char*>(d_workspace);
  c->stream = static_cast<hipStream_t>(hip_stream);
  pflbm_params p{};
  p.tau_H = p.tau_L = 0.53;
  p.mobility = 0.02;
  p.xi = 4.0;
  p.sigma = 1e-4;
  p.rho_H = 1.0;
  p.rho_L = 1e-3;
  p.s_high = 1.0;
  p.fp16_scale_log2[0] = 12;
  p.fp16_scale_log2[1] = 12;
  p.normal_eps = 1e-4;
  p.s_bulk = 0.0;
  p.rho_g_ref = 0.0;
  c->p = p;
  *out = c;
  return PFLBM_OK;
}

pflbm_status pflbm_destroy(pflbm_ctx* ctx) {
  if (!ctx) return PFLBM_ERR_ARG;
  delete ctx;
  return PFLBM_OK;
}

pflbm_status pflbm_set_params(pflbm_ctx* c, const pflbm_params* p) {
  if (!c) return PFLBM_ERR_ARG;
  std::string why;
  if (pflbm_status s = params_ok(p, why)) return fail(c, s, why);
  // the stored FP16 populations are scaled by 2^k: a new k would silently
  // rescale the state (and saved states) by 2^(k_old - k_new)
  if (c->d.precision == PFLBM_FP32_FP16S && c->initialised &&
      (p->fp16_scale_log2[0] != c->p.fp16_scale_log2[0] || p->fp16_scale_log2[1] != c->p.fp16_scale_log2[1]))
    return fail(c, PFLBM_ERR_STATE,
                "fp16_scale_log2 cannot change once the FP16-storage state is initialised "
                "(initialise again with the new scale)");
  c->p = *p;
  return PFLBM_OK;
}

pflbm_status pflbm_set_mask(pflbm_ctx* c, const uint8_t* d_solid) {
  if (!c) return PFLBM_ERR_ARG;
  if (!c->d.has_mask) return fail(c, PFLBM_ERR_STATE, "context created without a mask");
  if (!d_solid) return fail(c, PFLBM_ERR_ARG, "mask pointer is NULL");
  pflbm_status s = check_hip(c, hipMemcpyAsync(mask_ptr(c), d_solid, (size_t)c->L.N,
                                               hipMemcpyDeviceToDevice, c->stream), "pflbm_set_mask");
  if (s) return s;
  const unsigned nb = (unsigned)((c->L.N + 255) / 256);
  hipLaunchKernelGGL(k_nbr_bits, dim3(nb), dim3(256), 0, c->stream, mask_ptr(c), make_geom(c), nbr_ptr(c));
  s = check_hip(c, hipGetLastError(), "pflbm_set_mask");
  if (!s) c->mask_set = true;
  return s;
}

pflbm_status pflbm_init_equilibrium(pflbm_ctx* c, const double* phi0, const double* u0,
                                    const double* p0) {
  if (!c) return PFLBM_ERR_ARG;
  if (!phi0) return fail(c, PFLBM_ERR_ARG, "phi0 is NULL");
  if (c->d.has_mask && !c->mask_set) return fail(c, PFLBM_ERR_STATE, "mask not set");
  DISPATCH(c, do_init, c, phi0, u0, p0);
}

pflbm_status pflbm_set_check_interval(pflbm_ctx* c, int64_t every) {
  if (!c) return PFLBM_ERR_ARG;
  if (every < 0) return fail(c, PFLBM_ERR_ARG, "negative check interval");
  c->check_every = every;
  return PFLBM_OK;
}

pflbm_status pflbm_step(pflbm_ctx* c, int64_t n) {
  if (!c) return PFLBM_ERR_ARG;
  if (n < 0) return fail(c, PFLBM_ERR_ARG, "negative step count");
  if (!c->initialised) return fail(c, PFLBM_ERR_STATE, "not initialised");
  DISPATCH(c, do_steps, c, n);
}

pflbm_status pflbm_profile_step(pflbm_ctx* c, int64_t n, double* out_ms) {
  if (!c) return PFLBM_ERR_ARG;
  if (n < 0 || !out_ms) return fail(c, PFLBM_ERR_ARG, "bad step count or output");
  if (!c->initialised) return fail(c, PFLBM_ERR_STATE, "not initialised");
  DISPATCH(c, do_profile, c, n, out_ms);
}

pflbm_status pflbm_read_moments(pflbm_ctx* c, double* phi, double* u, double* p) {
  if (!c) return PFLBM_ERR_ARG;
  if (!c->initialised) return fail(c, PFLBM_ERR_STATE, "not initialised");
  DISPATCH(c, do_moments, c, phi, u, p);
}

pflbm_status pflbm_read_phi(pflbm_ctx* c, double* d_phi) {
  if (!c) return PFLBM_ERR_ARG;
  if (!d_phi) return fail(c, PFLBM_ERR_ARG, "output is NULL");
  if (!c->initialised) return fail(c, PFLBM_ERR_STATE, "not initialised");
  DISPATCH(c, do_read_phi, c, d_phi);
}

pflbm_status pflbm_pack_faces(pflbm_ctx* c, void* dst, size_t dst_bytes, size_t* bytes_needed) {
  if (!c) return PFLBM_ERR_ARG;
  if (!bytes_needed) return fail(c, PFLBM_ERR_ARG, "pflbm_pack_faces: bytes_needed is NULL");
  const size_t need = (size_t)2 * pack_rows().n * (size_t)c->d.nx * (size_t)c->d.ny * store_size(c->d.precision);
  *bytes_needed = need;
  if (!dst) return PFLBM_OK;
  if (reinterpret_cast<uintptr_t>(dst) % store_size(c->d.precision) != 0)
    return fail(c, PFLBM_ERR_ARG, "pflbm_pack_faces: the buffer is not aligned to the storage size");
  if (dst_bytes < need)
    return fail(c, PFLBM_ERR_ARG, "pflbm_pack_faces: the buffer holds " + std::to_string(dst_bytes) +
                                      " bytes, the two faces need " + std::to_string(need));
  if (c->d.streaming != PFLBM_STREAM_AB)
    return fail(c, PFLBM_ERR_STATE, "pflbm_pack_faces: needs the two-buffer scheme PFLBM_STREAM_AB");
  if (!c->initialised) return fail(c, PFLBM_ERR_STATE, "not initialised");
  DISPATCH(c, do_pack_faces, c, dst);
}

pflbm_status pflbm_read_populations(pflbm_ctx* c, double* h, double* g) {
  if (!c) return PFLBM_ERR_ARG;
  if (!h || !g) return fail(c, PFLBM_ERR_ARG, "output is NULL");
  if (!c->initialised) return fail(c, PFLBM_ERR_STATE, "not initialised");
  DISPATCH(c, do_read_pops, c, h, g);
}

pflbm_status pflbm_reduce(pflbm_ctx* c, double out_host[5]) {
  if (!c) return PFLBM_ERR_ARG;
  if (!out_host) return fail(c, PFLBM_ERR_ARG, "output is NULL");
  if (!c->initialised) return fail(c, PFLBM_ERR_STATE, "not initialised");
  DISPATCH(c, do_reduce, c, out_host);
}

pflbm_status pflbm_reduce_static(pflbm_ctx* c, double out_host[5]) {
  if (!c) return PFLBM_ERR_ARG;
  if (!out_host) return fail(c, PFLBM_ERR_ARG, "output is NULL");
  const size_t need = static_scratch_bytes(c->L);
  if (need > kStaticScratchBytes)
    return fail(c, PFLBM_ERR_ARG, "pflbm_reduce_static: the lattice needs " + std::to_string(need) +
                                      " bytes of partial sums, the static scratch holds " +
                                      std::to_string(kStaticScratchBytes));
  if (!c->initialised) return fail(c, PFLBM_ERR_STATE, "not initialised");
  // the device of the context is the device of its workspace
  hipPointerAttribute_t attr{};
  if (pflbm_status s = check_hip(c, hipPointerGetAttributes(&attr, c->ws), "pflbm_reduce_static workspace"))
    return s;
  char* base = nullptr;
  if (pflbm_status s = scratch_of(c, attr.device, &base)) return s;
  double* part = reinterpret_cast<double*>(base);
  double* red = reinterpret_cast<double*>(base + align_up((size_t)c->L.nblocks * 5 * sizeof(double)));
  DISPATCH(c, do_reduce_via, c, part, red, out_host);
}

size_t pflbm_state_bytes(const pflbm_ctx* c) {
  if (!c) return 0;
  return state_view(c).total;
}

pflbm_status pflbm_save_state(pflbm_ctx* c, void* dst) {
  if (!c) return PFLBM_ERR_ARG;
  if (!dst) return fail(c, PFLBM_ERR_ARG, "destination is NULL");
  if (!c->initialised) return fail(c, PFLBM_ERR_STATE, "not initialised");
  DISPATCH(c, do_save_state, c, dst);
}

pflbm_status pflbm_load_state(pflbm_ctx* c, const void* src, int64_t step_count) {
  if (!c) return PFLBM_ERR_ARG;
  if (!src || step_count < 0) return fail(c, PFLBM_ERR_ARG, "bad source or step count");
  if (c->d.has_mask && !c->mask_set) return fail(c, PFLBM_ERR_STATE, "mask not set");
  const char* o = static_cast<const char*>(src);
  const StateView v = state_view(c);
  c->pcur = 0;
  c->iprev = 1;
  hipError_t e = hipMemcpyAsync(c->ws + c->L.off_h[0], o + v.oh, c->L.bytes_h, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ws + c->L.off_g[0], o + v.og, c->L.bytes_g, hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(c->ws + c->L.off_phi[phi_cur_idx(c)], o + v.ophi, c->L.bytes_phi,
                       hipMemcpyDeviceToDevice, c->stream);
  if (e == hipSuccess && shifted(c))
    e = hipMemcpyAsync(c->ws + c->L.off_phi[c->iprev], o + v.oprev, c->L.bytes_phi, hipMemcpyDeviceToDevice,
                       c->stream);
  c->phi_ok = true;
  c->steps = step_count;
  c->initialised = e == hipSuccess;
  return check_hip(c, e, "pflbm_load_state");
}

pflbm_status pflbm_step_states(pflbm_ctx* c, void* src, void* dst, int64_t n, int32_t flags) {
  if (!c) return PFLBM_ERR_ARG;
  if (!src || !dst || src == dst || n < 0) return fail(c, PFLBM_ERR_ARG, "bad state buffers or step index");
  if (flags & ~(PFLBM_STATES_WRITE_SRC_PHI | PFLBM_STATES_SKIP_DST_PHI))
    return fail(c, PFLBM_ERR_ARG, "unknown pflbm_step_states flags");
  if (flags && is_aa(c)) return fail(c, PFLBM_ERR_ARG, "pflbm_step_states flags need PFLBM_STREAM_AB");
  if (c->d.has_mask && !c->mask_set) return fail(c, PFLBM_ERR_STATE, "mask not set");
  DISPATCH(c, do_step_states, c, src, dst, n, flags);
}

int64_t pflbm_step_count(const pflbm_ctx* c) { return c ? c->steps : -1; }

pflbm_status pflbm_sync(pflbm_ctx* c) {
  if (!c) return PFLBM_ERR_ARG;
  return check_hip(c, hipStreamSynchronize(c->stream), "pflbm_sync");
}

pflbm_status pflbm_lattice(int32_t q, int32_t* c_out, double* w_out) {
  if (q != Q_H && q != Q_G) return PFLBM_ERR_ARG;
  for (int i = 0; i < q; ++i) {
    const Dir d = q == Q_H ? ch(i) : cg(i);
    if (c_out) { c_out[3 * i] = d.x; c_out[3 * i + 1] = d.y; c_out[3 * i + 2] = d.z; }
    if (w_out) w_out[i] = q == Q_H ? wh(i) : wg(i);
  }
  return PFLBM_OK;
}

int32_t pflbm_phase_q(void) { return Q_H; }

pflbm_status pflbm_hbm_copy(const void* d_src, void* d_dst, size_t bytes, int32_t form, void* hip_stream) {
  if (!d_src || !d_dst || d_src == d_dst || bytes == 0) return PFLBM_ERR_ARG;
  const uintptr_t a = reinterpret_cast<uintptr_t>(d_src) | reinterpret_cast<uintptr_t>(d_dst);
  if ((a % 16) != 0 || (bytes % 16) != 0) return PFLBM_ERR_ARG;
  hipStream_t s = static_cast<hipStream_t>(hip_stream);
  const dim3 blk(256);
  auto grid = [](long long n, int per_block) { return dim3((unsigned)((n + per_block - 1) / per_block)); };
  switch (form) {
    case PFLBM_COPY_W4: {
      const long long n = (long long)(bytes / 4);
      if ((n + 2047) / 2048 >= (1ll << 31)) return PFLBM_ERR_ARG;
      hipLaunchKernelGGL((k_copy_lines<unsigned, 8, true>), grid(n, 2048), blk, 0, s,
                         static_cast<const unsigned*>(d_src), static_cast<unsigned*>(d_dst), n);
      break;
    }
    case PFLBM_COPY_W16: {
      const long long n = (long long)(bytes / 16);
      if ((n + 1023) / 1024 >= (1ll << 31)) return PFLBM_ERR_ARG;
      hipLaunchKernelGGL((k_copy_lines<u32x4, 4, true>), grid(n, 1024), blk, 0, s,
                         static_cast<const u32x4*>(d_src), static_cast<u32x4*>(d_dst), n);
      break;
    }
    case PFLBM_COPY_W16_CACHED: {
      const long long n = (long long)(bytes / 16);
      if ((n + 1023) / 1024 >= (1ll << 31)) return PFLBM_ERR_ARG;
      hipLaunchKernelGGL((k_copy_lines<u32x4, 4, false>), grid(n, 1024), blk, 0, s,
                         static_cast<const u32x4*>(d_src), static_cast<u32x4*>(d_dst), n);
      break;
    }
    case PFLBM_COPY_SOA43:
    case PFLBM_COPY_SOA43_NT: {
      // 43 rows of N floats on each side
      if (bytes % (43 * 4) != 0) return PFLBM_ERR_ARG;
      const long long N = (long long)(bytes / (43 * 4));
      if ((N + 255) / 256 >= (1ll << 31)) return PFLBM_ERR_ARG;
      if (form == PFLBM_COPY_SOA43)
        hipLaunchKernelGGL((k_copy_soa<42, false>), grid(N, 256), blk, 0, s, static_cast<const float*>(d_src),
                           static_cast<float*>(d_dst), N);
      else
        hipLaunchKernelGGL((k_copy_soa<42, true>), grid(N, 256), blk, 0, s, static_cast<const float*>(d_src),
                           static_cast<float*>(d_dst), N);
      break;
    }
    case PFLBM_COPY_SOA43_F64:
    case PFLBM_COPY_SOA43_F64_NT: {
      // 43 rows of N doubles on each side
      if (bytes % (43 * 8) != 0) return PFLBM_ERR_ARG;
      const long long N = (long long)(bytes / (43 * 8));
      if ((N + 255) / 256 >= (1ll << 31)) return PFLBM_ERR_ARG;
      if (form == PFLBM_COPY_SOA43_F64)
        hipLaunchKernelGGL((k_copy_soa<42, false, double>), grid(N, 256), blk, 0, s,
                           static_cast<const double*>(d_src), static_cast<double*>(d_dst), N);
      else
        hipLaunchKernelGGL((k_copy_soa<42, true, double>), grid(N, 256), blk, 0, s,
                           static_cast<const double*>(d_src), static_cast<double*>(d_dst), N);
      break;
    }
    default:
      return PFLBM_ERR_ARG;
  }
  return hipGetLastError() == hipSuccess ? PFLBM_OK : PFLBM_ERR_HIP;
}

const char* pflbm_status_string(pflbm_status s) {
  switch (s) {
    case PFLBM_OK: return "ok";
    case PFLBM_ERR_ARG: return "invalid argument";
    case PFLBM_ERR_STATE: return "invalid state";
    case PFLBM_ERR_HIP: return "HIP error";
    case PFLBM_ERR_UNSTABLE: return "unstable (non-finite reduction)";
    case PFLBM_ERR_UNSUPPORTED: return "unsupported";
  }
  return "unknown status";
}

const char* pflbm_last_error(const pflbm_ctx* c) { return c ? c->err.c_str() : "no context"; }

}  // extern "C"

#include "adjoint_api.inc"
