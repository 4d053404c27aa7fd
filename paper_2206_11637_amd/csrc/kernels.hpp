// Forward kernels of the coupled phase-field LBM step on gfx950.
//
// Data layout in HBM (all structure-of-arrays, x fastest):
//   h[i * N + idx], i < 15       phase-field populations (storage type S),
//   g[i * N + idx], i < 27       hydrodynamic populations; two state buffers
//                                of each (the step reads one, writes the other)
//   phi[2][N]                    phase field (compute type R)
//   mask[N], nbr[N]              optional solids (1 = solid) and, per cell, the
//                                bit set of its solid neighbours (bit 0: the
//                                cell itself is solid)
//
// Streaming (paper: streaming eq., bounce-back walls) comes in two schemes.
//
// Two buffers, pull form (the default, fastest).  Slot (i, x) of a state
// buffer holds the post-collision value f*_i(x) of the step that wrote it
// (the initialisation writes the equivalent values).  The pre-collision
// population i of cell y is
//     slot(i, y - c_i)   if y - c_i is fluid,
//     slot(opp i, y)     otherwise (halfway bounce-back),
// so every fluid slot is read exactly once per step, and a step writes only
// its own cells' slots of the other buffer (aligned, coalesced stores).
// The fused step kernel k_step gives each block a bx * by tile and a chunk of
// z planes and marches up the chunk.  The phase field phi^n = sum_i h_i is
// never read from HBM: for each plane the block pulls the h populations of
// its cells and of a one-cell ring around the tile and sums them into a
// 4-plane LDS ring (sentinel for walls and solids); its own cells' pulled h
// wait in thread-private LDS slots for the collision one plane later.  The
// grad/lap stencils read three ring planes.  Pulling the ring cells' h re-reads data that the
// neighbouring tiles read too (mostly from L2).  This needs the second
// buffer: in place, a neighbouring block could overwrite a ring cell's
// populations before they are summed.  The FP32 form runs k_step_dma, the
// same step with the h pulls of plane z + 2 sent straight into LDS while
// plane z collides.
//
// In-place AA pattern (one buffer per lattice, half the population memory):
//   even step: read own slots f[i][x], write f*_i into own slot f[opp i][x];
//   odd step:  read f_i(x) from f[opp i][x - c_i] (or f[i][x] when x - c_i is
//              a wall/solid: the value bounced back there), write f*_i into
//              f[i][x + c_i] (or f[opp i][x] when x + c_i is a wall/solid).
// Every slot is read and written by exactly one cell per step, so the update
// is race-free in place; after an odd step the buffer holds the natural
// layout f[i][x] = f_i(x).  k_cell_aa does one plane of one tile per block
// with phi^n staged from the stored field (tile + halo, 3 planes, in LDS),
// and a light pass (k_light, gather) then forms phi^{n+1}.
//
// Shifted storage (FP32 and FP16 forms): a slot holds h_i - w_i phi^n(r),
// where r is the cell that reads it in the next step (x + c_i, or x itself
// behind a wall; the writer knows phi^n(r) from its stencil planes), so the
// reader finds its reference at its own index of the previous phi buffer and
// works on deviations from w_i phi^{n-1}(self) without adding anything (see
// phi_of in cell.hpp).  Values of the size of the per-step change are stored
// and rounded instead of h ~ w_i; with plain FP32 storage the heavy phase
// loses updates below its rounding unit while the light phase keeps them,
// which made the FP32 phase mass drift by ~5e-9 per step in slow runs.  g is
// stored unshifted (small in the p* gauge), and so is everything in FP64.
//
// Blocks are issued round-robin over the 8 XCDs; xcd_remap() renumbers them
// so that each XCD walks one contiguous range of tiles, keeping the ring and
// neighbour-population reuse inside one XCD's L2.
#pragma once
#include <hip/hip_runtime.h>

#include "cell.hpp"
#include "lattice.hpp"

namespace pflbm {

struct Geom {
  int nx, ny, nz;
  int px, py, pz;         // periodic flags
  int bx, by;             // tile shape (bx * by == 256)
  int tiles_x, tiles_y;
  unsigned nblocks;       // tiles_x * tiles_y * nz (one plane per block)
  int zc, nchunks;        // z-chunk length and count of the marching step kernel
  unsigned nblocks_step;  // tiles_x * tiles_y * nchunks
  long long N;
};

// ---- storage codecs -------------------------------------------------------
// ld/st convert between the stored value and the compute type; FP16 storage
// also scales by 2^k (stored = value * 2^k).  kShift: h is stored shifted
// (see the header).
template <typename S>
struct Store;
template <bool NT, typename T>
__device__ __forceinline__ T ld_nt(const T* p) {
  if constexpr (NT) return __builtin_nontemporal_load(p); else return *p;
}
template <bool NT, typename T>
__device__ __forceinline__ void st_nt(T* p, T v) {
  if constexpr (NT) __builtin_nontemporal_store(v, p); else *p = v;
}
template <>
struct Store<double> {
  using R = double;
  static constexpr bool kShift = false;
  template <bool NT = true>
  __device__ static R ld(const double* p, R) { return ld_nt<NT>(p); }
  template <bool NT = true>
  __device__ static void st(double* p, R v, R) { st_nt<NT>(p, v); }
};
template <>
struct Store<float> {
  using R = float;
  static constexpr bool kShift = true;
  template <bool NT = true>
  __device__ static R ld(const float* p, R) { return ld_nt<NT>(p); }
  template <bool NT = true>
  __device__ static void st(float* p, R v, R) { st_nt<NT>(p, v); }
};
template <>
struct Store<_Float16> {
  using R = float;
  static constexpr bool kShift = true;
  template <bool NT = true>
  __device__ static R ld(const _Float16* p, R inv_scale) {
    return static_cast<float>(ld_nt<NT>(p)) * inv_scale;
  }
  template <bool NT = true>
  __device__ static void st(_Float16* p, R v, R scale) {
    st_nt<NT>(p, static_cast<_Float16>(v * scale));
  }
};

// Cache policy of the population streams: pulls read rows one element off
// alignment whose lines neighbouring waves and the ring share (cached loads);
// the step's stores are written once and read only in the next step
// (non-temporal).  Measured on the rising-bubble lattice (FP32): all pulls
// non-temporal -12 %, only the g pulls non-temporal -4 %.
#ifndef PFLBM_NT_PULL
#define PFLBM_NT_PULL 0
#endif
#ifndef PFLBM_NT_STORE
#define PFLBM_NT_STORE 1
#endif
#ifndef PFLBM_NT_GPULL
#define PFLBM_NT_GPULL PFLBM_NT_PULL
#endif
constexpr bool kNtPull = PFLBM_NT_PULL;
constexpr bool kNtGPull = PFLBM_NT_GPULL;
constexpr bool kNtStore = PFLBM_NT_STORE;

template <typename R>
struct Codec {
  R scale_h, inv_scale_h, scale_g, inv_scale_g;
};

template <typename R>
__device__ __forceinline__ R sentinel() { return R(-1e30); }

__device__ __forceinline__ unsigned xcd_remap(unsigned b, unsigned nb) {
  const unsigned q = nb >> 3, r = nb & 7u, x = b & 7u, k = b >> 3;
  return (x < r) ? x * (q + 1) + k : r * (q + 1) + (x - r) * q + k;
}

struct TileCoord { int x0, y0, z; };

__device__ __forceinline__ TileCoord tile_of_block(const Geom& G) {
  const unsigned L = xcd_remap(blockIdx.x, G.nblocks);
  const unsigned tx = L % G.tiles_x;
  const unsigned rest = L / G.tiles_x;
  const unsigned ty = rest % G.tiles_y;
  return TileCoord{int(tx) * G.bx, int(ty) * G.by, int(rest / G.tiles_y)};
}

struct ChunkCoord { int x0, y0, z0, z1; };

__device__ __forceinline__ ChunkCoord chunk_of_block(const Geom& G) {
  const unsigned L = xcd_remap(blockIdx.x, G.nblocks_step);
  const unsigned tx = L % G.tiles_x;
  const unsigned rest = L / G.tiles_x;
  const unsigned ty = rest % G.tiles_y;
  const int z0 = int(rest / G.tiles_y) * G.zc;
  return ChunkCoord{int(tx) * G.bx, int(ty) * G.by, z0, min(z0 + G.zc, G.nz)};
}

// Coordinate one step outside [0, n): wrapped on a periodic axis, else a
// wall (false).  Positions further out (a ragged tile's padding) are never a
// neighbour of a cell and report false as well.
__device__ __forceinline__ bool wrap(int& v, int n, int periodic) {
  if (v == -1) { if (!periodic) return false; v = n - 1; }
  else if (v == n) { if (!periodic) return false; v = 0; }
  else if (v < -1 || v > n) return false;
  return true;
}

// ---- wall bits -------------------------------------------------------------
// Bit k set: the neighbour in direction kC27[k] is outside a wall or solid.
struct AxisMasks { unsigned xm, xp, ym, yp, zm, zp; };
constexpr AxisMasks make_axis_masks() {
  AxisMasks m{0u, 0u, 0u, 0u, 0u, 0u};
  for (int k = 1; k < 27; ++k) {
    if (kC27[k].x < 0) m.xm |= 1u << k;
    if (kC27[k].x > 0) m.xp |= 1u << k;
    if (kC27[k].y < 0) m.ym |= 1u << k;
    if (kC27[k].y > 0) m.yp |= 1u << k;
    if (kC27[k].z < 0) m.zm |= 1u << k;
    if (kC27[k].z > 0) m.zp |= 1u << k;
  }
  return m;
}
constexpr AxisMasks kAxis = make_axis_masks();

// the box faces that are walls, from the coordinates alone
__device__ __forceinline__ unsigned box_walls(int x, int y, int z, const Geom& G) {
  unsigned b = 0;
  if (!G.px) { b |= (x == 0) ? kAxis.xm : 0u; b |= (x == G.nx - 1) ? kAxis.xp : 0u; }
  if (!G.py) { b |= (y == 0) ? kAxis.ym : 0u; b |= (y == G.ny - 1) ? kAxis.yp : 0u; }
  if (!G.pz) { b |= (z == 0) ? kAxis.zm : 0u; b |= (z == G.nz - 1) ? kAxis.zp : 0u; }
  return b;
}

// Box walls plus solid neighbours; `solid` reports the cell itself.
template <bool MASK>
__device__ __forceinline__ unsigned cell_walls(int x, int y, int z, unsigned idx, const Geom& G,
                                               const unsigned* __restrict__ nbr, bool& solid) {
  unsigned b = box_walls(x, y, z, G);
  solid = false;
  if (MASK) {
    const unsigned m = nbr[idx];
    solid = m & 1u;
    b |= m & ~1u;
  }
  return b;
}

// Stage phi of the tile + halo (3 planes) into LDS; sentinel for walls/solids.
template <typename R, bool MASK>
__device__ __forceinline__ void load_phi_tile(R* tile, const R* __restrict__ phi,
                                              const unsigned char* __restrict__ mask,
                                              const Geom& G, TileCoord t) {
  const int TX = G.bx + 2, TY = G.by + 2, total = TX * TY * 3;
  const int tid = threadIdx.x + threadIdx.y * G.bx;
  for (int e = tid; e < total; e += 256) {
    const int ix = e % TX, r = e / TX, iy = r % TY, iz = r / TY;
    int X = t.x0 - 1 + ix, Y = t.y0 - 1 + iy, Z = t.z - 1 + iz;
    R v = sentinel<R>();
    if (wrap(X, G.nx, G.px) && wrap(Y, G.ny, G.py) && wrap(Z, G.nz, G.pz)) {
      const long long id = X + (long long)G.nx * (Y + (long long)G.ny * Z);
      if (!MASK || !mask[id]) v = phi[id];
    }
    tile[e] = v;
  }
}

// Linear indices of the 3x3x3 neighbourhood (periodic wrap; out-of-box
// entries are never dereferenced because the wall bits mark them).
// 32-bit: the library limits N * sizeof(storage) below 2^32.
struct Nbhd {
  unsigned xs[3], ys[3], zs[3];
  __device__ __forceinline__ unsigned at(int dx, int dy, int dz) const {
    return xs[dx + 1] + ys[dy + 1] + zs[dz + 1];
  }
};

__device__ __forceinline__ Nbhd make_nbhd(int x, int y, int z, const Geom& G) {
  Nbhd n;
  n.xs[0] = x == 0 ? G.nx - 1 : x - 1;
  n.xs[1] = x;
  n.xs[2] = x == G.nx - 1 ? 0 : x + 1;
  const unsigned sy = G.nx, sz = (unsigned)G.nx * (unsigned)G.ny;
  n.ys[0] = (y == 0 ? G.ny - 1 : y - 1) * sy;
  n.ys[1] = y * sy;
  n.ys[2] = (y == G.ny - 1 ? 0 : y + 1) * sy;
  n.zs[0] = (z == 0 ? G.nz - 1 : z - 1) * sz;
  n.zs[1] = z * sz;
  n.zs[2] = (z == G.nz - 1 ? 0 : z + 1) * sz;
  return n;
}

// Address of population `pop` of cell `cell`: a wave-uniform base (scalar
// registers) plus a 32-bit per-lane byte offset, which maps onto the
// saddr + voffset form of global loads and stores.
template <typename S>
__device__ __forceinline__ S* slot(S* base, long long N, int pop, unsigned cell) {
  char* b = reinterpret_cast<char*>(base + (long long)pop * N);
  return reinterpret_cast<S*>(b + (unsigned)(cell * (unsigned)sizeof(S)));
}
template <typename S>
__device__ __forceinline__ const S* slot(const S* base, long long N, int pop, unsigned cell) {
  const char* b = reinterpret_cast<const char*>(base + (long long)pop * N);
  return reinterpret_cast<const S*>(b + (unsigned)(cell * (unsigned)sizeof(S)));
}

// Wall bits of a cell from an LDS tile of 3 planes (sentinel = wall/solid).
template <typename R>
__device__ __forceinline__ unsigned wall_bits(const R* tile, int TX, int TY, int lx, int ly) {
  unsigned b = 0;
#pragma unroll
  for (int k = 1; k < 27; ++k) {
    const Dir d = cg(k);
    const R v = tile[((1 + d.z) * TY + (ly + 1 + d.y)) * TX + (lx + 1 + d.x)];
    if (v == sentinel<R>()) b |= 1u << k;
  }
  return b;
}

// grad phi and lap phi from three LDS planes (below, own, above), over the
// D3Q27 stencil grad = 3 sum_k w_k c_k phi_k, lap = 6 sum_k w_k (phi_k - phi).
// Its weights factor as w_abc = v_a v_b v_c (v_0 = 2/3, v_-1 = v_+1 = 1/6;
// a, b, c the x, y, z offsets), so both are products of one-dimensional sums:
//   A_ab = sum_c v_c phi_abc,   B_ab = phi_ab+ - phi_ab-,
//   S_a = sum_b v_b A_ab,       Y_a = A_a+ - A_a-,       Z_a = sum_b v_b B_ab,
//   grad = 3 v_1 (S_+ - S_-,  sum_a v_a Y_a,  sum_a v_a Z_a),
//   lap = 6 (sum_a v_a S_a - phi),
// 27 loads and ~60 operations instead of a weighted sum over 26 neighbours.
// A missing neighbour (wall or solid: the sentinel) takes phi of the cell
// itself (no-flux rule).  XWALLS: the caller knows that the only neighbours
// that can be missing are whole x columns of a box wall (xm: the column at
// x - 1, xp: at x + 1), so only those are replaced; both forms give the same
// bits where both apply.
// a * b + c rounded once (explicit, so that every copy of an expression that
// must give the same bits does, whatever the compiler's contraction choices)
__device__ __forceinline__ float fmad(float a, float b, float c) { return __builtin_fmaf(a, b, c); }
__device__ __forceinline__ double fmad(double a, double b, double c) { return __builtin_fma(a, b, c); }

template <typename R, bool XWALLS>
__device__ __forceinline__ void stencil_sep(const R* pm, const R* p0, const R* pp, int TX, int lx,
                                            int ly, bool xm, bool xp, R& Gx, R& Gy, R& Gz, R& lap) {
  const R c0 = p0[(ly + 1) * TX + lx + 1];
  const R v0 = R(2) / R(3), v1 = R(1) / R(6);
  R S[3], Y[3], Z[3];
#pragma unroll
  for (int a = -1; a <= 1; ++a) {
    R A[3], B[3];
#pragma unroll
    for (int b = -1; b <= 1; ++b) {
      const int o = (ly + 1 + b) * TX + (lx + 1 + a);
      R fm = pm[o], f0 = p0[o], fp = pp[o];
      if (XWALLS) {
        if (a != 0) {
          const bool miss = a < 0 ? xm : xp;
          fm = miss ? c0 : fm;
          f0 = miss ? c0 : f0;
          fp = miss ? c0 : fp;
        }
      } else {
        fm = fm == sentinel<R>() ? c0 : fm;
        fp = fp == sentinel<R>() ? c0 : fp;
        if (a != 0 || b != 0) f0 = f0 == sentinel<R>() ? c0 : f0;
      }
      A[b + 1] = fmad(v0, f0, v1 * (fm + fp));
      B[b + 1] = fp - fm;
    }
    S[a + 1] = fmad(v0, A[1], v1 * (A[0] + A[2]));
    Y[a + 1] = A[2] - A[0];
    Z[a + 1] = fmad(v0, B[1], v1 * (B[0] + B[2]));
  }
  Gx = R(0.5) * (S[2] - S[0]);
  Gy = R(0.5) * fmad(v0, Y[1], v1 * (Y[0] + Y[2]));
  Gz = R(0.5) * fmad(v0, Z[1], v1 * (Z[0] + Z[2]));
  lap = R(6) * (fmad(v0, S[1], v1 * (S[0] + S[2])) - c0);
}

template <typename R>
__device__ __forceinline__ void stencil3(const R* pm, const R* p0, const R* pp, int TX, int lx,
                                         int ly, R& Gx, R& Gy, R& Gz, R& lap) {
  stencil_sep<R, false>(pm, p0, pp, TX, lx, ly, false, false, Gx, Gy, Gz, lap);
}

// the same from a contiguous 3-plane tile
template <typename R>
__device__ __forceinline__ void stencil(const R* tile, int TX, int TY, int lx, int ly, R& Gx,
                                        R& Gy, R& Gz, R& lap) {
  stencil3(tile, tile + TX * TY, tile + 2 * TX * TY, TX, lx, ly, Gx, Gy, Gz, lap);
}

// ---- population access (pull form) -----------------------------------------
// An opposite pair (i, i+1), i odd, is addressed from the pair's first
// population (a wave-uniform base); the per-lane part is one 32-bit byte
// offset, cell * sizeof(S) plus N * sizeof(S) for the pair's second member.
// The pull picks between the neighbour's slot and the cell's own
// (bounce-back) slot with a single select on that offset.
__device__ __forceinline__ constexpr int pair_first(int i) { return i == 0 ? 0 : ((i & 1) ? i : i - 1); }
__device__ __forceinline__ constexpr bool pair_second(int i) { return i != 0 && !(i & 1); }

template <typename S>
__device__ __forceinline__ const char* pair_base(const S* base, long long N, int i) {
  return reinterpret_cast<const char*>(base + (long long)pair_first(i) * N);
}
template <typename S>
__device__ __forceinline__ char* pair_base(S* base, long long N, int i) {
  return reinterpret_cast<char*>(base + (long long)pair_first(i) * N);
}

// byte offset of population i of the cell at element index `cell`, relative to
// its pair base
template <typename S>
__device__ __forceinline__ unsigned pair_off(int i, unsigned cell, unsigned NS) {
  return cell * (unsigned)sizeof(S) + (pair_second(i) ? NS : 0u);
}

// offset of the slot that population i of cell idx is pulled from
template <typename S, bool G27>
__device__ __forceinline__ unsigned pull_off(int i, unsigned idx, const Nbhd& nb, unsigned walls,
                                             unsigned NS) {
  if (i == 0) return pair_off<S>(0, idx, NS);
  const Dir d = cdir<G27>(i);
  return (walls & (1u << nb27(-d.x, -d.y, -d.z))) ? pair_off<S>(opp(i), idx, NS)
                                                   : pair_off<S>(i, nb.at(-d.x, -d.y, -d.z), NS);
}

// The step kernel takes the x-wall form below for fast waves in FP64 only.
// Measured on the rising-bubble lattice, all builds on one GPU: FP64 step
// -1.3 % (1.183 -> 1.168 ms); FP32 unchanged (0.633 ms); FP16 storage +7 %
// (0.434 -> 0.466 ms: the duplicated pull code, although it issued 9 % fewer
// vector instructions).
template <typename S>
struct FastWaves { static constexpr bool value = sizeof(S) == 8; };

// Wall situation of one wave in one plane.  fast: no lane of the wave has a
// box wall in y or z or a solid among its neighbours, so the only neighbours
// that can be missing are whole x columns behind a box wall in x, marked per
// lane by xm (x = 0) and xp (x = nx - 1).  fast is wave-uniform, so a fast
// wave takes cheaper pulls, stencil and shift reference with the same results.
struct XWalls {
  bool fast, xm, xp;
};

template <bool MASK>
__device__ __forceinline__ XWalls x_walls(bool on, int x, int y, int z, unsigned nbits,
                                          const Geom& G) {
  const bool yz = (!G.py && (y == 0 || y == G.ny - 1)) || (!G.pz && (z == 0 || z == G.nz - 1));
  const bool sol = MASK && (nbits & ~1u) != 0u;
  XWalls w;
  w.fast = __ballot(on && (yz || sol)) == 0ull;
  w.xm = !G.px && x == 0;
  w.xp = !G.px && x == G.nx - 1;
  return w;
}

// pull offset where only box walls in x can hide the source cell x - c_i
template <typename S, bool G27>
__device__ __forceinline__ unsigned pull_off_x(int i, unsigned idx, const Nbhd& nb, bool xm, bool xp,
                                               unsigned NS) {
  if (i == 0) return pair_off<S>(0, idx, NS);
  const Dir d = cdir<G27>(i);
  const unsigned from_nb = pair_off<S>(i, nb.at(-d.x, -d.y, -d.z), NS);
  if (d.x == 0) return from_nb;
  return (d.x > 0 ? xm : xp) ? pair_off<S>(opp(i), idx, NS) : from_nb;
}

template <typename S, bool NT>
__device__ __forceinline__ void load_h_x(const S* __restrict__ H, long long N, unsigned idx,
                                         const Nbhd& nb, bool xm, bool xp,
                                         typename Store<S>::R inv_scale,
                                         typename Store<S>::R (&h)[Q_H]) {
  const unsigned NS = (unsigned)(N * (long long)sizeof(S));
#pragma unroll
  for (int i = 0; i < Q_H; ++i) {
    const S* p = reinterpret_cast<const S*>(pair_base(H, N, i) + pull_off_x<S, false>(i, idx, nb, xm, xp, NS));
    h[i] = Store<S>::template ld<NT>(p, inv_scale);
  }
}

template <typename S, bool NT>
__device__ __forceinline__ void load_g_x(const S* __restrict__ Gp, long long N, unsigned idx,
                                         const Nbhd& nb, bool xm, bool xp,
                                         typename Store<S>::R inv_scale,
                                         typename Store<S>::R (&g)[Q_G]) {
  const unsigned NS = (unsigned)(N * (long long)sizeof(S));
#pragma unroll
  for (int i = 0; i < Q_G; ++i) {
    const S* p = reinterpret_cast<const S*>(pair_base(Gp, N, i) + pull_off_x<S, true>(i, idx, nb, xm, xp, NS));
    g[i] = Store<S>::template ld<NT>(p, inv_scale);
  }
}

// ---- read rules of a state ---------------------------------------------------
// RULE_AB: two-buffer pull; RULE_AA_EVEN / RULE_AA_ODD: the AA parity of the
// next step (a state after n steps is read with the rule of parity n).
enum Rule { RULE_AB = 0, RULE_AA_EVEN = 1, RULE_AA_ODD = 2 };

// offset of the slot population i of cell idx is read from (pair base relative)
template <typename S, bool G27, int RULE>
__device__ __forceinline__ unsigned read_off(int i, unsigned idx, const Nbhd& nb, unsigned walls,
                                             unsigned NS) {
  if (RULE == RULE_AB) return pull_off<S, G27>(i, idx, nb, walls, NS);
  if (RULE == RULE_AA_EVEN || i == 0) return pair_off<S>(i, idx, NS);
  const Dir d = cdir<G27>(i);
  return (walls & (1u << nb27(-d.x, -d.y, -d.z))) ? pair_off<S>(i, idx, NS)
                                                   : pair_off<S>(opp(i), nb.at(-d.x, -d.y, -d.z), NS);
}

// Pre-collision h of one cell as read (deviations from w_i phi^{n-1}(self)
// for the shifted forms, plain values in FP64).
template <typename S, int RULE, bool NT>
__device__ __forceinline__ void load_h(const S* __restrict__ H, long long N, unsigned idx,
                                       const Nbhd& nb, unsigned walls,
                                       typename Store<S>::R inv_scale,
                                       typename Store<S>::R (&h)[Q_H]) {
  using St = Store<S>;
  const unsigned NS = (unsigned)(N * (long long)sizeof(S));
#pragma unroll
  for (int i = 0; i < Q_H; ++i) {
    const S* p = reinterpret_cast<const S*>(pair_base(H, N, i) + read_off<S, false, RULE>(i, idx, nb, walls, NS));
    h[i] = St::template ld<NT>(p, inv_scale);
  }
}

template <typename S, int RULE, bool NT>
__device__ __forceinline__ void load_g(const S* __restrict__ Gp, long long N, unsigned idx,
                                       const Nbhd& nb, unsigned walls,
                                       typename Store<S>::R inv_scale,
                                       typename Store<S>::R (&g)[Q_G]) {
  using St = Store<S>;
  const unsigned NS = (unsigned)(N * (long long)sizeof(S));
#pragma unroll
  for (int i = 0; i < Q_G; ++i) {
    const S* p = reinterpret_cast<const S*>(pair_base(Gp, N, i) + read_off<S, true, RULE>(i, idx, nb, walls, NS));
    g[i] = St::template ld<NT>(p, inv_scale);
  }
}

// The same pulls of g with the stored values kept as they are, each in a
// register of its own (an FP16 value zero-extended, so no load writes half a
// register), and decoded where they are used, so that the loads stay in
// flight until then.
template <typename S> struct Raw { using T = S; };
template <> struct Raw<_Float16> { using T = unsigned; };
template <typename S, int RULE, bool NT>
__device__ __forceinline__ void load_g_raw(const S* __restrict__ Gp, long long N, unsigned idx,
                                           const Nbhd& nb, unsigned walls,
                                           typename Raw<S>::T (&g)[Q_G]) {
  const unsigned NS = (unsigned)(N * (long long)sizeof(S));
#pragma unroll
  for (int i = 0; i < Q_G; ++i) {
    const char* p = pair_base(Gp, N, i) + read_off<S, true, RULE>(i, idx, nb, walls, NS);
    if constexpr (sizeof(S) == 2) g[i] = ld_nt<NT>(reinterpret_cast<const unsigned short*>(p));
    else g[i] = ld_nt<NT>(reinterpret_cast<const S*>(p));
  }
}
template <typename S>
__device__ __forceinline__ typename Store<S>::R decode_raw(typename Raw<S>::T v,
                                                          typename Store<S>::R inv_scale) {
  if constexpr (sizeof(S) == 2)
    return static_cast<float>(__builtin_bit_cast(_Float16, static_cast<unsigned short>(v))) * inv_scale;
  else return v;
}

// phi^{n-1}(self), the reference of the shifted forms (0 in FP64)
template <typename S>
__device__ __forceinline__ typename Store<S>::R phi_ref_of(const typename Store<S>::R* __restrict__ phi_prev,
                                                          unsigned idx) {
  using R = typename Store<S>::R;
  return Store<S>::kShift ? phi_prev[idx] : R(0);
}

// Stencil planes of one cell (below, own, above) in LDS: phi^n of the cell
// and of its neighbours, the sentinel marking walls and solids.
template <typename R>
struct Planes {
  const R* pm;
  const R* p0;
  const R* pp;
  int TX, lx, ly;
  // phi^n of the reader of outgoing population i (x + c_i, or x behind a wall)
  __device__ __forceinline__ R reader(int i, R self) const {
    if (i == 0) return self;
    const Dir d = ch(i);
    const R* pl = d.z < 0 ? pm : (d.z > 0 ? pp : p0);
    const R v = pl[(ly + 1 + d.y) * TX + (lx + 1 + d.x)];
    return v == sentinel<R>() ? self : v;
  }
};

// Post-collision value of population i for storage: the deviation h*'_i is
// relative to w_i phi_ref; the slot must be relative to w_i phi^n(reader).
// (Read from LDS per population, so no array of reader values stays live.)
template <typename S>
__device__ __forceinline__ typename Store<S>::R rebase(int i, typename Store<S>::R v,
                                                       typename Store<S>::R phi_ref,
                                                       typename Store<S>::R self,
                                                       const Planes<typename Store<S>::R>& pl) {
  using R = typename Store<S>::R;
  return Store<S>::kShift ? v + R(wh(i)) * (phi_ref - pl.reader(i, self)) : v;
}

// p + n for a per-lane global-memory address, which the compiler must take as
// a new value: the stores of one cell then walk its populations with one
// 64-bit add each, instead of keeping 41 population offsets (i * N) live in
// scalar registers, which spill into vector registers and cost two lane reads
// per store.  Measured on the rising-bubble lattice: FP32 step -1.7 %, FP64
// -0.3 %, FP16 storage +3.6 % (it then re-reads the stencil planes from LDS
// for the shift of each h), so the FP16 form keeps the per-population bases.
template <typename T>
__device__ __forceinline__ T* next_row(T* p, long long n) {
  using GT = __attribute__((address_space(1))) T;
  GT* g = (GT*)(p + n);
  asm volatile("" : "+v"(g));
  return (T*)g;
}

// Two buffers: post-collision values into the cell's own slots.
template <typename S, bool NT>
__device__ __forceinline__ void store_own(S* __restrict__ H, S* __restrict__ Gp, long long N,
                                          unsigned idx, const Codec<typename Store<S>::R>& cd,
                                          typename Store<S>::R phi_ref, typename Store<S>::R self,
                                          const Planes<typename Store<S>::R>& pl,
                                          const typename Store<S>::R (&h)[Q_H],
                                          const typename Store<S>::R (&g)[Q_G]) {
  using St = Store<S>;
  if constexpr (sizeof(S) == 2) {
#pragma unroll
    for (int i = 0; i < Q_H; ++i)
      St::template st<NT>(slot(H, N, i, idx), rebase<S>(i, h[i], phi_ref, self, pl), cd.scale_h);
#pragma unroll
    for (int i = 0; i < Q_G; ++i) St::template st<NT>(slot(Gp, N, i, idx), g[i], cd.scale_g);
  } else {
    S* p = next_row(H, (long long)idx);
#pragma unroll
    for (int i = 0; i < Q_H; ++i) {
      St::template st<NT>(p, rebase<S>(i, h[i], phi_ref, self, pl), cd.scale_h);
      if (i + 1 < Q_H) p = next_row(p, N);
    }
    p = next_row(Gp, (long long)idx);
#pragma unroll
    for (int i = 0; i < Q_G; ++i) {
      St::template st<NT>(p, g[i], cd.scale_g);
      if (i + 1 < Q_G) p = next_row(p, N);
    }
  }
}

// AA: post-collision values into the slots of the parity's write rule.
template <typename S, bool ODD, bool NT>
__device__ __forceinline__ void store_aa(S* __restrict__ H, S* __restrict__ Gp, long long N,
                                         unsigned idx, const Nbhd& nb, unsigned walls,
                                         const Codec<typename Store<S>::R>& cd,
                                         typename Store<S>::R phi_ref, typename Store<S>::R self,
                                         const Planes<typename Store<S>::R>& pl,
                                         const typename Store<S>::R (&h)[Q_H],
                                         const typename Store<S>::R (&g)[Q_G]) {
  using St = Store<S>;
  const unsigned NS = (unsigned)(N * (long long)sizeof(S));
#pragma unroll
  for (int i = 0; i < Q_H; ++i) {
    unsigned off = pair_off<S>(opp(i), idx, NS);
    if (ODD && i) {
      const Dir d = ch(i);
      if (!(walls & (1u << nb27(d.x, d.y, d.z)))) off = pair_off<S>(i, nb.at(d.x, d.y, d.z), NS);
    }
    S* p = reinterpret_cast<S*>(pair_base(H, N, i) + off);
    St::template st<NT>(p, rebase<S>(i, h[i], phi_ref, self, pl), cd.scale_h);
  }
#pragma unroll
  for (int i = 0; i < Q_G; ++i) {
    unsigned off = pair_off<S>(opp(i), idx, NS);
    if (ODD && i) {
      const Dir d = cg(i);
      if (!(walls & (1u << nb27(d.x, d.y, d.z)))) off = pair_off<S>(i, nb.at(d.x, d.y, d.z), NS);
    }
    S* p = reinterpret_cast<S*>(pair_base(Gp, N, i) + off);
    St::template st<NT>(p, g[i], cd.scale_g);
  }
}

// Occupancy request of the step kernels: 3 waves per SIMD (<= 168 VGPRs)
// for the FP32-arithmetic forms; the FP64 form keeps the compiler's choice.
#ifndef PFLBM_F64_WAVES
#define PFLBM_F64_WAVES 1
#endif
#ifndef PFLBM_F32_WAVES
#define PFLBM_F32_WAVES 3
#endif
template <typename S>
struct StepWaves { static constexpr int value = sizeof(S) == 8 ? PFLBM_F64_WAVES : PFLBM_F32_WAVES; };

template <typename S>
struct StepArgs {
  using R = typename Store<S>::R;
  const S* h_in;             // state n
  const S* g_in;
  S* h_out;                  // state n + 1
  S* g_out;
  const R* phi_prev;         // phi^{n-1}: shift reference of state n (shifted forms)
  R* phi_out;                // phi^n, the reference of state n + 1 (shifted forms)
  R* phi_src_out;            // phi^n into the read state's phi slot (may be null)
  const unsigned* nbr;       // solid-neighbour bits (mask only)
  Geom geo;
  Phys<R> P;
  Codec<R> cd;
};

// Fused step n -> n+1: pull, phi^n and its stencils, collide both lattices,
// store.  One barrier per plane; the 4-plane ring lets plane z+1 be written
// while plane z-1 is still being read.
template <typename S, bool MRT, bool MASK, bool GUO>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(StepWaves<S>::value)))
void k_step(StepArgs<S> a) {
  using St = Store<S>;
  using R = typename St::R;
  extern __shared__ unsigned char smem_raw[];
  const Geom& G = a.geo;
  const int TX = G.bx + 2, TY = G.by + 2, TXY = TX * TY;
  R* ring = reinterpret_cast<R*>(smem_raw);     // [4][TY][TX]
  R* hbuf = ring + 4 * TXY;                     // [2][15][256], thread-private slots
  const ChunkCoord t = chunk_of_block(G);
  const int lx = threadIdx.x, ly = threadIdx.y, tid = lx + ly * G.bx;
  const int x = t.x0 + lx, y = t.y0 + ly;
  const bool active = x < G.nx && y < G.ny;
  // the cell whose phi fills this thread's own ring position (x, y wrapped
  // for a ragged tile's first padding column/row on a periodic axis)
  int ox = x, oy = y;
  const bool own_ok = wrap(ox, G.nx, G.px) && wrap(oy, G.ny, G.py);
  const int opos = (ly + 1) * TX + lx + 1;
  // ring cell handled by this thread: rows below/above the tile, then the
  // columns left/right of it
  const int NH = 2 * TX + 2 * G.by;
  int hpos = 0, hx = 0, hy = 0;
  bool halo_ok = false;
  if (tid < NH) {
    int ix, iy;
    if (tid < TX) { ix = tid; iy = 0; }
    else if (tid < 2 * TX) { ix = tid - TX; iy = TY - 1; }
    else if (tid < 2 * TX + G.by) { ix = 0; iy = 1 + tid - 2 * TX; }
    else { ix = TX - 1; iy = 1 + tid - 2 * TX - G.by; }
    hpos = iy * TX + ix;
    hx = t.x0 - 1 + ix;
    hy = t.y0 - 1 + iy;
    halo_ok = wrap(hx, G.nx, G.px) && wrap(hy, G.ny, G.py);
  }
  const unsigned sxy = (unsigned)G.nx * (unsigned)G.ny;

  // phi^n of plane p into the ring (own position: also its reference, walls
  // and solid flag for the collision one plane later, and its pulled h in a
  // thread-private LDS slot of the plane's parity: no registers held across
  // the plane, no second pull)
  R refn = R(0);
  unsigned wn = 0;
  bool sn = true;
  XWalls xwn{false, false, false};
  auto plane = [&](int p) {
    int pz = p;
    const bool zok = wrap(pz, G.nz, G.pz);
    R* rp = ring + (p & 3) * TXY;
    R v = sentinel<R>();
    sn = true;
    {
      const unsigned idx = ox + G.nx * oy + sxy * pz;
      bool sol = true;
      if (own_ok && zok) wn = cell_walls<MASK>(ox, oy, pz, idx, G, a.nbr, sol);
      xwn = x_walls<MASK>(own_ok && zok && !sol, ox, oy, pz, MASK ? wn : 0u, G);
      if (own_ok && zok && !sol) {
        R hh[Q_H];
        refn = phi_ref_of<S>(a.phi_prev, idx);
        const Nbhd nbp = make_nbhd(ox, oy, pz, G);
        if (FastWaves<S>::value && xwn.fast) {
          asm volatile("");
          load_h_x<S, kNtPull>(a.h_in, G.N, idx, nbp, xwn.xm, xwn.xp, a.cd.inv_scale_h, hh);
        } else {
          load_h<S, RULE_AB, kNtPull>(a.h_in, G.N, idx, nbp, wn, a.cd.inv_scale_h, hh);
        }
        v = phi_of(hh, refn);
        sn = false;
        R* hs = hbuf + (p & 1) * (Q_H * 256) + tid;
#pragma unroll
        for (int i = 0; i < Q_H; ++i) hs[i * 256] = hh[i];
      }
    }
    rp[opos] = v;
    if (tid < NH) {
      R hv = sentinel<R>();
      const unsigned idx = hx + G.nx * hy + sxy * pz;
      bool sol = true;
      unsigned w = 0;
      if (halo_ok && zok) w = cell_walls<MASK>(hx, hy, pz, idx, G, a.nbr, sol);
      const XWalls xw = x_walls<MASK>(halo_ok && zok && !sol, hx, hy, pz, MASK ? w : 0u, G);
      if (halo_ok && zok && !sol) {
        R hh[Q_H];
        const Nbhd nbh = make_nbhd(hx, hy, pz, G);
        if (FastWaves<S>::value && xw.fast) {
          asm volatile("");
          load_h_x<S, false>(a.h_in, G.N, idx, nbh, xw.xm, xw.xp, a.cd.inv_scale_h, hh);
        } else {
          load_h<S, RULE_AB, false>(a.h_in, G.N, idx, nbh, w, a.cd.inv_scale_h, hh);
        }
        hv = phi_of(hh, phi_ref_of<S>(a.phi_prev, idx));
      }
      rp[hpos] = hv;
    }
  };

  plane(t.z0 - 1);
  plane(t.z0);
  for (int z = t.z0; z < t.z1; ++z) {
    const R ref = refn;
    const unsigned walls = wn;
    const XWalls xw = xwn;
    const bool work = active && !sn;
    const unsigned idx = x + G.nx * y + sxy * z;
    const Nbhd nb = make_nbhd(x, y, z, G);
    R g[Q_G];
    if (work) {
      if (FastWaves<S>::value && xw.fast) {
        asm volatile("");
        load_g_x<S, kNtGPull>(a.g_in, G.N, idx, nb, xw.xm, xw.xp, a.cd.inv_scale_g, g);
      } else {
        load_g<S, RULE_AB, kNtGPull>(a.g_in, G.N, idx, nb, walls, a.cd.inv_scale_g, g);
      }
    }
    plane(z + 1);
    __syncthreads();
    if (work) {
      R h[Q_H];
      const R* hs = hbuf + (z & 1) * (Q_H * 256) + tid;
#pragma unroll
      for (int i = 0; i < Q_H; ++i) h[i] = hs[i * 256];
      const R* pm = ring + ((z - 1) & 3) * TXY;
      const R* p0 = ring + (z & 3) * TXY;
      const R* pp = ring + ((z + 1) & 3) * TXY;
      R Gx, Gy, Gz, lap;
      if (FastWaves<S>::value && xw.fast) stencil_sep<R, true>(pm, p0, pp, TX, lx, ly, xw.xm, xw.xp, Gx, Gy, Gz, lap);
      else stencil3(pm, p0, pp, TX, lx, ly, Gx, Gy, Gz, lap);
      // phi as the ring holds it (ref + sum h'); dphi = sum h' itself, so the
      // equilibrium's zeroth moment matches the populations' without phi's
      // rounding
      const R phi = p0[opos];
      CellState<R> c;
      prologue(phi, sum_h(h), g, Gx, Gy, Gz, lap, a.P, c);
      collide_g<R, MRT, GUO>(g, c, a.P);
      collide_h<R, MRT>(h, c, a.P);
      if (St::kShift) a.phi_out[idx] = phi;
      if (a.phi_src_out) a.phi_src_out[idx] = phi;
      const Planes<R> pl{pm, p0, pp, TX, lx, ly};
      store_own<S, kNtStore>(a.h_out, a.g_out, G.N, idx, a.cd, ref, phi, pl, h, g);
    }
  }
}

// ---- pipelined step: h pulls straight into LDS, two planes ahead ------------
// The FP32 form of the D3Q15 build issues the h pulls of plane z + 2 as
// global-to-LDS loads (one dword per lane) while plane z collides, and the g
// pulls of plane z + 1 once plane z's g has been stored, so that neither
// waits in registers nor exposes its latency at the next plane's phase-field
// sum.  Same arithmetic in the same order as k_step (bitwise the same
// results); the own cells' raw h wait in LDS until their collision, the ring
// cells' raw h until their phi.  Measured against k_step on one GPU: FP32
// drop impact 384^3 4.34 against 4.51 ms, rising bubble equal (0.635 /
// 0.632 ms).  The kernel is written for FP16 storage too (an FP16 value lands
// in the low half of its dword; tested bitwise against the in-place scheme),
// but there it needs 168 VGPRs with scratch spills at 3 waves per SIMD (5.26
// against 3.21 ms on the drop) and is 3-6 % slower at 2, so FP16 storage
// keeps k_step.  The D3Q27 phase lattice's 27 h per cell do not fit the LDS.
template <typename S>
struct DmaStep { static constexpr bool value = sizeof(S) == 4 && Q_H == 15; };
constexpr int kRingMax = 140;   // ring cells of the 64 x 4 tile, the largest of the tile shapes

template <typename R>
struct PlaneState {
  unsigned walls;   // own cell's wall bits (box faces and solid neighbours)
  bool skip;        // own position outside the lattice or solid
  R ref;            // own cell's shift reference phi^{n-1}
  bool hskip;       // ring cell outside the lattice or solid (or no ring cell)
  R href;           // ring cell's shift reference
};

// every LDS read issued so far has returned (lgkmcnt 0), and the compiler
// moves no memory access across this point
__device__ __forceinline__ void lds_settled() {
  asm volatile("s_waitcnt lgkmcnt(0)" ::: "memory");
}

// every global-to-LDS load issued so far by this wave has landed (vmcnt 0):
// their LDS writes are tracked by the vector memory counter only, and the
// compiler places its own waits for them inside the branches that read the
// slots, so a wave whose own cells are all skipped would read its ring
// cells' slots without one
__device__ __forceinline__ void dma_settled() {
  asm volatile("s_waitcnt vmcnt(0)" ::: "memory");
}

// one element per lane from global memory straight into LDS: lane l's value
// lands in the dword at lds_wave + l (an FP16 value in its low half); the
// size is written as a literal (a template-dependent size crashes this
// compiler's instruction selection)
template <typename S>
__device__ __forceinline__ void dma_pull(const S* gp, unsigned* lds_wave) {
  auto* l = (__attribute__((address_space(3))) void*)lds_wave;
  if constexpr (sizeof(S) == 2) __builtin_amdgcn_global_load_lds(gp, l, 2, 0, 0);
  else __builtin_amdgcn_global_load_lds(gp, l, 4, 0, 0);
}

template <typename S, bool MRT, bool MASK, bool GUO>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(StepWaves<S>::value)))
void k_step_dma(StepArgs<S> a) {
  using St = Store<S>;
  using R = typename St::R;
  static_assert(sizeof(S) != 8 && Q_H == 15, "pipelined step: FP32 arithmetic, D3Q15 phase field");
  constexpr int E = 4 / (int)sizeof(S);      // S elements per LDS dword
  __shared__ unsigned own_raw[2][Q_H][256];
  __shared__ unsigned ring_raw[2][Q_H][kRingMax];
  extern __shared__ unsigned char smem_raw[];
  const Geom& G = a.geo;
  const int TX = G.bx + 2, TY = G.by + 2, TXY = TX * TY;
  R* ring = reinterpret_cast<R*>(smem_raw);     // [4][TY][TX]
  const ChunkCoord t = chunk_of_block(G);
  const int lx = threadIdx.x, ly = threadIdx.y, tid = lx + ly * G.bx;
  const unsigned wave0 = __builtin_amdgcn_readfirstlane(tid & ~63);
  const int x = t.x0 + lx, y = t.y0 + ly;
  const bool active = x < G.nx && y < G.ny;
  int ox = x, oy = y;
  const bool own_ok = wrap(ox, G.nx, G.px) && wrap(oy, G.ny, G.py);
  const int opos = (ly + 1) * TX + lx + 1;
  // ring cells beyond the LDS slots (no tile shape has them) are not pulled
  const int NH = min(2 * TX + 2 * G.by, kRingMax);
  int hpos = 0, hx = 0, hy = 0;
  bool halo_ok = false;
  if (tid < NH) {
    int ix, iy;
    if (tid < TX) { ix = tid; iy = 0; }
    else if (tid < 2 * TX) { ix = tid - TX; iy = TY - 1; }
    else if (tid < 2 * TX + G.by) { ix = 0; iy = 1 + tid - 2 * TX; }
    else { ix = TX - 1; iy = 1 + tid - 2 * TX - G.by; }
    hpos = iy * TX + ix;
    hx = t.x0 - 1 + ix;
    hy = t.y0 - 1 + iy;
    halo_ok = wrap(hx, G.nx, G.px) && wrap(hy, G.ny, G.py);
  }
  const unsigned sxy = (unsigned)G.nx * (unsigned)G.ny;
  const unsigned NS = (unsigned)(G.N * (long long)sizeof(S));

  // pulls of plane p into the LDS slots of its parity; the plane's wall bits,
  // skip flags and shift references into ps
  auto issue = [&](int p, PlaneState<R>& ps) {
    int pz = p;
    const bool zok = wrap(pz, G.nz, G.pz);
    ps.skip = true;
    ps.hskip = true;
    ps.walls = 0;
    ps.ref = R(0);
    ps.href = R(0);
    {
      const unsigned idx = ox + G.nx * oy + sxy * pz;
      bool sol = true;
      if (own_ok && zok) ps.walls = cell_walls<MASK>(ox, oy, pz, idx, G, a.nbr, sol);
      if (own_ok && zok && !sol) {
        ps.skip = false;
        ps.ref = phi_ref_of<S>(a.phi_prev, idx);
        const Nbhd nb = make_nbhd(ox, oy, pz, G);
#pragma unroll
        for (int i = 0; i < Q_H; ++i)
          dma_pull(reinterpret_cast<const S*>(pair_base(a.h_in, G.N, i) +
                                              read_off<S, false, RULE_AB>(i, idx, nb, ps.walls, NS)),
                   &own_raw[p & 1][i][wave0]);
      }
    }
    if (tid < NH) {
      const unsigned idx = hx + G.nx * hy + sxy * pz;
      bool sol = true;
      unsigned w = 0;
      if (halo_ok && zok) w = cell_walls<MASK>(hx, hy, pz, idx, G, a.nbr, sol);
      if (halo_ok && zok && !sol) {
        ps.hskip = false;
        ps.href = phi_ref_of<S>(a.phi_prev, idx);
        const Nbhd nb = make_nbhd(hx, hy, pz, G);
#pragma unroll
        for (int i = 0; i < Q_H; ++i)
          dma_pull(reinterpret_cast<const S*>(pair_base(a.h_in, G.N, i) +
                                              read_off<S, false, RULE_AB>(i, idx, nb, w, NS)),
                   &ring_raw[p & 1][i][wave0]);
      }
    }
  };
  // raw h of this thread's own cell (plane parity s), decoded
  auto own_h = [&](int s, R (&h)[Q_H]) {
#pragma unroll
    for (int i = 0; i < Q_H; ++i)
      h[i] = St::template ld<false>(reinterpret_cast<const S*>(&own_raw[s][i][0]) + E * tid,
                                    a.cd.inv_scale_h);
  };
  // phi^n of plane p into the ring (sentinel for walls and solids)
  auto phi_plane = [&](int p, const PlaneState<R>& ps) {
    R* rp = ring + (p & 3) * TXY;
    R v = sentinel<R>();
    if (!ps.skip) {
      R hh[Q_H];
      own_h(p & 1, hh);
      v = phi_of(hh, ps.ref);
    }
    rp[opos] = v;
    if (tid < NH) {
      R hv = sentinel<R>();
      if (!ps.hskip) {
        R hh[Q_H];
#pragma unroll
        for (int i = 0; i < Q_H; ++i)
          hh[i] = St::template ld<false>(reinterpret_cast<const S*>(&ring_raw[p & 1][i][0]) + E * tid,
                                         a.cd.inv_scale_h);
        hv = phi_of(hh, ps.href);
      }
      rp[hpos] = hv;
    }
  };

  PlaneState<R> s0, s1, s2;
  issue(t.z0 - 1, s0);
  issue(t.z0, s1);
  dma_settled();
  phi_plane(t.z0 - 1, s0);
  lds_settled();
  issue(t.z0 + 1, s2);         // into the slots of plane z0 - 1, consumed above
  phi_plane(t.z0, s1);
  s0 = s1;
  s1 = s2;
  typename Raw<S>::T graw[Q_G];
  {
    const unsigned idx = x + G.nx * y + sxy * t.z0;
    if (active && !s0.skip)
      load_g_raw<S, RULE_AB, kNtGPull>(a.g_in, G.N, idx, make_nbhd(x, y, t.z0, G), s0.walls, graw);
  }
  for (int z = t.z0; z < t.z1; ++z) {
    // s0: plane z (phi in the ring, raw h in LDS, raw g in registers);
    // s1: plane z + 1 (pulls in flight, landed after the wait)
    dma_settled();
    phi_plane(z + 1, s1);
    __syncthreads();
    const bool work = active && !s0.skip;
    const unsigned idx = x + G.nx * y + sxy * z;
    R h[Q_H];
    if (work) own_h(z & 1, h);
    // the slot's values are in registers before its refill is issued
    lds_settled();
    const R* pm = ring + ((z - 1) & 3) * TXY;
    const R* p0 = ring + (z & 3) * TXY;
    const R* pp = ring + ((z + 1) & 3) * TXY;
    const R phi = p0[opos];
    CellState<R> c;
    if (work) {
      R g[Q_G];
#pragma unroll
      for (int i = 0; i < Q_G; ++i) g[i] = decode_raw<S>(graw[i], a.cd.inv_scale_g);
      R Gx, Gy, Gz, lap;
      stencil3(pm, p0, pp, TX, lx, ly, Gx, Gy, Gz, lap);
      prologue(phi, sum_h(h), g, Gx, Gy, Gz, lap, a.P, c);
      collide_g<R, MRT, GUO>(g, c, a.P);
      // the stores walk the population rows (one address add each); g first
      // so that its registers take the next plane's pulls
      S* p = next_row(a.g_out, (long long)idx);
#pragma unroll
      for (int i = 0; i < Q_G; ++i) {
        St::template st<kNtStore>(p, g[i], a.cd.scale_g);
        if (i + 1 < Q_G) p = next_row(p, G.N);
      }
    }
    // g of plane z + 1, then the h of plane z + 2 into the slots plane z has
    // left: in flight over the h collision and stores of this plane and the
    // next plane's phase-field sum, with only the h stores issued after them
    if (z + 1 < t.z1 && active && !s1.skip)
      load_g_raw<S, RULE_AB, kNtGPull>(a.g_in, G.N, idx + sxy, make_nbhd(x, y, z + 1, G), s1.walls,
                                       graw);
    if (z + 2 <= t.z1) issue(z + 2, s2);
    if (work) {
      collide_h<R, MRT>(h, c, a.P);
      if (St::kShift) a.phi_out[idx] = phi;
      if (a.phi_src_out) a.phi_src_out[idx] = phi;
      const Planes<R> pl{pm, p0, pp, TX, lx, ly};
      S* p = next_row(a.h_out, (long long)idx);
#pragma unroll
      for (int i = 0; i < Q_H; ++i) {
        St::template st<kNtStore>(p, rebase<S>(i, h[i], s0.ref, phi, pl), a.cd.scale_h);
        if (i + 1 < Q_H) p = next_row(p, G.N);
      }
    }
    s0 = s1;
    s1 = s2;
  }
}

template <typename S>
struct CellArgs {
  using R = typename Store<S>::R;
  const S* h_in;             // populations read
  const S* g_in;
  S* h;                      // populations written (AA step; == h_in in place)
  S* g;
  const R* phi;              // phi^n (stencil source)
  const R* phi_prev;         // phi^{n-1}: shift reference of the state read
  const unsigned char* mask;
  Geom geo;
  Phys<R> P;
  Codec<R> cd;
  double* out_phi;           // FP64 outputs of the moments kernel (may be null)
  double* out_u;
  double* out_p;
};

// AA cache policy (measured on the rising-bubble lattice, FP32): even steps
// (own slots, aligned rows) stream with non-temporal loads and stores; odd
// steps (neighbour slots, rows one element off alignment, lines shared by
// neighbouring waves) use cached loads and non-temporal stores (non-temporal
// odd loads: AA step -10 %; cached odd stores: no change).
template <bool ODD> struct AaPolicy {
  static constexpr bool nt_load = !ODD;
  static constexpr bool nt_store = true;
};

// In-place AA collide-and-stream of both lattices for one plane of one tile
// (phi^n staged in LDS).  Also runs out of place (h_in != h) between saved
// states.
template <typename S, bool MRT, bool ODD, bool MASK, bool GUO>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(StepWaves<S>::value)))
void k_cell_aa(CellArgs<S> a) {
  using St = Store<S>;
  using R = typename St::R;
  extern __shared__ unsigned char smem_raw[];
  R* tile = reinterpret_cast<R*>(smem_raw);
  const Geom& G = a.geo;
  const int TX = G.bx + 2, TY = G.by + 2;
  const TileCoord t = tile_of_block(G);
  load_phi_tile<R, MASK>(tile, a.phi, a.mask, G, t);
  __syncthreads();
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int x = t.x0 + lx, y = t.y0 + ly, z = t.z;
  if (x >= G.nx || y >= G.ny) return;
  const unsigned idx = x + (unsigned)G.nx * (y + (unsigned)G.ny * z);
  const R* pm = tile;
  const R* p0 = tile + TX * TY;
  const R* pp = tile + 2 * TX * TY;
  const R phi = p0[(ly + 1) * TX + lx + 1];
  if (phi == sentinel<R>()) return;   // solid cell
  const unsigned walls = wall_bits(tile, TX, TY, lx, ly);
  const Nbhd nb = make_nbhd(x, y, z, G);
  R h[Q_H], g[Q_G];
  constexpr int RULE = ODD ? RULE_AA_ODD : RULE_AA_EVEN;
  load_h<S, RULE, AaPolicy<ODD>::nt_load>(a.h_in, G.N, idx, nb, walls, a.cd.inv_scale_h, h);
  load_g<S, RULE, AaPolicy<ODD>::nt_load>(a.g_in, G.N, idx, nb, walls, a.cd.inv_scale_g, g);
  const R ref = phi_ref_of<S>(a.phi_prev, idx);
  R Gx, Gy, Gz, lap;
  stencil3(pm, p0, pp, TX, lx, ly, Gx, Gy, Gz, lap);
  CellState<R> c;
  prologue(phi, sum_h(h), g, Gx, Gy, Gz, lap, a.P, c);
  collide_g<R, MRT, GUO>(g, c, a.P);
  collide_h<R, MRT>(h, c, a.P);
  const Planes<R> pl{pm, p0, pp, TX, lx, ly};
  store_aa<S, ODD, AaPolicy<ODD>::nt_store>(a.h, a.g, G.N, idx, nb, walls, a.cd, ref, phi, pl, h, g);
}

// Cell moments phi, u, p* of the current state with the step's force
// prologue (one plane per block, phi^n from the stored field).
template <typename S, int RULE, bool MASK>
__global__ __launch_bounds__(256) void k_moments(CellArgs<S> a) {
  using R = typename Store<S>::R;
  extern __shared__ unsigned char smem_raw[];
  R* tile = reinterpret_cast<R*>(smem_raw);
  const Geom& G = a.geo;
  const int TX = G.bx + 2, TY = G.by + 2;
  const TileCoord t = tile_of_block(G);
  load_phi_tile<R, MASK>(tile, a.phi, a.mask, G, t);
  __syncthreads();
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int x = t.x0 + lx, y = t.y0 + ly, z = t.z;
  if (x >= G.nx || y >= G.ny) return;
  const unsigned idx = x + (unsigned)G.nx * (y + (unsigned)G.ny * z);
  const R phi = tile[(TY + ly + 1) * TX + lx + 1];
  if (phi == sentinel<R>()) {   // solid cell
    if (a.out_phi) a.out_phi[idx] = 0.0;
    if (a.out_p) a.out_p[idx] = 0.0;
    if (a.out_u) { a.out_u[idx] = 0.0; a.out_u[G.N + idx] = 0.0; a.out_u[2 * G.N + idx] = 0.0; }
    return;
  }
  const unsigned walls = wall_bits(tile, TX, TY, lx, ly);
  const Nbhd nb = make_nbhd(x, y, z, G);
  R g[Q_G];
  load_g<S, RULE, false>(a.g_in, G.N, idx, nb, walls, a.cd.inv_scale_g, g);
  R Gx, Gy, Gz, lap;
  stencil(tile, TX, TY, lx, ly, Gx, Gy, Gz, lap);
  CellState<R> c;
  prologue(phi, phi, g, Gx, Gy, Gz, lap, a.P, c);
  if (a.out_phi) a.out_phi[idx] = double(c.phi);
  if (a.out_p) a.out_p[idx] = double(c.p);
  if (a.out_u) {
    a.out_u[idx] = double(c.ux);
    a.out_u[G.N + idx] = double(c.uy);
    a.out_u[2 * G.N + idx] = double(c.uz);
  }
}

template <typename S>
struct LightArgs {
  using R = typename Store<S>::R;
  const S* h;
  const S* g;
  const unsigned* nbr;
  const R* phi_prev;   // phi^{n-1}: shift reference of the state read
  Geom geo;
  Codec<R> cd;
  R* phi_out;          // gather target (compute precision)
  double* out_h;       // natural-order FP64 populations
  double* out_g;
  double* partials;    // [nblocks][5]
};

enum LightMode { LM_GATHER = 0, LM_READ_POPS = 1, LM_REDUCE = 2 };

// phi of the state (phi_ref + sum of the h deviations the next step reads,
// in the order the step uses), population readout, or per-block FP64 sums.
template <typename S, int RULE, bool MASK, int LM>
__global__ __launch_bounds__(256) void k_light(LightArgs<S> a) {
  using R = typename Store<S>::R;
  const Geom& G = a.geo;
  const TileCoord t = tile_of_block(G);
  const int x = t.x0 + threadIdx.x, y = t.y0 + threadIdx.y, z = t.z;
  const bool in = x < G.nx && y < G.ny;
  double acc[5] = {0, 0, 0, 0, 0};
  if (in) {
    const unsigned idx = x + (unsigned)G.nx * (y + (unsigned)G.ny * z);
    bool solid;
    const unsigned walls = cell_walls<MASK>(x, y, z, idx, G, a.nbr, solid);
    if (solid) {
      if (LM == LM_GATHER) a.phi_out[idx] = R(0);
      if (LM == LM_READ_POPS) {
        for (int i = 0; i < Q_H; ++i) a.out_h[i * G.N + idx] = 0.0;
        for (int i = 0; i < Q_G; ++i) a.out_g[i * G.N + idx] = 0.0;
      }
    } else {
      const Nbhd nb = make_nbhd(x, y, z, G);
      const R ref = phi_ref_of<S>(a.phi_prev, idx);
      R h[Q_H], g[Q_G];
      // the gather of a state read with the even AA rule (own slots, aligned
      // rows) streams its rows non-temporally: measured on the rising-bubble
      // lattice (FP32) 0.114 ms against 0.170 ms cached, the AA step 2.3 %
      // faster; the odd rule's shifted rows keep cached loads
      load_h<S, RULE, RULE == RULE_AA_EVEN && LM == LM_GATHER>(a.h, G.N, idx, nb, walls,
                                                              a.cd.inv_scale_h, h);
      if (LM == LM_GATHER) {
        a.phi_out[idx] = phi_of(h, ref);
      } else {
        load_g<S, RULE, false>(a.g, G.N, idx, nb, walls, a.cd.inv_scale_g, g);
        // absolute populations: h_i = h'_i + w_i phi_ref
        if (LM == LM_READ_POPS) {
#pragma unroll
          for (int i = 0; i < Q_H; ++i) a.out_h[i * G.N + idx] = double(h[i]) + wh(i) * double(ref);
#pragma unroll
          for (int i = 0; i < Q_G; ++i) a.out_g[i * G.N + idx] = double(g[i]);
        } else {
          double s = double(ref);
#pragma unroll
          for (int i = 0; i < Q_H; ++i) s += double(h[i]);
          acc[0] = s;
#pragma unroll
          for (int i = 0; i < Q_G; ++i) {
            const Dir d = cg(i);
            const double v = double(g[i]);
            acc[1] += v;
            acc[2] += d.x * v;
            acc[3] += d.y * v;
            acc[4] += d.z * v;
          }
        }
      }
    }
  }
  if (LM == LM_REDUCE) {
    // wave64 butterfly, then the 4 waves of the block through LDS (fixed order)
    __shared__ double red[4][5];
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      double v = acc[k];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
      acc[k] = v;
    }
    const int tid = threadIdx.x + threadIdx.y * G.bx;
    if ((tid & 63) == 0) {
#pragma unroll
      for (int k = 0; k < 5; ++k) red[tid >> 6][k] = acc[k];
    }
    __syncthreads();
    if (tid < 5) {
      a.partials[(long long)blockIdx.x * 5 + tid] =
          ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
    }
  }
}

// Second reduction pass: one block sums nblocks x 5 partials in a fixed order.
__global__ __launch_bounds__(1024) void k_reduce_final(const double* __restrict__ partials,
                                                       unsigned nblocks, int ncomp,
                                                       double* __restrict__ out) {
  __shared__ double red[16][8];
  const int tid = threadIdx.x;
  double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
  for (unsigned b = tid; b < nblocks; b += 1024)
    for (int k = 0; k < ncomp; ++k) acc[k] += partials[(long long)b * ncomp + k];
  for (int k = 0; k < ncomp; ++k) {
    double v = acc[k];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    acc[k] = v;
  }
  if ((tid & 63) == 0)
    for (int k = 0; k < ncomp; ++k) red[tid >> 6][k] = acc[k];
  __syncthreads();
  if (tid < ncomp) {
    double s = 0;
    for (int w = 0; w < 16; ++w) s += red[w][tid];
    out[tid] = s;
  }
}

// Solid-neighbour bits from the mask (box faces are not included; the
// kernels add them from the coordinates).
__global__ __launch_bounds__(256) void k_nbr_bits(const unsigned char* __restrict__ mask, Geom G,
                                                  unsigned* __restrict__ out) {
  const long long i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= G.N) return;
  const int x = int(i % G.nx), y = int((i / G.nx) % G.ny), z = int(i / ((long long)G.nx * G.ny));
  unsigned b = mask[i] ? 1u : 0u;
  for (int k = 1; k < 27; ++k) {
    int X = x + kC27[k].x, Y = y + kC27[k].y, Z = z + kC27[k].z;
    if (wrap(X, G.nx, G.px) && wrap(Y, G.ny, G.py) && wrap(Z, G.nz, G.pz) &&
        mask[X + (long long)G.nx * (Y + (long long)G.ny * Z)])
      b |= 1u << k;
  }
  out[i] = b;
}

template <typename S>
struct InitArgs {
  using R = typename Store<S>::R;
  S* h;
  S* g;
  const unsigned* nbr;
  const double* phi0;
  const double* u0;      // may be null
  const double* p0;      // may be null
  const R* phi_ref;      // R(phi0): the shift reference of the initial state (shifted forms)
  Geom geo;
  Codec<R> cd;
};

// Equilibrium initialisation: every fluid cell writes its equilibrium
// populations where the first step reads them (two buffers: the pull slots;
// AA: its own slots, the even-step rule); the shifted forms store them
// relative to w_i R(phi0) of that cell, the first step's reference.
template <typename S, bool AA, bool MASK>
__global__ __launch_bounds__(256) void k_init(InitArgs<S> a) {
  using R = typename Store<S>::R;
  using St = Store<S>;
  const Geom& G = a.geo;
  const TileCoord t = tile_of_block(G);
  const int x = t.x0 + threadIdx.x, y = t.y0 + threadIdx.y, z = t.z;
  if (x >= G.nx || y >= G.ny) return;
  const unsigned idx = x + (unsigned)G.nx * (y + (unsigned)G.ny * z);
  bool solid;
  const unsigned walls = cell_walls<MASK>(x, y, z, idx, G, a.nbr, solid);
  if (solid) return;
  const Nbhd nb = make_nbhd(x, y, z, G);
  const R phi = R(a.phi0[idx]);
  R ux = R(0), uy = R(0), uz = R(0), p = R(0);
  if (a.u0) { ux = R(a.u0[idx]); uy = R(a.u0[G.N + idx]); uz = R(a.u0[2 * G.N + idx]); }
  if (a.p0) p = R(a.p0[idx]);
  const R uu = ux * ux + uy * uy + uz * uz;
  const R ref = phi_ref_of<S>(a.phi_ref, idx);
  constexpr int RULE = AA ? RULE_AA_EVEN : RULE_AB;
  const unsigned NS = (unsigned)(G.N * (long long)sizeof(S));
  // h^eq_i - w_i ref = w_i [(phi - ref) + phi (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)]
  const R dphi = phi - ref;
#pragma unroll
  for (int i = 0; i < Q_H; ++i) {
    const R cu = dot(ch(i), ux, uy, uz);
    const R v = R(wh(i)) * (dphi + phi * (cu * (R(3) + R(4.5) * cu) - R(1.5) * uu));
    S* q = reinterpret_cast<S*>(pair_base(a.h, G.N, i) + read_off<S, false, RULE>(i, idx, nb, walls, NS));
    St::st(q, v, a.cd.scale_h);
  }
  const R baseg = p - R(1.5) * uu;
#pragma unroll
  for (int i = 0; i < Q_G; ++i) {
    const R cu = dot(cg(i), ux, uy, uz);
    const R v = R(wg(i)) * (baseg + cu * (R(3) + R(4.5) * cu));
    S* q = reinterpret_cast<S*>(pair_base(a.g, G.N, i) + read_off<S, true, RULE>(i, idx, nb, walls, NS));
    St::st(q, v, a.cd.scale_g);
  }
}

// zero n 16-byte words (grid-stride)
__global__ __launch_bounds__(256) void k_zero16(uint4* __restrict__ p, size_t n) {
  const size_t stride = (size_t)gridDim.x * 256;
  for (size_t i = (size_t)blockIdx.x * 256 + threadIdx.x; i < n; i += stride) p[i] = make_uint4(0, 0, 0, 0);
}

// FP64 phi0 -> compute precision (zero in solids)
template <typename R>
__global__ __launch_bounds__(256) void k_phi_from_f64(const double* __restrict__ in,
                                                       const unsigned char* __restrict__ mask,
                                                       long long N, R* __restrict__ out) {
  const long long i = blockIdx.x * 256ll + threadIdx.x;
  if (i < N) out[i] = (mask && mask[i]) ? R(0) : R(in[i]);
}

// ---- halo pack of the z-slab decomposition ---------------------------------
// Split along z into slabs, each step needs from a neighbouring slab the
// populations that stream across the shared face: those with c_z = -1 stored
// at plane 0 go to the slab below, those with c_z = +1 stored at plane nz - 1
// to the slab above.  k_pack_faces copies them into a staging buffer, row by
// row (blockIdx.y = face * rows + row): face 0 then face 1, within a face the
// h rows then the g rows, each the nx * ny values of one population on that
// plane in the storage type, unchanged.
struct PackRows {
  int n;                     // rows per face
  int nh;                    // of which the first nh are h rows
  int pop[2][Q_H + Q_G];     // population index of each row, per face
};

template <typename S>
__global__ __launch_bounds__(256) void k_pack_faces(const S* __restrict__ h, const S* __restrict__ g,
                                                    S* __restrict__ dst, long long N, long long nxy,
                                                    int nz, PackRows r) {
  const long long e = (long long)blockIdx.x * 256 + threadIdx.x;
  if (e >= nxy) return;
  const int row = blockIdx.y;
  const int face = row >= r.n ? 1 : 0;
  const int k = row - face * r.n;
  const long long plane = face ? (long long)(nz - 1) * nxy : 0;
  const S* src = (k < r.nh ? h : g) + (long long)r.pop[face][k] * N + plane + e;
  dst[(long long)row * nxy + e] = *src;
}

// phi (compute precision) -> FP64
template <typename R>
__global__ __launch_bounds__(256) void k_phi_to_f64(const R* __restrict__ phi, long long N,
                                                     double* __restrict__ out) {
  const long long i = blockIdx.x * 256ll + threadIdx.x;
  if (i < N) out[i] = double(phi[i]);
}

}  // namespace pflbm
