// Forward kernels of the coupled phase-field LBM step on gfx950.
//
// Data layout in HBM (all structure-of-arrays, x fastest):
//   h[i * N + idx], i < 15       phase-field populations (storage type S)
//   g[i * N + idx], i < 27       hydrodynamic populations
//   phi[2][N]                    phase field, double-buffered (compute type R):
//                                phi^n (stencil source) and phi^{n-1}
//   mask[N]                      optional solids (1 = solid)
//
// Streaming is the in-place AA pattern (one population buffer per lattice):
//   even step: read own slots f[i][x], write f*_i into own slot f[opp i][x];
//   odd step:  read f_i(x) from f[opp i][x - c_i] (or f[i][x] when x - c_i is
//              a wall/solid: the value bounced back there), write f*_i into
//              f[i][x + c_i] (or f[opp i][x] when x + c_i is a wall/solid).
// Every slot is read and written by exactly one cell per step, which makes
// the update race-free without a second population buffer; halfway
// bounce-back falls out of the redirected addresses (paper: streaming
// eq. and bounce-back walls).  After an odd step the buffer holds the
// natural layout f[i][x] = f_i(x).
//
// One thread per cell.  A block is a bx * by tile of one z plane (256
// threads); it stages phi of the tile plus a one-cell halo on three planes in
// LDS, where out-of-box and solid neighbours carry a sentinel.  The sentinel
// both selects the wall rule of the phi stencils and tells the AA addressing
// which neighbours are walls, so no mask read is needed on the hot path.
//
// Blocks are issued round-robin over the 8 XCDs; xcd_remap() renumbers them
// so that each XCD walks one contiguous slab of tiles, keeping the halo and
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
  unsigned nblocks;       // tiles_x * tiles_y * nz
  long long N;
};

// ---- storage codecs -------------------------------------------------------
// ld/st take the shift s and the scale: stored = (f - s) * 2^k.  FP64 and
// FP32 store f itself.  FP16 storage shifts every h population by w_i times
// the phase field of the cell that wrote it (phi^n of the writer, which the
// reader finds in the previous phi buffer), so both pure phases store values
// near zero; g is stored unshifted (it is small in the p* gauge).
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
  __device__ static R ld(const double* p, R, R) { return ld_nt<NT>(p); }
  template <bool NT = true>
  __device__ static void st(double* p, R v, R, R) { st_nt<NT>(p, v); }
};
template <>
struct Store<float> {
  using R = float;
  static constexpr bool kShift = false;
  template <bool NT = true>
  __device__ static R ld(const float* p, R, R) { return ld_nt<NT>(p); }
  template <bool NT = true>
  __device__ static void st(float* p, R v, R, R) { st_nt<NT>(p, v); }
};
template <>
struct Store<_Float16> {
  using R = float;
  static constexpr bool kShift = true;
  template <bool NT = true>
  __device__ static R ld(const _Float16* p, R shift, R inv_scale) {
    return static_cast<float>(ld_nt<NT>(p)) * inv_scale + shift;
  }
  template <bool NT = true>
  __device__ static void st(_Float16* p, R v, R shift, R scale) {
    st_nt<NT>(p, static_cast<_Float16>((v - shift) * scale));
  }
};

// Cache policy of the population streams (measured on the rising-bubble
// lattice, FP32, per step: 0.849 ms all-streaming -> 0.721 ms with this one):
//   even steps (own slots, aligned rows): non-temporal loads and stores;
//   odd steps (neighbour slots, rows one element off alignment, lines shared
//     by neighbouring waves): cached loads, non-temporal stores;
//   phi update: cached loads (the next collide-and-stream re-reads h, part of
//     which the 256 MB last-level cache then still holds).
template <bool ODD> struct PopPolicy {
  static constexpr bool nt_load = !ODD;
  static constexpr bool nt_store = true;
};
constexpr bool kNtGather = false;

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

// Neighbour coordinates with periodic wrap; returns false outside a wall.
__device__ __forceinline__ bool wrap(int& v, int n, int periodic) {
  if (v < 0) { if (!periodic) return false; v += n; }
  else if (v >= n) { if (!periodic) return false; v -= n; }
  return true;
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
// entries are never dereferenced because the tile marks them as walls).
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

// Bit k of the result: neighbour in direction kC27[k] is a wall or solid.
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

// grad phi and lap phi from the LDS tile (missing neighbours repeat phi(x)),
// over opposite pairs: the gradient takes each pair's difference, the
// Laplacian its sum.
template <typename R>
__device__ __forceinline__ void stencil(const R* tile, int TX, int TY, int lx, int ly, R& Gx,
                                        R& Gy, R& Gz, R& lap) {
  const R p0 = tile[(TY + ly + 1) * TX + lx + 1];
  Gx = Gy = Gz = lap = R(0);
#pragma unroll
  for (int k = 1; k < 27; k += 2) {
    const Dir d = cg(k);
    const R va = tile[((1 + d.z) * TY + (ly + 1 + d.y)) * TX + (lx + 1 + d.x)];
    const R vb = tile[((1 - d.z) * TY + (ly + 1 - d.y)) * TX + (lx + 1 - d.x)];
    const R da = (va == sentinel<R>()) ? R(0) : va - p0;
    const R db = (vb == sentinel<R>()) ? R(0) : vb - p0;
    const R w = R(wg(k));
    const R odd = w * (da - db);
    if (d.x) Gx += d.x > 0 ? odd : -odd;
    if (d.y) Gy += d.y > 0 ? odd : -odd;
    if (d.z) Gz += d.z > 0 ? odd : -odd;
    lap += w * (da + db);
  }
  Gx *= R(3);
  Gy *= R(3);
  Gz *= R(3);
  lap *= R(6);
}

// ---- population access (AA pattern) --------------------------------------
// Population i arriving at cell x was written by x - c_i, or by x itself when
// x - c_i is a wall or solid (bounce-back); this holds for both parities.
// phw[i] is the phase field of that writer (only used by FP16 storage).
//
// Addresses: an opposite pair (i, i+1), i odd, is addressed from the pair's
// first population (a wave-uniform base); the per-lane part is one 32-bit byte
// offset, cell * sizeof(S) plus N * sizeof(S) for the pair's second member.
// In odd steps the lane picks between the neighbour slot and its own
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

template <typename S, bool ODD>
__device__ __forceinline__ void load_pops(const S* __restrict__ H, const S* __restrict__ Gp,
                                          long long N, unsigned idx, const Nbhd& nb,
                                          unsigned walls, const Codec<typename Store<S>::R>& cd,
                                          const typename Store<S>::R (&phw)[Q_H],
                                          typename Store<S>::R (&h)[Q_H],
                                          typename Store<S>::R (&g)[Q_G]) {
  using St = Store<S>;
  using R = typename St::R;
  const unsigned NS = (unsigned)(N * (long long)sizeof(S));
#pragma unroll
  for (int i = 0; i < Q_H; ++i) {
    unsigned off = pair_off<S>(i, idx, NS);
    if (ODD && i) {
      const Dir d = ch(i);
      if (!(walls & (1u << nb27(-d.x, -d.y, -d.z)))) off = pair_off<S>(opp(i), nb.at(-d.x, -d.y, -d.z), NS);
    }
    const S* p = reinterpret_cast<const S*>(pair_base(H, N, i) + off);
    h[i] = St::template ld<PopPolicy<ODD>::nt_load>(p, St::kShift ? R(wh(i)) * phw[i] : R(0), cd.inv_scale_h);
  }
#pragma unroll
  for (int i = 0; i < Q_G; ++i) {
    unsigned off = pair_off<S>(i, idx, NS);
    if (ODD && i) {
      const Dir d = cg(i);
      if (!(walls & (1u << nb27(-d.x, -d.y, -d.z)))) off = pair_off<S>(opp(i), nb.at(-d.x, -d.y, -d.z), NS);
    }
    const S* p = reinterpret_cast<const S*>(pair_base(Gp, N, i) + off);
    g[i] = St::template ld<PopPolicy<ODD>::nt_load>(p, R(0), cd.inv_scale_g);
  }
}

// phi_self: the writer's own phi^n (the field value, bit-identical to what
// the readers of the next step look up).
template <typename S, bool ODD>
__device__ __forceinline__ void store_pops(S* __restrict__ H, S* __restrict__ Gp, long long N,
                                           unsigned idx, const Nbhd& nb, unsigned walls,
                                           const Codec<typename Store<S>::R>& cd,
                                           typename Store<S>::R phi_self,
                                           const typename Store<S>::R (&h)[Q_H],
                                           const typename Store<S>::R (&g)[Q_G]) {
  using St = Store<S>;
  using R = typename St::R;
  const unsigned NS = (unsigned)(N * (long long)sizeof(S));
#pragma unroll
  for (int i = 0; i < Q_H; ++i) {
    unsigned off = pair_off<S>(opp(i), idx, NS);
    if (ODD && i) {
      const Dir d = ch(i);
      if (!(walls & (1u << nb27(d.x, d.y, d.z)))) off = pair_off<S>(i, nb.at(d.x, d.y, d.z), NS);
    }
    S* p = reinterpret_cast<S*>(pair_base(H, N, i) + off);
    St::template st<PopPolicy<ODD>::nt_store>(p, h[i], St::kShift ? R(wh(i)) * phi_self : R(0), cd.scale_h);
  }
#pragma unroll
  for (int i = 0; i < Q_G; ++i) {
    unsigned off = pair_off<S>(opp(i), idx, NS);
    if (ODD && i) {
      const Dir d = cg(i);
      if (!(walls & (1u << nb27(d.x, d.y, d.z)))) off = pair_off<S>(i, nb.at(d.x, d.y, d.z), NS);
    }
    S* p = reinterpret_cast<S*>(pair_base(Gp, N, i) + off);
    St::template st<PopPolicy<ODD>::nt_store>(p, g[i], R(0), cd.scale_g);
  }
}

// Writer phase fields from an LDS tile (3 planes + halo) of phi^{n-1}.
template <typename R>
__device__ __forceinline__ void writer_phi_tile(const R* tp, int TX, int TY, int lx, int ly,
                                                unsigned walls, R (&phw)[Q_H]) {
  const R self = tp[(TY + ly + 1) * TX + lx + 1];
#pragma unroll
  for (int i = 0; i < Q_H; ++i) {
    const Dir d = ch(i);
    phw[i] = (walls & (1u << nb27(-d.x, -d.y, -d.z)))
                 ? self
                 : tp[((1 - d.z) * TY + (ly + 1 - d.y)) * TX + (lx + 1 - d.x)];
  }
}

// Writer phase fields read directly from a phi buffer.
template <typename R>
__device__ __forceinline__ void writer_phi_direct(const R* __restrict__ phi, unsigned idx,
                                                  const Nbhd& nb, unsigned walls, R (&phw)[Q_H]) {
  const R self = phi[idx];
#pragma unroll
  for (int i = 0; i < Q_H; ++i) {
    const Dir d = ch(i);
    phw[i] = (walls & (1u << nb27(-d.x, -d.y, -d.z))) ? self : phi[nb.at(-d.x, -d.y, -d.z)];
  }
}

template <typename S>
struct CellArgs {
  using R = typename Store<S>::R;
  const S* h_in;             // populations read (== h, g for the in-place step)
  const S* g_in;
  S* h;                      // populations written
  S* g;
  const R* phi;              // phi^n (stencil source)
  const R* phi_prev;         // phi^{n-1} (writers of the populations read now)
  const unsigned char* mask;
  Geom geo;
  Phys<R> P;
  Codec<R> cd;
  // outputs of the moments mode (FP64, may be null)
  double* out_phi;
  double* out_u;
  double* out_p;
};

enum Mode { MODE_STEP = 0, MODE_MOMENTS = 1 };

// Occupancy request of the fused kernel: 3 waves per SIMD (<= 168 VGPRs)
// for the FP32-arithmetic forms, measured faster than the unconstrained 2;
// the FP64 form keeps the compiler's choice (forcing it spills).
template <typename S>
struct StepWaves { static constexpr int value = sizeof(S) == 8 ? 1 : 3; };

// Fused collide + stream of both lattices (MODE_STEP), or the cell moments
// with the same force prologue (MODE_MOMENTS).
template <typename S, bool MRT, bool ODD, bool MASK, int MODE>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(StepWaves<S>::value)))
void k_cell(CellArgs<S> a) {
  using R = typename Store<S>::R;
  extern __shared__ unsigned char smem_raw[];
  R* tile = reinterpret_cast<R*>(smem_raw);
  const Geom& G = a.geo;
  const int TX = G.bx + 2, TY = G.by + 2;
  R* tile_prev = tile + TX * TY * 3;          // only with FP16 storage
  const TileCoord t = tile_of_block(G);
  load_phi_tile<R, MASK>(tile, a.phi, a.mask, G, t);
  if (Store<S>::kShift) load_phi_tile<R, MASK>(tile_prev, a.phi_prev, a.mask, G, t);
  __syncthreads();
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int x = t.x0 + lx, y = t.y0 + ly, z = t.z;
  if (x >= G.nx || y >= G.ny) return;
  const long long idx = x + (long long)G.nx * (y + (long long)G.ny * z);
  if (tile[(TY + ly + 1) * TX + lx + 1] == sentinel<R>()) {   // solid cell
    if (MODE == MODE_MOMENTS) {
      if (a.out_phi) a.out_phi[idx] = 0.0;
      if (a.out_p) a.out_p[idx] = 0.0;
      if (a.out_u) { a.out_u[idx] = 0.0; a.out_u[G.N + idx] = 0.0; a.out_u[2 * G.N + idx] = 0.0; }
    }
    return;
  }
  const unsigned walls = wall_bits(tile, TX, TY, lx, ly);
  const Nbhd nb = make_nbhd(x, y, z, G);
  R phw[Q_H];
  if (Store<S>::kShift) writer_phi_tile(tile_prev, TX, TY, lx, ly, walls, phw);
  R h[Q_H], g[Q_G];
  load_pops<S, ODD>(a.h_in, a.g_in, G.N, (unsigned)idx, nb, walls, a.cd, phw, h, g);
  R Gx, Gy, Gz, lap;
  stencil(tile, TX, TY, lx, ly, Gx, Gy, Gz, lap);
  CellState<R> c;
  prologue(h, g, Gx, Gy, Gz, lap, a.P, c);
  if (MODE == MODE_MOMENTS) {
    if (a.out_phi) a.out_phi[idx] = double(c.phi);
    if (a.out_p) a.out_p[idx] = double(c.p);
    if (a.out_u) {
      a.out_u[idx] = double(c.ux);
      a.out_u[G.N + idx] = double(c.uy);
      a.out_u[2 * G.N + idx] = double(c.uz);
    }
    return;
  }
  collide_g<R, MRT>(g, c, a.P);
  collide_h<R, MRT>(h, c, a.P);
  store_pops<S, ODD>(a.h, a.g, G.N, (unsigned)idx, nb, walls, a.cd,
                    tile[(TY + ly + 1) * TX + lx + 1], h, g);
}

// Neighbour-is-wall bits for the populations of one cell, without LDS
// (used by the light kernels: gather, readout, reductions).
template <bool MASK>
__device__ __forceinline__ unsigned wall_bits_direct(int x, int y, int z, const Geom& G,
                                                     const unsigned char* __restrict__ mask) {
  unsigned b = 0;
#pragma unroll
  for (int k = 1; k < 27; ++k) {
    const Dir d = cg(k);
    int X = x + d.x, Y = y + d.y, Z = z + d.z;
    bool ok = wrap(X, G.nx, G.px) && wrap(Y, G.ny, G.py) && wrap(Z, G.nz, G.pz);
    if (ok && MASK) ok = !mask[X + (long long)G.nx * (Y + (long long)G.ny * Z)];
    if (!ok) b |= 1u << k;
  }
  return b;
}

template <typename S>
struct LightArgs {
  using R = typename Store<S>::R;
  const S* h;
  const S* g;
  const unsigned char* mask;
  const R* phi_writers;  // phase field of the writers of the populations read
  Geom geo;
  Codec<R> cd;
  R* phi_out;          // gather target (compute precision)
  double* out_h;       // natural-order FP64 populations
  double* out_g;
  double* out_phi64;   // FP64 phi
  double* partials;    // [nblocks][5]
};

enum LightMode { LM_GATHER = 0, LM_READ_POPS = 1, LM_REDUCE = 2 };

// phi gather (phi = sum h with the read rule of the next step), population
// readout, or per-block FP64 sums.
template <typename S, bool ODD, bool MASK, int LM>
__global__ __launch_bounds__(256) void k_light(LightArgs<S> a) {
  using R = typename Store<S>::R;
  const Geom& G = a.geo;
  const TileCoord t = tile_of_block(G);
  const int x = t.x0 + threadIdx.x, y = t.y0 + threadIdx.y, z = t.z;
  const bool in = x < G.nx && y < G.ny;
  double acc[5] = {0, 0, 0, 0, 0};
  if (in) {
    const long long idx = x + (long long)G.nx * (y + (long long)G.ny * z);
    const bool solid = MASK && a.mask[idx];
    if (solid) {
      if (LM == LM_GATHER) a.phi_out[idx] = R(0);
      if (LM == LM_READ_POPS) {
        for (int i = 0; i < Q_H; ++i) a.out_h[i * G.N + idx] = 0.0;
        for (int i = 0; i < Q_G; ++i) a.out_g[i * G.N + idx] = 0.0;
      }
    } else {
      const unsigned walls =
          (ODD || Store<S>::kShift) ? wall_bits_direct<MASK>(x, y, z, G, a.mask) : 0u;
      const Nbhd nb = make_nbhd(x, y, z, G);
      R phw[Q_H];
      if (Store<S>::kShift) writer_phi_direct(a.phi_writers, (unsigned)idx, nb, walls, phw);
      R h[Q_H], g[Q_G];
      if (LM == LM_GATHER) {
        using St = Store<S>;
        const unsigned NS = (unsigned)(G.N * (long long)sizeof(S));
#pragma unroll
        for (int i = 0; i < Q_H; ++i) {
          unsigned off = pair_off<S>(i, (unsigned)idx, NS);
          if (ODD && i) {
            const Dir d = ch(i);
            if (!(walls & (1u << nb27(-d.x, -d.y, -d.z))))
              off = pair_off<S>(opp(i), nb.at(-d.x, -d.y, -d.z), NS);
          }
          const S* p = reinterpret_cast<const S*>(pair_base(a.h, G.N, i) + off);
          h[i] = St::template ld<kNtGather>(p, St::kShift ? R(wh(i)) * phw[i] : R(0),
                                                  a.cd.inv_scale_h);
        }
        const R s = sum_h(h);
        a.phi_out[idx] = s;
        if (a.out_phi64) a.out_phi64[idx] = double(s);
      } else {
        load_pops<S, ODD>(a.h, a.g, G.N, (unsigned)idx, nb, walls, a.cd, phw, h, g);
        if (LM == LM_READ_POPS) {
#pragma unroll
          for (int i = 0; i < Q_H; ++i) a.out_h[i * G.N + idx] = double(h[i]);
#pragma unroll
          for (int i = 0; i < Q_G; ++i) a.out_g[i * G.N + idx] = double(g[i]);
        } else {
          double s = 0;
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

template <typename S>
struct InitArgs {
  using R = typename Store<S>::R;
  S* h;
  S* g;
  const unsigned char* mask;
  const double* phi0;
  const double* u0;      // may be null
  const double* p0;      // may be null
  const R* phi_ref;      // R(phi0): the phase field the FP16 shifts refer to
  Geom geo;
  Codec<R> cd;
};

// Equilibrium initialisation in the natural layout (the even-step read rule).
template <typename S, bool MASK>
__global__ __launch_bounds__(256) void k_init(InitArgs<S> a) {
  using R = typename Store<S>::R;
  using St = Store<S>;
  const Geom& G = a.geo;
  const TileCoord t = tile_of_block(G);
  const int x = t.x0 + threadIdx.x, y = t.y0 + threadIdx.y, z = t.z;
  if (x >= G.nx || y >= G.ny) return;
  const long long idx = x + (long long)G.nx * (y + (long long)G.ny * z);
  const bool solid = MASK && a.mask[idx];
  const R phi = solid ? R(0) : R(a.phi0[idx]);
  R ux = R(0), uy = R(0), uz = R(0), p = R(0);
  if (!solid && a.u0) { ux = R(a.u0[idx]); uy = R(a.u0[G.N + idx]); uz = R(a.u0[2 * G.N + idx]); }
  if (!solid && a.p0) p = R(a.p0[idx]);
  const R base = R(1) - R(1.5) * (ux * ux + uy * uy + uz * uz);
  // the natural layout is read with the even rule, whose writer of
  // population i is x - c_i (or x at a wall): shift by that cell's phi0
  R phw[Q_H];
  if (St::kShift && !solid) {
    const unsigned walls = wall_bits_direct<MASK>(x, y, z, G, a.mask);
    writer_phi_direct(a.phi_ref, (unsigned)idx, make_nbhd(x, y, z, G), walls, phw);
  }
#pragma unroll
  for (int i = 0; i < Q_H; ++i) {
    const R cu = dot(ch(i), ux, uy, uz);
    const R v = R(wh(i)) * phi * (base + cu * (R(3) + R(4.5) * cu));
    const R sh = (St::kShift && !solid) ? R(wh(i)) * phw[i] : R(0);
    St::st(a.h + (long long)i * G.N + idx, v, sh, a.cd.scale_h);
  }
  const R baseg = p - R(1.5) * (ux * ux + uy * uy + uz * uz);
#pragma unroll
  for (int i = 0; i < Q_G; ++i) {
    const R cu = dot(cg(i), ux, uy, uz);
    const R v = R(wg(i)) * (baseg + cu * (R(3) + R(4.5) * cu));
    St::st(a.g + (long long)i * G.N + idx, v, R(0), a.cd.scale_g);
  }
}

// FP64 phi0 -> compute precision (zero in solids)
template <typename R>
__global__ __launch_bounds__(256) void k_phi_from_f64(const double* __restrict__ in,
                                                       const unsigned char* __restrict__ mask,
                                                       long long N, R* __restrict__ out) {
  const long long i = blockIdx.x * 256ll + threadIdx.x;
  if (i < N) out[i] = (mask && mask[i]) ? R(0) : R(in[i]);
}

// phi (compute precision) -> FP64
template <typename R>
__global__ __launch_bounds__(256) void k_phi_to_f64(const R* __restrict__ phi, long long N,
                                                     double* __restrict__ out) {
  const long long i = blockIdx.x * 256ll + threadIdx.x;
  if (i < N) out[i] = double(phi[i]);
}

}  // namespace pflbm
