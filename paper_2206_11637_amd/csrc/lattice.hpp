// Velocity sets of the library (D3Q15 for the phase field, D3Q27 for the
// hydrodynamics) as compile-time tables.  Every loop over directions is fully
// unrolled, so c_i and w_i fold into immediates.  Built with
// PFLBM_PHASE_D3Q27 the phase field uses D3Q27 as well (the velocity set the
// paper uses for both lattices in 3D); that build is a separate library.
//
// Ordering: 0 = rest; 1..6 the faces +x,-x,+y,-y,+z,-z; D3Q27 then has the 12
// edges and both sets end with the 8 corners.  Opposite directions sit in
// adjacent pairs (odd i <-> i + 1), so opp(i) is a bit trick.
#pragma once

namespace pflbm {

#ifdef PFLBM_PHASE_D3Q27
constexpr int Q_H = 27;
#else
constexpr int Q_H = 15;
#endif
constexpr int Q_G = 27;

struct Dir { int x, y, z; };

constexpr Dir kC27[27] = {
    {0, 0, 0},
    {1, 0, 0}, {-1, 0, 0}, {0, 1, 0}, {0, -1, 0}, {0, 0, 1}, {0, 0, -1},
    {1, 1, 0}, {-1, -1, 0}, {1, -1, 0}, {-1, 1, 0},
    {1, 0, 1}, {-1, 0, -1}, {1, 0, -1}, {-1, 0, 1},
    {0, 1, 1}, {0, -1, -1}, {0, 1, -1}, {0, -1, 1},
    {1, 1, 1}, {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1},
    {1, -1, 1}, {-1, 1, -1}, {-1, 1, 1}, {1, -1, -1}};

// D3Q15 = rest, faces, corners of the table above
constexpr int kH2G[15] = {0, 1, 2, 3, 4, 5, 6, 19, 20, 21, 22, 23, 24, 25, 26};

__host__ __device__ constexpr int opp(int i) { return i == 0 ? 0 : ((i & 1) ? i + 1 : i - 1); }

__host__ __device__ constexpr Dir cg(int i) { return kC27[i]; }
#ifdef PFLBM_PHASE_D3Q27
__host__ __device__ constexpr Dir ch(int i) { return kC27[i]; }
#else
__host__ __device__ constexpr Dir ch(int i) { return kC27[kH2G[i]]; }
#endif

__host__ __device__ constexpr int norm2(Dir d) { return d.x * d.x + d.y * d.y + d.z * d.z; }

__host__ __device__ constexpr double wg(int i) {
  return norm2(cg(i)) == 0 ? 8.0 / 27.0
       : norm2(cg(i)) == 1 ? 2.0 / 27.0
       : norm2(cg(i)) == 2 ? 1.0 / 54.0 : 1.0 / 216.0;
}
#ifdef PFLBM_PHASE_D3Q27
__host__ __device__ constexpr double wh(int i) { return wg(i); }
#else
__host__ __device__ constexpr double wh(int i) {
  return norm2(ch(i)) == 0 ? 2.0 / 9.0 : norm2(ch(i)) == 1 ? 1.0 / 9.0 : 1.0 / 72.0;
}
#endif

// index of direction (dx,dy,dz) in kC27 (the 3x3x3 neighbourhood), via a
// table built at compile time
struct NbTable { int v[27]; };
constexpr NbTable make_nb_table() {
  NbTable t{};
  for (int i = 0; i < 27; ++i)
    t.v[(kC27[i].x + 1) + 3 * (kC27[i].y + 1) + 9 * (kC27[i].z + 1)] = i;
  return t;
}
constexpr NbTable kNb = make_nb_table();
__host__ __device__ constexpr int nb27(int dx, int dy, int dz) {
  return kNb.v[(dx + 1) + 3 * (dy + 1) + 9 * (dz + 1)];
}

static_assert(opp(1) == 2 && opp(2) == 1 && opp(26) == 25, "pairs");
static_assert(kC27[opp(7)].x == -kC27[7].x && kC27[opp(7)].y == -kC27[7].y, "opp");
static_assert(nb27(1, -1, 1) == 23 && nb27(0, 0, 0) == 0, "neighbour table");

}  // namespace pflbm
