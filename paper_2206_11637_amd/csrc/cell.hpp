// Per-cell arithmetic of the coupled phase-field LBM step (registers only).
//
// Paper sec. "Conservative Allen-Cahn model" (arXiv:2206.11637):
//   phi = sum h_i (eq. zeroth_moment_phase); rho(phi), tau(phi) linear in phi;
//   counter-term 4 phi (1 - phi)/xi n (Guo forcing on the phase field);
//   p* = sum g_i (eq. zeroth_moment_hydro); F = F_s + F_b + F_p + F_mu with
//   F_s = mu_phi grad phi, F_b = rho g, F_p = -p* c_s^2 (rho_H - rho_L) grad phi
//   and F_mu from the non-equilibrium second moment of g (end of the LBE
//   section); incompressible equilibrium (eq. feq, rho_0 = 1); MRT (eq. mrt).
//
// MRT here is written in its projected form.  With one rate per polynomial
// degree of a weighted-orthogonal moment basis (s_lo for degree <= 2, s_hi
// above), M^-1 S M Delta = s_hi Delta + (s_lo - s_hi) P Delta, where P is the
// weighted projection onto quadratic polynomials of c:
//   (P Delta)_i = w_i [a0 + 3 c_i.a1 + 9/2 (c_i c_i - I/3) : A2],
//   a0 = sum Delta, a1 = sum c Delta, A2 = sum (c c - I/3) Delta.
// The moments of the equilibria are known in closed form (4th-order isotropic
// lattices), so a0 = 0, and a1, A2 follow from a handful of moments of the
// pre-collision populations instead of a q x q product.  BGK is s_hi = s_lo.
#pragma once
#include "lattice.hpp"

namespace pflbm {

template <typename R>
struct Phys {
  R tau_L, dtau;      // tau(phi) = tau_L + phi dtau
  R rho_L, drho;      // rho(phi) = rho_L + phi drho
  R theta_k;          // 4/xi (0 when xi = inf):  theta = theta_k phi (1 - phi)
  R beta4;            // 4 beta = 48 sigma / xi
  R kappa;            // 3 sigma xi / 2
  R gx, gy, gz;       // body acceleration
  R omega_phi;        // 1 / (3 M + 1/2)
  R s_high;           // rate of degree >= 3 moments (MRT)
  R eps2;             // eps^2: n = grad phi / sqrt(|grad phi|^2 + eps^2)
  R s_bulk;           // rate of the bulk mode of g (MRT); 0: the second-order rate
  R rho_gref;         // F_b = (rho - rho_gref) g
};

// second-moment tensor of a population set, symmetric storage xx yy zz xy xz yz
template <typename R>
struct Sym { R xx, yy, zz, xy, xz, yz; };

template <typename R>
__device__ __forceinline__ R sum_h(const R (&h)[Q_H]) {
  R s = h[0];
#pragma unroll
  for (int i = 1; i < Q_H; ++i) s += h[i];
  return s;
}

template <bool G27>
__device__ __forceinline__ constexpr Dir cdir(int i) { return G27 ? cg(i) : ch(i); }
template <bool G27>
__device__ __forceinline__ constexpr double wdir(int i) { return G27 ? wg(i) : wh(i); }

// First and second moments (sum c f, sum c c f) over opposite pairs: the
// library orders each pair as (i, i + 1) with c_{i+1} = -c_i for odd i, so
// a pair contributes its difference to odd moments and its sum to even ones.
template <typename R, bool G27, int Q>
__device__ __forceinline__ void pair_moments(const R (&f)[Q], R& mx, R& my, R& mz, Sym<R>& P) {
  mx = my = mz = R(0);
  P = Sym<R>{R(0), R(0), R(0), R(0), R(0), R(0)};
#pragma unroll
  for (int k = 1; k < Q; k += 2) {
    const Dir d = cdir<G27>(k);
    const R sm = f[k] + f[k + 1], df = f[k] - f[k + 1];
    if (d.x) { mx += d.x > 0 ? df : -df; P.xx += sm; }
    if (d.y) { my += d.y > 0 ? df : -df; P.yy += sm; }
    if (d.z) { mz += d.z > 0 ? df : -df; P.zz += sm; }
    if (d.x * d.y) P.xy += (d.x * d.y > 0) ? sm : -sm;
    if (d.x * d.z) P.xz += (d.x * d.z > 0) ? sm : -sm;
    if (d.y * d.z) P.yz += (d.y * d.z > 0) ? sm : -sm;
  }
}

// Shifted representation of the phase-field populations.  The collision
// works on deviations h'_i = h_i - w_i phi_ref from a per-cell reference
// (the cell's phase field one step earlier; zero for the FP64 form), so the
// rounding of every step acts on quantities of the size of the change instead
// of on h ~ w_i.  phi = phi_ref + sum_i h'_i.
template <typename R>
__device__ __forceinline__ R phi_of(const R (&hd)[Q_H], R phi_ref) {
  return phi_ref + sum_h(hd);
}

// Cell state after the force prologue (everything the collisions need).
template <typename R>
struct CellState {
  R phi, dphi;       // phi and phi - phi_ref
  R rho, omega, theta, nx, ny, nz;
  R p, jx, jy, jz;
  R ux, uy, uz;      // force-corrected velocity u = j + F/(2 rho)
  R Fx, Fy, Fz;      // total force
  Sym<R> Pi;         // sum c c g
};

// S1-S11: moments, chemical potential, forces and velocity of one cell.
// phi = phi_ref + dphi with dphi = sum of the h deviations (S1).
template <typename R>
__device__ __forceinline__ void prologue(R phi, R dphi, const R (&g)[Q_G], R Gx, R Gy, R Gz,
                                         R lap, const Phys<R>& P, CellState<R>& c) {
  c.phi = phi;
  c.dphi = dphi;
  c.rho = P.rho_L + phi * P.drho;
  const R tau = P.tau_L + phi * P.dtau;
  c.omega = R(1) / tau;
  c.theta = P.theta_k * phi * (R(1) - phi);
  const R ninv = R(1) / sqrt(Gx * Gx + Gy * Gy + Gz * Gz + P.eps2);
  c.nx = Gx * ninv;
  c.ny = Gy * ninv;
  c.nz = Gz * ninv;
  const R mu = P.beta4 * phi * (phi - R(1)) * (phi - R(0.5)) - P.kappa * lap;

  R p = g[0];
#pragma unroll
  for (int i = 1; i < Q_G; ++i) p += g[i];
  R jx, jy, jz;
  Sym<R> Pi;
  pair_moments<R, true, Q_G>(g, jx, jy, jz, Pi);
  c.p = p;
  c.jx = jx;
  c.jy = jy;
  c.jz = jz;
  c.Pi = Pi;

  // F_s + F_p share the direction grad phi; F_b = rho g
  const R cgrad = mu - p * (R(1) / R(3)) * P.drho;
  const R brho = c.rho - P.rho_gref;
  const R F0x = cgrad * Gx + brho * P.gx;
  const R F0y = cgrad * Gy + brho * P.gy;
  const R F0z = cgrad * Gz + brho * P.gz;
  const R inv2rho = R(0.5) / c.rho;
  const R u1x = jx + F0x * inv2rho;
  const R u1y = jy + F0y * inv2rho;
  const R u1z = jz + F0z * inv2rho;
  // Pi_neq with the equilibrium at u': sum c c g^eq(p*, u') = p*/3 I + u' u'^T
  const R p3 = p * (R(1) / R(3));
  const R nxx = Pi.xx - p3 - u1x * u1x;
  const R nyy = Pi.yy - p3 - u1y * u1y;
  const R nzz = Pi.zz - p3 - u1z * u1z;
  const R nxy = Pi.xy - u1x * u1y;
  const R nxz = Pi.xz - u1x * u1z;
  const R nyz = Pi.yz - u1y * u1z;
  const R fmu = -(R(1) - R(0.5) * c.omega) * P.drho;
  // with the bulk mode relaxed at s_bulk its non-equilibrium part carries the
  // trace of the strain rate scaled by 1/s_bulk instead of 1/omega
  const R kb = P.s_bulk > R(0) ? P.s_bulk * tau - R(1) : R(0);
  const R tb = kb * (nxx + nyy + nzz) * (R(1) / R(3));
  c.Fx = F0x + fmu * ((nxx + tb) * Gx + nxy * Gy + nxz * Gz);
  c.Fy = F0y + fmu * (nxy * Gx + (nyy + tb) * Gy + nyz * Gz);
  c.Fz = F0z + fmu * (nxz * Gx + nyz * Gy + (nzz + tb) * Gz);
  c.ux = jx + c.Fx * inv2rho;
  c.uy = jy + c.Fy * inv2rho;
  c.uz = jz + c.Fz * inv2rho;
}

template <typename R>
__device__ __forceinline__ R dot(Dir d, R x, R y, R z) {
  R r = R(0);
  if (d.x) r += d.x > 0 ? x : -x;
  if (d.y) r += d.y > 0 ? y : -y;
  if (d.z) r += d.z > 0 ? z : -z;
  return r;
}

// (c c - I/3) : A for symmetric A
template <typename R>
__device__ __forceinline__ R hermite2(Dir d, const Sym<R>& A) {
  R r = -(A.xx + A.yy + A.zz) * (R(1) / R(3));
  if (d.x) r += A.xx;
  if (d.y) r += A.yy;
  if (d.z) r += A.zz;
  if (d.x * d.y) r += (d.x * d.y > 0) ? R(2) * A.xy : -R(2) * A.xy;
  if (d.x * d.z) r += (d.x * d.z > 0) ? R(2) * A.xz : -R(2) * A.xz;
  if (d.y * d.z) r += (d.y * d.z > 0) ? R(2) * A.yz : -R(2) * A.yz;
  return r;
}

// d^T B d for a lattice direction d (components in {-1, 0, 1}) and symmetric
// B, with the off-diagonals passed doubled (t = 2 B_ab): a face picks one
// diagonal entry, an edge two plus one off-diagonal, a corner all six.
template <typename R>
__device__ __forceinline__ R quad(Dir d, const Sym<R>& B, R txy, R txz, R tyz) {
  R r = R(0);
  if (d.x) r += B.xx;
  if (d.y) r += B.yy;
  if (d.z) r += B.zz;
  if (d.x * d.y) r += (d.x * d.y > 0) ? txy : -txy;
  if (d.x * d.z) r += (d.x * d.z > 0) ? txz : -txz;
  if (d.y * d.z) r += (d.y * d.z > 0) ? tyz : -tyz;
  return r;
}

// One relaxation with projected MRT and Guo forcing, folded per opposite pair.
// With f^eq_i = w_i [e + 3 c.u' + 9/2 (c.u')^2 - 3/2 u'.u'] the post-collision
//   f*_i = f_i + s_hi (f^eq_i - f_i) + (s_lo - s_hi) (P Delta)_i + forcing_i
// splits into a part even in c,  w_i [e0 + 9/2 c^T B c]  with
//   B = s_hi u u^T + (s_lo - s_hi) A2,  e0 = s_hi e - 3/2 s_hi u.u - 3/2 (s_lo - s_hi) tr A2,
// and a part odd in c,  w_i c.V  with  V = 3 s_hi u + 3 (s_lo - s_hi) a1 + forcing vector,
// so f*_i = (1 - s_hi) f_i + even_i + odd_i and f*_{i+1} = (1 - s_hi) f_{i+1} + even_i - odd_i.
// (a1, A2: first and traceless-complete second moments of f^eq - f; BGK is
// s_lo = s_hi.)  Each pair costs a handful of operations instead of
// re-forming the equilibrium, the projection and the force term separately.
template <typename R, bool G27, int Q>
__device__ __forceinline__ void relax_pairs(R (&f)[Q], R shi, R e0, const Sym<R>& B, R Vx, R Vy,
                                            R Vz) {
  const R keep = R(1) - shi;
  const R txy = R(2) * B.xy, txz = R(2) * B.xz, tyz = R(2) * B.yz;
  {
    // rest population: c = 0
    f[0] = keep * f[0] + R(wdir<G27>(0)) * e0;
  }
#pragma unroll
  for (int k = 1; k < Q; k += 2) {
    const Dir d = cdir<G27>(k);
    const R w = R(wdir<G27>(k));
    const R ev = w * (e0 + R(4.5) * quad(d, B, txy, txz, tyz));
    const R od = w * dot(d, Vx, Vy, Vz);
    const R fi = f[k], fj = f[k + 1];
    f[k] = keep * fi + (ev + od);
    f[k + 1] = keep * fj + (ev - od);
  }
}

// S12-S13: hydrodynamic collision in place.  Equilibrium g^eq = w [p* + 3 c.u
// + 9/2 (c.u)^2 - 3/2 u.u]; moments of Delta = g^eq - g: a1 = u - j,
// A2 = p/3 I + u u - Pi; Guo source 3 w c.F / rho applied with (1 - omega/2).
// With s_bulk set, the trace part of the second-order relaxation uses it.
// GUO: Guo's full source, whose second-order part 4.5 w (c c - I/3):S / rho,
// S = u F^T + F u^T, is applied with (1 - omega/2) (its bulk part with
// (1 - s_bulk/2) when that rate is set).
template <typename R, bool MRT, bool GUO>
__device__ __forceinline__ void collide_g(R (&g)[Q_G], const CellState<R>& c, const Phys<R>& P) {
  const R uu = c.ux * c.ux + c.uy * c.uy + c.uz * c.uz;
  const R om = c.omega;
  const R shi = MRT ? P.s_high : om;
  const R dlo = om - shi;
  const R fk = (R(1) - R(0.5) * om) * R(3) / c.rho;   // Guo: (1 - om/2) 3 F / rho per w c.F
  Sym<R> B{shi * c.ux * c.ux, shi * c.uy * c.uy, shi * c.uz * c.uz,
           shi * c.ux * c.uy, shi * c.ux * c.uz, shi * c.uy * c.uz};
  R e0 = shi * (c.p - R(1.5) * uu);
  R Vx = R(3) * shi * c.ux + fk * c.Fx, Vy = R(3) * shi * c.uy + fk * c.Fy,
    Vz = R(3) * shi * c.uz + fk * c.Fz;
  if (MRT) {
    const R p3 = c.p * (R(1) / R(3));
    const Sym<R> A2{p3 + c.ux * c.ux - c.Pi.xx, p3 + c.uy * c.uy - c.Pi.yy, p3 + c.uz * c.uz - c.Pi.zz,
                    c.ux * c.uy - c.Pi.xy, c.ux * c.uz - c.Pi.xz, c.uy * c.uz - c.Pi.yz};
    // the bulk mode w (|c|^2 - 1) tr(A2)/3 relaxes at s_bulk instead of omega
    const R trA2 = A2.xx + A2.yy + A2.zz;
    const R db = P.s_bulk > R(0) ? (P.s_bulk - om) * trA2 * (R(1) / R(3)) : R(0);
    B.xx += dlo * A2.xx + db; B.yy += dlo * A2.yy + db; B.zz += dlo * A2.zz + db;
    B.xy += dlo * A2.xy; B.xz += dlo * A2.xz; B.yz += dlo * A2.yz;
    e0 -= R(1.5) * dlo * trA2 + R(4.5) * db;
    const R d3 = R(3) * dlo;
    Vx += d3 * (c.ux - c.jx);
    Vy += d3 * (c.uy - c.jy);
    Vz += d3 * (c.uz - c.jz);
  }
  if constexpr (GUO) {
    const R kf = (R(1) - R(0.5) * om) / c.rho;
    const R Sxx = R(2) * c.ux * c.Fx, Syy = R(2) * c.uy * c.Fy, Szz = R(2) * c.uz * c.Fz;
    const R trS = Sxx + Syy + Szz;
    const R kd = (MRT && P.s_bulk > R(0)) ? R(0.5) * (om - P.s_bulk) / c.rho * trS * (R(1) / R(3))
                                          : R(0);
    B.xx += kf * Sxx + kd; B.yy += kf * Syy + kd; B.zz += kf * Szz + kd;
    B.xy += kf * (c.ux * c.Fy + c.uy * c.Fx);
    B.xz += kf * (c.ux * c.Fz + c.uz * c.Fx);
    B.yz += kf * (c.uy * c.Fz + c.uz * c.Fy);
    e0 -= R(1.5) * kf * trS + R(4.5) * kd;
  }
  relax_pairs<R, true, Q_G>(g, shi, e0, B, Vx, Vy, Vz);
}

// S14-S15: phase-field collision in place on the deviations h' (needs u
// from the hydro prologue).  With the reference subtracted,
// h^eq_i - w_i phi_ref = w_i [dphi + phi (3 c.u + 9/2 (c.u)^2 - 3/2 u.u)], the
// moments of Delta are a1 = phi u - j and A2 = dphi/3 I + phi u u - Pi' (Pi'
// the second moment of h'), and the counter-term source w_i theta c.n is
// applied with (1 - omega_phi/2).
template <typename R, bool MRT>
__device__ __forceinline__ void collide_h(R (&h)[Q_H], const CellState<R>& c, const Phys<R>& P) {
  const R uu = c.ux * c.ux + c.uy * c.uy + c.uz * c.uz;
  const R om = P.omega_phi;
  const R shi = MRT ? P.s_high : om;
  const R dlo = om - shi;
  const R fk = (R(1) - R(0.5) * om) * c.theta;
  const R phi = c.phi;
  const R sp = shi * phi;
  Sym<R> B{sp * c.ux * c.ux, sp * c.uy * c.uy, sp * c.uz * c.uz,
           sp * c.ux * c.uy, sp * c.ux * c.uz, sp * c.uy * c.uz};
  R e0 = shi * (c.dphi - R(1.5) * phi * uu);
  R Vx = R(3) * sp * c.ux + fk * c.nx, Vy = R(3) * sp * c.uy + fk * c.ny,
    Vz = R(3) * sp * c.uz + fk * c.nz;
  if (MRT) {
    R jx, jy, jz;
    Sym<R> Pi;
    pair_moments<R, false, Q_H>(h, jx, jy, jz, Pi);
    const R p3 = c.dphi * (R(1) / R(3));
    const Sym<R> A2{p3 + phi * c.ux * c.ux - Pi.xx, p3 + phi * c.uy * c.uy - Pi.yy,
                    p3 + phi * c.uz * c.uz - Pi.zz, phi * c.ux * c.uy - Pi.xy,
                    phi * c.ux * c.uz - Pi.xz, phi * c.uy * c.uz - Pi.yz};
    B.xx += dlo * A2.xx; B.yy += dlo * A2.yy; B.zz += dlo * A2.zz;
    B.xy += dlo * A2.xy; B.xz += dlo * A2.xz; B.yz += dlo * A2.yz;
    e0 -= R(1.5) * dlo * (A2.xx + A2.yy + A2.zz);
    const R d3 = R(3) * dlo;
    Vx += d3 * (phi * c.ux - jx);
    Vy += d3 * (phi * c.uy - jy);
    Vz += d3 * (phi * c.uz - jz);
  }
  relax_pairs<R, false, Q_H>(h, shi, e0, B, Vx, Vy, Vz);
}

}  // namespace pflbm
