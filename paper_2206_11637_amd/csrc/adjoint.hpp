// Reverse mode of the coupled phase-field LBM step.
//
// One forward step maps the post-streaming state (h^n, g^n) to (h^{n+1},
// g^{n+1}); the phase field phi^n = sum_i h_i^n enters each cell twice: through
// the cell's own phi (density, relaxation time, counter-term, chemical
// potential, equilibria) and through the grad/lap stencils of its neighbours.
// The adjoint of a time level is therefore kept as
//     Lambda_h,i(x) = lam_h,i(x) + a_phi(x),   Lambda_g,i(x) = lam_g,i(x)
// where lam are the per-cell parts and a_phi the stencil part (dL/dphi^n
// through neighbours' stencils plus any loss sensitivity to phi^n).
//
// Reverse step n+1 -> n (two kernels, no atomics, deterministic):
//   k_adj_cell   pull the post-collision adjoints through the transposed
//                streaming (Lambda of the slot each f*_i(x) was streamed to:
//                (i, x + c_i), or (opp i, x) after a bounce-back), recompute
//                the forward cell arithmetic from the saved primal state, and
//                apply its vector-Jacobian product; writes lam^n, the stencil
//                adjoints s(x) = (dL/d grad phi, dL/d lap phi) and FP64 block
//                sums of dL/domega_phi, dL/dsigma and dL/dxi.
//   k_adj_stencil  (z-marching like the forward step)
//                a_phi^n(y) = sum over valid neighbours m of
//                -3 w_m c_m . (s_G(y + c_m) + s_G(y)) + 6 w_m (s_L(y + c_m) - s_L(y)),
//                the transpose of grad phi = 3 sum w c (phi_m - phi) and
//                lap phi = 6 sum w (phi_m - phi) with the wall rule.
#pragma once
#include "kernels.hpp"

namespace pflbm {

// the four stencil adjoints of one cell, stored together (one 16- or 32-byte
// access per cell)
template <typename R>
struct alignas(4 * sizeof(R)) S4 { R gx, gy, gz, l; };

template <typename R>
struct AdjConst {
  R beta4_per_sigma;   // 48 / xi  (0 if xi = inf)
  R kappa_per_sigma;   // 3 xi / 2 (0 if xi = inf)
  R inv_xi;            // 1 / xi   (0 if xi = inf)
};

// d(H_i : A)/dA for the symmetric storage xx yy zz xy xz yz (off-diagonals
// appear twice in the full contraction)
template <typename R>
__device__ __forceinline__ void hermite2_grad(Dir d, R coef, Sym<R>& acc) {
  const R t = -coef * (R(1) / R(3));
  acc.xx += t + (d.x ? coef : R(0));
  acc.yy += t + (d.y ? coef : R(0));
  acc.zz += t + (d.z ? coef : R(0));
  if (d.x * d.y) acc.xy += (d.x * d.y > 0) ? R(2) * coef : -R(2) * coef;
  if (d.x * d.z) acc.xz += (d.x * d.z > 0) ? R(2) * coef : -R(2) * coef;
  if (d.y * d.z) acc.yz += (d.y * d.z > 0) ? R(2) * coef : -R(2) * coef;
}

// sum_c lamPi_c (c c)_c for one direction (the transpose of Pi = sum c c f)
template <typename R>
__device__ __forceinline__ R second_moment_t(Dir d, const Sym<R>& L) {
  R r = R(0);
  if (d.x) r += L.xx;
  if (d.y) r += L.yy;
  if (d.z) r += L.zz;
  if (d.x * d.y) r += (d.x * d.y > 0) ? L.xy : -L.xy;
  if (d.x * d.z) r += (d.x * d.z > 0) ? L.xz : -L.xz;
  if (d.y * d.z) r += (d.y * d.z > 0) ? L.yz : -L.yz;
  return r;
}

// Vector-Jacobian product of one cell's collision (S1-S15).  lh, lg: in =
// adjoints of the post-collision populations, out = adjoints of the
// pre-collision ones (the cell-local part).  Outputs the adjoints of the
// stencil inputs (grad phi, lap phi) and of omega_phi, sigma and xi (xi enters
// through theta = 4 phi (1 - phi)/xi, beta = 12 sigma/xi and kappa = 3 sigma
// xi/2, so dtheta/dxi = -theta/xi and dmu/dxi = -(4 beta p3c + kappa lap)/xi
// with p3c = phi (phi - 1)(phi - 1/2)).  BULK: the
// bulk mode of g relaxes at P.s_bulk (MRT only); GUO: Guo's full source.
template <typename R, bool MRT, bool BULK, bool GUO, typename LoadL>
__device__ __forceinline__ void cell_vjp(const R (&h)[Q_H], const R (&g)[Q_G], R Gx, R Gy, R Gz,
                                         R lap, const Phys<R>& P, const AdjConst<R>& K,
                                         R (&lh)[Q_H], R (&lg)[Q_G], LoadL&& load_l, R& lGx, R& lGy,
                                         R& lGz, R& lL, R& l_omphi, R& l_sigma, R& l_xi) {
  // ---------------- forward recomputation ----------------
  const R phi = sum_h(h);
  const R rho = P.rho_L + phi * P.drho;
  const R tau = P.tau_L + phi * P.dtau;
  const R om = R(1) / tau;
  const R theta = P.theta_k * phi * (R(1) - phi);
  const R rn = R(1) / sqrt(Gx * Gx + Gy * Gy + Gz * Gz + P.eps2);
  const R nx = Gx * rn, ny = Gy * rn, nz = Gz * rn;
  const R p3c = phi * (phi - R(1)) * (phi - R(0.5));
  const R mu = P.beta4 * p3c - P.kappa * lap;
  R p = g[0];
#pragma unroll
  for (int i = 1; i < Q_G; ++i) p += g[i];
  R jx, jy, jz;
  Sym<R> Pi;
  pair_moments<R, true, Q_G>(g, jx, jy, jz, Pi);
  const R third = R(1) / R(3);
  const R cgr = mu - p * third * P.drho;
  const R brho = rho - P.rho_gref;
  const R F0x = cgr * Gx + brho * P.gx, F0y = cgr * Gy + brho * P.gy, F0z = cgr * Gz + brho * P.gz;
  const R i2 = R(0.5) / rho;
  const R u1x = jx + F0x * i2, u1y = jy + F0y * i2, u1z = jz + F0z * i2;
  const R p3 = p * third;
  const Sym<R> Nq{Pi.xx - p3 - u1x * u1x, Pi.yy - p3 - u1y * u1y, Pi.zz - p3 - u1z * u1z,
                  Pi.xy - u1x * u1y, Pi.xz - u1x * u1z, Pi.yz - u1y * u1z};
  const R fm = -(R(1) - R(0.5) * om) * P.drho;
  R NGx, NGy, NGz;
  R kb = R(0), trN = R(0), tb = R(0);
  if constexpr (BULK) {   // the trace of N enters F_mu scaled by s_bulk tau
    kb = P.s_bulk * tau - R(1);
    trN = Nq.xx + Nq.yy + Nq.zz;
    tb = kb * trN * third;
    NGx = (Nq.xx + tb) * Gx + Nq.xy * Gy + Nq.xz * Gz;
    NGy = Nq.xy * Gx + (Nq.yy + tb) * Gy + Nq.yz * Gz;
    NGz = Nq.xz * Gx + Nq.yz * Gy + (Nq.zz + tb) * Gz;
  } else {
    NGx = Nq.xx * Gx + Nq.xy * Gy + Nq.xz * Gz;
    NGy = Nq.xy * Gx + Nq.yy * Gy + Nq.yz * Gz;
    NGz = Nq.xz * Gx + Nq.yz * Gy + Nq.zz * Gz;
  }
  const R Fx = F0x + fm * NGx, Fy = F0y + fm * NGy, Fz = F0z + fm * NGz;
  const R ux = jx + Fx * i2, uy = jy + Fy * i2, uz = jz + Fz * i2;
  const R uu = ux * ux + uy * uy + uz * uz;

  // ---------------- phase-field collision, reverse ----------------
  load_l(lh, 0);
  const R omp = P.omega_phi;
  const R fkh = (R(1) - R(0.5) * omp) * theta;
  const R sh = MRT ? P.s_high : omp;
  const R dloh = omp - sh;
  R a1hx = R(0), a1hy = R(0), a1hz = R(0);
  Sym<R> A2h{R(0), R(0), R(0), R(0), R(0), R(0)};
  if (MRT) {
    R hx, hy, hz;
    Sym<R> Ph;
    pair_moments<R, false, Q_H>(h, hx, hy, hz, Ph);
    a1hx = phi * ux - hx;
    a1hy = phi * uy - hy;
    a1hz = phi * uz - hz;
    const R pp3 = phi * third;
    A2h = Sym<R>{pp3 + phi * ux * ux - Ph.xx, pp3 + phi * uy * uy - Ph.yy, pp3 + phi * uz * uz - Ph.zz,
                 phi * ux * uy - Ph.xy, phi * ux * uz - Ph.xz, phi * uy * uz - Ph.yz};
  }
  const R hbase = R(1) - R(1.5) * uu;
  R l_phi = R(0), l_hbase = R(0), l_fkh = R(0);
  R lux = R(0), luy = R(0), luz = R(0);
  R lnx = R(0), lny = R(0), lnz = R(0);
  R la1hx = R(0), la1hy = R(0), la1hz = R(0);
  Sym<R> lA2h{R(0), R(0), R(0), R(0), R(0), R(0)};
  R lomp = R(0);
  {  // rest population: c = 0
    const R w = R(wh(0));
    const R lam = lh[0];
    l_phi += sh * lam * w * hbase;
    l_hbase += sh * lam * w * phi;
    if (MRT) {
      hermite2_grad(ch(0), R(4.5) * dloh * lam * w, lA2h);
      lomp += lam * w * R(4.5) * hermite2(ch(0), A2h);
    } else {
      lomp += lam * (w * phi * hbase - h[0]);
    }
  }
  // opposite pairs (k, k+1): sp/sm are the sum/difference of their adjoints,
  // E/O the parts of the equilibrium polynomial even/odd in c
#pragma unroll
  for (int k = 1; k < Q_H; k += 2) {
    const Dir d = ch(k);
    const R w = R(wh(k));
    const R la = lh[k], lb = lh[k + 1];
    const R sp = la + lb, sm = la - lb;
    const R cu = dot(d, ux, uy, uz);
    const R E = hbase + R(4.5) * cu * cu, O = R(3) * cu;
    const R cn = dot(d, nx, ny, nz);
    l_phi += sh * w * (sp * E + sm * O);
    l_hbase += sh * w * phi * sp;
    const R lcu = sh * w * phi * (R(3) * sm + R(9) * cu * sp);
    if (d.x) lux += d.x > 0 ? lcu : -lcu;
    if (d.y) luy += d.y > 0 ? lcu : -lcu;
    if (d.z) luz += d.z > 0 ? lcu : -lcu;
    l_fkh += w * cn * sm;
    const R ln = w * fkh * sm;
    if (d.x) lnx += d.x > 0 ? ln : -ln;
    if (d.y) lny += d.y > 0 ? ln : -ln;
    if (d.z) lnz += d.z > 0 ? ln : -ln;
    if (MRT) {
      const R PO = w * R(3) * dot(d, a1hx, a1hy, a1hz);
      const R PE = w * R(4.5) * hermite2(d, A2h);
      const R l3 = R(3) * dloh * w * sm;
      if (d.x) la1hx += d.x > 0 ? l3 : -l3;
      if (d.y) la1hy += d.y > 0 ? l3 : -l3;
      if (d.z) la1hz += d.z > 0 ? l3 : -l3;
      hermite2_grad(d, R(4.5) * dloh * w * sp, lA2h);
      lomp += sp * PE + sm * PO;
    } else {
      lomp += la * (w * phi * (E + O) - h[k]) + lb * (w * phi * (E - O) - h[k + 1]);
    }
    lomp -= R(0.5) * theta * w * cn * sm;
  }
  const R l_theta = (R(1) - R(0.5) * omp) * l_fkh;
  R lhjx = R(0), lhjy = R(0), lhjz = R(0);
  Sym<R> lPh{R(0), R(0), R(0), R(0), R(0), R(0)};
  if (MRT) {
    l_phi += la1hx * ux + la1hy * uy + la1hz * uz + (lA2h.xx + lA2h.yy + lA2h.zz) * third +
             lA2h.xx * ux * ux + lA2h.yy * uy * uy + lA2h.zz * uz * uz + lA2h.xy * ux * uy +
             lA2h.xz * ux * uz + lA2h.yz * uy * uz;
    lux += phi * (la1hx + R(2) * lA2h.xx * ux + lA2h.xy * uy + lA2h.xz * uz);
    luy += phi * (la1hy + R(2) * lA2h.yy * uy + lA2h.xy * ux + lA2h.yz * uz);
    luz += phi * (la1hz + R(2) * lA2h.zz * uz + lA2h.xz * ux + lA2h.yz * uy);
    lhjx = -la1hx;
    lhjy = -la1hy;
    lhjz = -la1hz;
    lPh = Sym<R>{-lA2h.xx, -lA2h.yy, -lA2h.zz, -lA2h.xy, -lA2h.xz, -lA2h.yz};
  }
  R l_uu = -R(1.5) * l_hbase;

  // ---------------- hydrodynamic collision, reverse ----------------
  load_l(lg, 1);
  const R fk = (R(1) - R(0.5) * om) * R(3) / rho;
  const R base = p - R(1.5) * uu;
  const R s = MRT ? P.s_high : om;
  const R dlo = om - s;
  const R a1x = ux - jx, a1y = uy - jy, a1z = uz - jz;
  const Sym<R> A2{p3 + ux * ux - Pi.xx, p3 + uy * uy - Pi.yy, p3 + uz * uz - Pi.zz,
                  ux * uy - Pi.xy, ux * uz - Pi.xz, uy * uz - Pi.yz};
  R l_base = R(0), l_fk = R(0), lFx = R(0), lFy = R(0), lFz = R(0), lom = R(0);
  R la1x = R(0), la1y = R(0), la1z = R(0);
  Sym<R> lA2{R(0), R(0), R(0), R(0), R(0), R(0)};
  R Lb = R(0);   // sum_i lambda_i w_i (|c_i|^2 - 1): adjoint of the bulk-mode term
  Sym<R> LG2{R(0), R(0), R(0), R(0), R(0), R(0)};   // d/dS of sum_i lambda_i 4.5 w_i H2(c_i):S
  {  // rest population
    const R w = R(wg(0));
    const R lam = lg[0];
    l_base += s * lam * w;
    if constexpr (BULK) Lb -= lam * w;
    if constexpr (GUO) hermite2_grad(cg(0), R(4.5) * lam * w, LG2);
    if (MRT) {
      hermite2_grad(cg(0), R(4.5) * dlo * lam * w, lA2);
      lom += lam * w * R(4.5) * hermite2(cg(0), A2);
    } else {
      lom += lam * (w * base - g[0]);
    }
  }
#pragma unroll
  for (int k = 1; k < Q_G; k += 2) {
    const Dir d = cg(k);
    const R w = R(wg(k));
    const R la = lg[k], lb = lg[k + 1];
    const R sp = la + lb, sm = la - lb;
    const R cu = dot(d, ux, uy, uz);
    l_base += s * w * sp;
    if constexpr (BULK) Lb += R(d.x * d.x + d.y * d.y + d.z * d.z - 1) * w * sp;
    if constexpr (GUO) hermite2_grad(d, R(4.5) * w * sp, LG2);
    const R lcu = s * w * (R(3) * sm + R(9) * cu * sp);
    if (d.x) lux += d.x > 0 ? lcu : -lcu;
    if (d.y) luy += d.y > 0 ? lcu : -lcu;
    if (d.z) luz += d.z > 0 ? lcu : -lcu;
    l_fk += w * dot(d, Fx, Fy, Fz) * sm;
    const R lf = w * fk * sm;
    if (d.x) lFx += d.x > 0 ? lf : -lf;
    if (d.y) lFy += d.y > 0 ? lf : -lf;
    if (d.z) lFz += d.z > 0 ? lf : -lf;
    if (MRT) {
      const R PO = w * R(3) * dot(d, a1x, a1y, a1z);
      const R PE = w * R(4.5) * hermite2(d, A2);
      const R l3 = R(3) * dlo * w * sm;
      if (d.x) la1x += d.x > 0 ? l3 : -l3;
      if (d.y) la1y += d.y > 0 ? l3 : -l3;
      if (d.z) la1z += d.z > 0 ? l3 : -l3;
      hermite2_grad(d, R(4.5) * dlo * w * sp, lA2);
      lom += sp * PE + sm * PO;
    } else {
      const R E = base + R(4.5) * cu * cu, O = R(3) * cu;
      lom += la * (w * (E + O) - g[k]) + lb * (w * (E - O) - g[k + 1]);
    }
  }
  if constexpr (MRT && BULK) {
    // g*_i += 4.5 w_i (|c_i|^2 - 1) db, db = (s_bulk - omega) tr(A2) / 3
    const R trA2 = A2.xx + A2.yy + A2.zz;
    const R l_db = R(4.5) * Lb;
    lom -= l_db * trA2 * third;
    const R ltr = l_db * (P.s_bulk - om) * third;
    lA2.xx += ltr; lA2.yy += ltr; lA2.zz += ltr;
  }
  lom += l_fk * (-R(1.5) / rho);
  R l_rho = -l_fk * fk / rho;
  if constexpr (GUO) {
    // g*_i += 4.5 w_i kf H2(c_i):S, kf = (1 - omega/2)/rho, S = u F^T + F u^T
    const R kf = (R(1) - R(0.5) * om) / rho;
    const R Sxx = R(2) * ux * Fx, Syy = R(2) * uy * Fy, Szz = R(2) * uz * Fz;
    const R Sxy = ux * Fy + uy * Fx, Sxz = ux * Fz + uz * Fx, Syz = uy * Fz + uz * Fy;
    const R LS = LG2.xx * Sxx + LG2.yy * Syy + LG2.zz * Szz + LG2.xy * Sxy + LG2.xz * Sxz +
                 LG2.yz * Syz;
    lom -= LS / (R(2) * rho);
    l_rho -= LS * kf / rho;
    lux += kf * (R(2) * LG2.xx * Fx + LG2.xy * Fy + LG2.xz * Fz);
    luy += kf * (LG2.xy * Fx + R(2) * LG2.yy * Fy + LG2.yz * Fz);
    luz += kf * (LG2.xz * Fx + LG2.yz * Fy + R(2) * LG2.zz * Fz);
    lFx += kf * (R(2) * LG2.xx * ux + LG2.xy * uy + LG2.xz * uz);
    lFy += kf * (LG2.xy * ux + R(2) * LG2.yy * uy + LG2.yz * uz);
    lFz += kf * (LG2.xz * ux + LG2.yz * uy + R(2) * LG2.zz * uz);
    if constexpr (MRT && BULK) {
      // its trace with (1 - s_bulk/2): g*_i += 4.5 w_i (|c_i|^2 - 1) kd,
      // kd = (omega - s_bulk) tr(S) / (6 rho), tr(S) = 2 u.F
      const R trS = Sxx + Syy + Szz;
      const R kd = (om - P.s_bulk) * trS / (R(6) * rho);
      const R l_kd = R(4.5) * Lb;
      lom += l_kd * trS / (R(6) * rho);
      l_rho -= l_kd * kd / rho;
      const R ltr = R(2) * l_kd * (om - P.s_bulk) / (R(6) * rho);
      lux += ltr * Fx; luy += ltr * Fy; luz += ltr * Fz;
      lFx += ltr * ux; lFy += ltr * uy; lFz += ltr * uz;
    }
  }
  R l_p = l_base;
  l_uu += -R(1.5) * l_base;
  R ljx = R(0), ljy = R(0), ljz = R(0);
  Sym<R> lPi{R(0), R(0), R(0), R(0), R(0), R(0)};
  if (MRT) {
    lux += la1x + R(2) * lA2.xx * ux + lA2.xy * uy + lA2.xz * uz;
    luy += la1y + R(2) * lA2.yy * uy + lA2.xy * ux + lA2.yz * uz;
    luz += la1z + R(2) * lA2.zz * uz + lA2.xz * ux + lA2.yz * uy;
    ljx -= la1x;
    ljy -= la1y;
    ljz -= la1z;
    l_p += (lA2.xx + lA2.yy + lA2.zz) * third;
    lPi = Sym<R>{-lA2.xx, -lA2.yy, -lA2.zz, -lA2.xy, -lA2.xz, -lA2.yz};
  }
  lux += R(2) * ux * l_uu;
  luy += R(2) * uy * l_uu;
  luz += R(2) * uz * l_uu;

  // ---------------- force prologue, reverse ----------------
  // u = j + F i2
  ljx += lux; ljy += luy; ljz += luz;
  lFx += lux * i2; lFy += luy * i2; lFz += luz * i2;
  R l_i2 = lux * Fx + luy * Fy + luz * Fz;
  // F = F0 + fm N G
  R lF0x = lFx, lF0y = lFy, lF0z = lFz;
  const R l_fm = lFx * NGx + lFy * NGy + lFz * NGz;
  Sym<R> lN{fm * lFx * Gx, fm * lFy * Gy, fm * lFz * Gz, fm * (lFx * Gy + lFy * Gx),
            fm * (lFx * Gz + lFz * Gx), fm * (lFy * Gz + lFz * Gy)};
  lGx = fm * (Nq.xx * lFx + Nq.xy * lFy + Nq.xz * lFz);
  lGy = fm * (Nq.xy * lFx + Nq.yy * lFy + Nq.yz * lFz);
  lGz = fm * (Nq.xz * lFx + Nq.yz * lFy + Nq.zz * lFz);
  lom += R(0.5) * P.drho * l_fm;
  R l_tau = R(0);
  if constexpr (BULK) {   // tb = (s_bulk tau - 1) tr(N) / 3
    lGx += fm * tb * lFx;
    lGy += fm * tb * lFy;
    lGz += fm * tb * lFz;
    const R l_tb = fm * (lFx * Gx + lFy * Gy + lFz * Gz);
    const R ltrN = l_tb * kb * third;
    lN.xx += ltrN; lN.yy += ltrN; lN.zz += ltrN;
    l_tau = l_tb * trN * third * P.s_bulk;
  }
  // N = Pi - p/3 I - u1 u1^T
  lPi.xx += lN.xx; lPi.yy += lN.yy; lPi.zz += lN.zz;
  lPi.xy += lN.xy; lPi.xz += lN.xz; lPi.yz += lN.yz;
  l_p -= (lN.xx + lN.yy + lN.zz) * third;
  const R lu1x = -(R(2) * lN.xx * u1x + lN.xy * u1y + lN.xz * u1z);
  const R lu1y = -(R(2) * lN.yy * u1y + lN.xy * u1x + lN.yz * u1z);
  const R lu1z = -(R(2) * lN.zz * u1z + lN.xz * u1x + lN.yz * u1y);
  // u1 = j + F0 i2
  ljx += lu1x; ljy += lu1y; ljz += lu1z;
  lF0x += lu1x * i2; lF0y += lu1y * i2; lF0z += lu1z * i2;
  l_i2 += lu1x * F0x + lu1y * F0y + lu1z * F0z;
  // i2 = 1/(2 rho)
  l_rho += -l_i2 * i2 / rho;
  // F0 = cgr G + rho g
  const R l_cgr = lF0x * Gx + lF0y * Gy + lF0z * Gz;
  lGx += cgr * lF0x; lGy += cgr * lF0y; lGz += cgr * lF0z;
  l_rho += lF0x * P.gx + lF0y * P.gy + lF0z * P.gz;
  // cgr = mu - p drho / 3
  const R l_mu = l_cgr;
  l_p -= P.drho * third * l_cgr;
  // mu = beta4 p3c(phi) - kappa lap
  l_phi += l_mu * P.beta4 * (R(3) * phi * phi - R(3) * phi + R(0.5));
  lL = -P.kappa * l_mu;
  l_sigma = l_mu * (K.beta4_per_sigma * p3c - K.kappa_per_sigma * lap);
  l_xi = -K.inv_xi * (l_theta * theta + l_mu * (P.beta4 * p3c + P.kappa * lap));
  // n = G rn
  const R Gln = Gx * lnx + Gy * lny + Gz * lnz;
  const R rn3 = rn * rn * rn;
  lGx += rn * lnx - rn3 * Gln * Gx;
  lGy += rn * lny - rn3 * Gln * Gy;
  lGz += rn * lnz - rn3 * Gln * Gz;
  // theta, omega, rho of phi
  l_phi += l_theta * P.theta_k * (R(1) - R(2) * phi);
  l_phi += (l_tau - lom * om * om) * P.dtau;
  l_phi += l_rho * P.drho;
  l_omphi = lomp;

  // ---------------- adjoints of the pre-collision populations ----------------
  lg[0] = (R(1) - s) * lg[0] + l_p;
#pragma unroll
  for (int k = 1; k < Q_G; k += 2) {
    const Dir d = cg(k);
    const R ev = l_p + second_moment_t(d, lPi), od = dot(d, ljx, ljy, ljz);
    lg[k] = (R(1) - s) * lg[k] + ev + od;
    lg[k + 1] = (R(1) - s) * lg[k + 1] + ev - od;
  }
  lh[0] = (R(1) - sh) * lh[0] + l_phi;
#pragma unroll
  for (int k = 1; k < Q_H; k += 2) {
    const Dir d = ch(k);
    R ev = l_phi, od = R(0);
    if (MRT) {
      ev += second_moment_t(d, lPh);
      od = dot(d, lhjx, lhjy, lhjz);
    }
    lh[k] = (R(1) - sh) * lh[k] + ev + od;
    lh[k + 1] = (R(1) - sh) * lh[k + 1] + ev - od;
  }
}

template <typename S>
struct AdjArgs {
  using R = typename Store<S>::R;
  // primal state of level n (a saved state: populations in the layout of the
  // streaming scheme, then phi^n and, for FP16 storage, phi^{n-1})
  const S* ph;
  const S* pg;
  const R* pphi;
  const R* pphi_prev;   // phi^{n-1}: shift reference of the level-n populations (shifted forms)
  const unsigned char* mask;
  // adjoint of level n+1 (natural layout) and of level n
  const R* lh_in;
  const R* lg_in;
  const R* aphi_in;
  R* lh_out;
  R* lg_out;
  S4<R>* sadj;      // [N]: dL/d(grad phi x, y, z), dL/d(lap phi)
  double* gsum;     // [nblocks][3] running sums of dL/domega_phi, dL/dsigma, dL/dxi
  Geom geo;
  Phys<R> P;
  AdjConst<R> K;
  Codec<R> cd;
};

// Occupancy request of the reverse cell kernel (FP32 arithmetic): 3 waves
// per SIMD.  With the Lambda loads issued where they are first needed, the
// FP16-storage MRT kernels fit its 168 VGPRs (the masked one, the Taylor
// tube's, without a spill) and the FP32 ones spill about 4; measured: the
// tube's reverse pass 3.41 s per 1000 steps against 3.75 s at 2 waves with
// the earlier load order, the 2000-step capillary rollout 64 x 128 x 64 in
// FP32 0.239 s against 0.252 s at 2 waves.  Before the load order changed, 3
// waves spilled 15-40 VGPRs and lost (0.277 s on the capillary rollout).
#ifndef PFLBM_ADJ_WAVES
#define PFLBM_ADJ_WAVES 3
#endif
#ifndef PFLBM_ADJ_F16_WAVES
#define PFLBM_ADJ_F16_WAVES PFLBM_ADJ_WAVES
#endif
template <typename S>
struct AdjWaves {
  static constexpr int value = sizeof(S) == 8 ? 1 : (sizeof(S) == 2 ? PFLBM_ADJ_F16_WAVES : PFLBM_ADJ_WAVES);
};

template <typename S, bool MRT, int RULE, bool MASK, bool BULK, bool GUO>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(AdjWaves<S>::value)))
void k_adj_cell(AdjArgs<S> a) {
  using St = Store<S>;
  using R = typename St::R;
  extern __shared__ unsigned char smem_raw[];
  R* tile = reinterpret_cast<R*>(smem_raw);
  __shared__ double red[4][3];
  const Geom& G = a.geo;
  const int TX = G.bx + 2, TY = G.by + 2;
  const TileCoord t = tile_of_block(G);
  load_phi_tile<R, MASK>(tile, a.pphi, a.mask, G, t);
  __syncthreads();
  const int lx = threadIdx.x, ly = threadIdx.y;
  const int x = t.x0 + lx, y = t.y0 + ly, z = t.z;
  double acc0 = 0.0, acc1 = 0.0, acc2 = 0.0;
  if (x < G.nx && y < G.ny && tile[(TY + ly + 1) * TX + lx + 1] != sentinel<R>()) {
    const unsigned idx = x + (unsigned)G.nx * (y + (unsigned)G.ny * z);
    const unsigned walls = wall_bits(tile, TX, TY, lx, ly);
    const Nbhd nb = make_nbhd(x, y, z, G);
    // primal populations of level n, absolute (h_i = h'_i + w_i phi_ref)
    R h[Q_H], g[Q_G];
    load_h<S, RULE, false>(a.ph, G.N, idx, nb, walls, a.cd.inv_scale_h, h);
    load_g<S, RULE, false>(a.pg, G.N, idx, nb, walls, a.cd.inv_scale_g, g);
    if (St::kShift) {
      const R ref = a.pphi_prev[idx];
#pragma unroll
      for (int i = 0; i < Q_H; ++i) h[i] += R(wh(i)) * ref;
    }
    R Gx, Gy, Gz, lap;
    stencil(tile, TX, TY, lx, ly, Gx, Gy, Gz, lap);
    // transposed streaming: Lambda of the slot each post-collision value went to
    R lh[Q_H], lg[Q_G];
    const unsigned NS = (unsigned)(G.N * (long long)sizeof(R));
    // the Lambda loads are issued where the reverse step first needs them
    // (lh before the phase-field part, lg before the hydrodynamic part), so
    // neither array is held in registers through the other part
    auto load_l = [&](auto& l, int which) {
      if (which == 0) {
#pragma unroll
        for (int i = 0; i < Q_H; ++i) {
          const Dir d = ch(i);
          unsigned cell = idx;
          unsigned off = pair_off<R>(opp(i), idx, NS);
          if (i && !(walls & (1u << nb27(d.x, d.y, d.z)))) {
            cell = nb.at(d.x, d.y, d.z);
            off = pair_off<R>(i, cell, NS);
          }
          l[i] = *reinterpret_cast<const R*>(pair_base(a.lh_in, G.N, i) + off) + a.aphi_in[cell];
        }
      } else {
#pragma unroll
        for (int i = 0; i < Q_G; ++i) {
          const Dir d = cg(i);
          unsigned off = pair_off<R>(opp(i), idx, NS);
          if (i && !(walls & (1u << nb27(d.x, d.y, d.z)))) off = pair_off<R>(i, nb.at(d.x, d.y, d.z), NS);
          l[i] = *reinterpret_cast<const R*>(pair_base(a.lg_in, G.N, i) + off);
        }
      }
    };
    R lGx, lGy, lGz, lL, lomp, lsig, lxi;
    cell_vjp<R, MRT, BULK, GUO>(h, g, Gx, Gy, Gz, lap, a.P, a.K, lh, lg, load_l, lGx, lGy, lGz, lL,
                                lomp, lsig, lxi);
#pragma unroll
    for (int i = 0; i < Q_H; ++i) *slot(a.lh_out, G.N, i, idx) = lh[i];
#pragma unroll
    for (int i = 0; i < Q_G; ++i) *slot(a.lg_out, G.N, i, idx) = lg[i];
    a.sadj[idx] = S4<R>{lGx, lGy, lGz, lL};
    acc0 = double(lomp);
    acc1 = double(lsig);
    acc2 = double(lxi);
  }
  // FP64 block sums in a fixed order, added to this block's running slot
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) {
    acc0 += __shfl_xor(acc0, off, 64);
    acc1 += __shfl_xor(acc1, off, 64);
    acc2 += __shfl_xor(acc2, off, 64);
  }
  const int tid = threadIdx.x + threadIdx.y * G.bx;
  if ((tid & 63) == 0) {
    red[tid >> 6][0] = acc0;
    red[tid >> 6][1] = acc1;
    red[tid >> 6][2] = acc2;
  }
  __syncthreads();
  if (tid < 3) {
    const double v = ((red[0][tid] + red[1][tid]) + red[2][tid]) + red[3][tid];
    a.gsum[(long long)blockIdx.x * 3 + tid] += v;
  }
}

template <typename R>
struct AdjStencilArgs {
  const S4<R>* sadj;  // [N]
  const unsigned* nbr; // solid-neighbour bits (mask only)
  R* aphi_out;        // [N]
  Geom geo;
};

// a_phi(y) = sum_m valid(y, m) [-3 w_m c_m.(s_G(y+c_m) + s_G(y)) + 6 w_m (s_L(y+c_m) - s_L(y))]
// Marching in z like the forward step: each block owns a tile and a chunk of
// planes and keeps the stencil adjoints of 4 planes (tile + one-cell ring) in
// an LDS ring, so every value is read from memory about once; the loads of
// plane z + 2 are in flight while plane z is summed.  valid(y, m) is the
// cell's wall bits (box faces and solid neighbours), as in the forward step.
template <typename R, bool MASK>
__global__ __launch_bounds__(256) void k_adj_stencil(AdjStencilArgs<R> a) {
  extern __shared__ unsigned char smem_raw[];
  const Geom& G = a.geo;
  const int TX = G.bx + 2, TY = G.by + 2, TXY = TX * TY;
  S4<R>* ts = reinterpret_cast<S4<R>*>(smem_raw);                        // [4 slots][TXY]
  const ChunkCoord t = chunk_of_block(G);
  const int lx = threadIdx.x, ly = threadIdx.y, tid = lx + ly * G.bx;
  const int x = t.x0 + lx, y = t.y0 + ly;
  const bool active = x < G.nx && y < G.ny;
  int ox = x, oy = y;
  const bool own_ok = wrap(ox, G.nx, G.px) && wrap(oy, G.ny, G.py);
  const int opos = (ly + 1) * TX + lx + 1;
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
  // stencil adjoints of solid or out-of-box positions are never used (the
  // wall bits exclude them), so they are simply not loaded
  auto fetch = [&](bool ok, int X, int Y, int Z) {
    S4<R> c{R(0), R(0), R(0), R(0)};
    if (ok) c = a.sadj[X + G.nx * Y + sxy * Z];
    return c;
  };
  S4<R> own{R(0), R(0), R(0), R(0)}, ring{R(0), R(0), R(0), R(0)};
  auto fetch_plane = [&](int p) {
    int pz = p;
    const bool zok = wrap(pz, G.nz, G.pz);
    own = fetch(own_ok && zok, ox, oy, pz);
    if (tid < NH) ring = fetch(halo_ok && zok, hx, hy, pz);
  };
  auto put_plane = [&](int p) {
    ts[(p & 3) * TXY + opos] = own;
    if (tid < NH) ts[(p & 3) * TXY + hpos] = ring;
  };
  fetch_plane(t.z0 - 1);
  put_plane(t.z0 - 1);
  fetch_plane(t.z0);
  put_plane(t.z0);
  fetch_plane(t.z0 + 1);
  for (int z = t.z0; z < t.z1; ++z) {
    // plane z + 1 (fetched one iteration ago) into the ring, then start the
    // loads of plane z + 2 so they overlap this plane's arithmetic
    put_plane(z + 1);
    if (z + 1 < t.z1) fetch_plane(z + 2);
    __syncthreads();
    if (active) {
      const unsigned idx = x + G.nx * y + sxy * z;
      bool solid;
      const unsigned walls = cell_walls<MASK>(x, y, z, idx, G, a.nbr, solid);
      if (!solid) {
        const S4<R>* pm = ts + ((z - 1) & 3) * TXY;
        const S4<R>* p0 = ts + (z & 3) * TXY;
        const S4<R>* pp = ts + ((z + 1) & 3) * TXY;
        const S4<R> c0 = p0[opos];
        R acc = R(0);
#pragma unroll
        for (int k = 1; k < 27; ++k) {
          if (!(walls & (1u << k))) {
            const Dir d = cg(k);
            const S4<R>* pl = d.z < 0 ? pm : (d.z > 0 ? pp : p0);
            const S4<R> m = pl[(ly + 1 + d.y) * TX + (lx + 1 + d.x)];
            const R w = R(wg(k));
            const R gsum = dot(d, m.gx + c0.gx, m.gy + c0.gy, m.gz + c0.gz);
            acc += R(-3) * w * gsum + R(6) * w * (m.l - c0.l);
          }
        }
        a.aphi_out[idx] = acc;
      }
    }
  }
}

// a_phi += dL/dphi (FP64 input)
template <typename R>
__global__ __launch_bounds__(256) void k_adj_inject(R* __restrict__ aphi, const double* __restrict__ d,
                                                     long long N) {
  const long long i = blockIdx.x * 256ll + threadIdx.x;
  if (i < N) aphi[i] = R(double(aphi[i]) + d[i]);
}

// dL/dphi0 = sum_i (lam_h,i + a_phi) Gamma_i(u0)
template <typename R, bool MASK>
__global__ __launch_bounds__(256) void k_adj_init(const R* __restrict__ lh, const R* __restrict__ aphi,
                                                   const double* __restrict__ u0,
                                                   const unsigned char* __restrict__ mask, long long N,
                                                   double* __restrict__ out) {
  const long long i = blockIdx.x * 256ll + threadIdx.x;
  if (i >= N) return;
  if (MASK && mask[i]) { out[i] = 0.0; return; }
  double ux = 0, uy = 0, uz = 0;
  if (u0) { ux = u0[i]; uy = u0[N + i]; uz = u0[2 * N + i]; }
  const R rx = R(ux), ry = R(uy), rz = R(uz);
  const R base = R(1) - R(1.5) * (rx * rx + ry * ry + rz * rz);
  R acc = R(0);
#pragma unroll
  for (int k = 0; k < Q_H; ++k) {
    const R cu = dot(ch(k), rx, ry, rz);
    acc += (lh[k * N + i] + aphi[i]) * R(wh(k)) * (base + cu * (R(3) + R(4.5) * cu));
  }
  out[i] = double(acc);
}

}  // namespace pflbm
