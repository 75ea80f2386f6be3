// Device arithmetic of one unsplit CTU/PPM step for an ideal gamma-law gas.
//
// The paper names the scheme (an unsplit piecewise parabolic method, section
// 3.2) and nothing more; the pieces below follow the published methods:
// PPM reconstruction, limiter and flattening of Colella & Woodward (1984),
// reference-state characteristic tracing and corner-transport-upwind
// coupling of Colella (1990), Saltzman (1994) and Miller & Colella (2002), and
// the HLLC flux of Toro, Spruce & Speares (1994) with Davis (1988) wave speeds,
// or the two-shock approximate Riemann solver of the PPM lineage (Colella
// 1982; Colella & Glaz 1985).
// Every expression keeps the parenthesisation of the stated formulas and the
// library is compiled without floating-point contraction, so each operation
// rounds once, in IEEE order.
#pragma once
#include <hip/hip_runtime.h>

#define CTU_DEV __device__ __forceinline__

namespace ctu {

CTU_DEV double dmin(double a, double b) { return a < b ? a : b; }
CTU_DEV double dmax(double a, double b) { return a > b ? a : b; }

// Monotonised-central slope of the middle of three cell values.
CTU_DEV double mc_slope(double am, double a0, double ap) {
  const double dm = a0 - am, dp = ap - a0, dc = 0.5 * (ap - am);
  if (dm * dp > 0.0) {
    const double lim = dmin(fabs(dc), dmin(2.0 * fabs(dm), 2.0 * fabs(dp)));
    return copysign(lim, dc);
  }
  return 0.0;
}

// Parabola of one cell from its 5-cell stencil s[0..4] and flattening phi:
// interface values (CW84 eq. 1.6), blend towards the average, CW84 eq. 1.10
// monotonicity; returns (aL, aR, da, a6).
struct Parab { double aL, aR, da, a6; };

// With eta > 0 (contact steepening, CW84 section 1.3) the interface values
// first move towards the edge values of the neighbours' linear profiles,
// s1 + dl/2 and s3 - dr/2, by the weight eta.
CTU_DEV Parab ppm(double s0, double s1, double s2, double s3, double s4, double phi, double eta = 0.0) {
  const double C6 = 1.0 / 6.0;
  const double dl = mc_slope(s0, s1, s2);
  const double dcen = mc_slope(s1, s2, s3);
  const double dr = mc_slope(s2, s3, s4);
  double aL = 0.5 * (s1 + s2) - C6 * (dcen - dl);
  double aR = 0.5 * (s2 + s3) - C6 * (dr - dcen);
  if (eta > 0.0) {
    const double aLd = s1 + 0.5 * dl;
    const double aRd = s3 - 0.5 * dr;
    aL = aL * (1.0 - eta) + eta * aLd;
    aR = aR * (1.0 - eta) + eta * aRd;
  }
  aL = phi * aL + (1.0 - phi) * s2;
  aR = phi * aR + (1.0 - phi) * s2;
  if ((aR - s2) * (s2 - aL) <= 0.0) {
    aL = s2;
    aR = s2;
  } else {
    const double d = aR - aL;
    const double m = s2 - 0.5 * (aL + aR);
    if (d * m > C6 * (d * d)) aL = 3.0 * s2 - 2.0 * aR;
    else if (-C6 * (d * d) > d * m) aR = 3.0 * s2 - 2.0 * aL;
  }
  Parab p;
  p.aL = aL;
  p.aR = aR;
  p.da = aR - aL;
  p.a6 = 6.0 * (s2 - 0.5 * (aL + aR));
  return p;
}

// Extremum-preserving variant (Colella & Sekora 2008): fourth-order interface
// values 7/12 (a0 + a1) - 1/12 (am1 + a2), limited where not between their two
// cells through second differences (C = 1.25); flattening towards the
// average; at a local extremum of the parabola or of the averages the
// parabola's second difference -2 (6 a - 3 (aL + aR)) is limited against the
// neighbouring ones and both edge offsets scale by lim / d2 (flat if d2 = 0);
// elsewhere an edge farther than twice the other from the average moves to
// twice (right edge first).
CTU_DEV double cs_lim3(double a, double b, double c) {
  const double C = 1.25;
  if ((a > 0.0 && b > 0.0 && c > 0.0) || (a < 0.0 && b < 0.0 && c < 0.0))
    return copysign(dmin(dmin(C * fabs(b), C * fabs(c)), fabs(a)), a);
  return 0.0;
}
CTU_DEV double cs_lim4(double a, double b, double c, double d) {
  const double C = 1.25;
  if ((a > 0.0 && b > 0.0 && c > 0.0 && d > 0.0) || (a < 0.0 && b < 0.0 && c < 0.0 && d < 0.0))
    return copysign(dmin(dmin(C * fabs(b), C * fabs(c)), dmin(C * fabs(d), fabs(a))), a);
  return 0.0;
}
CTU_DEV double cs_face(double am1, double a0, double a1, double a2) {
  double f = (7.0 / 12.0) * (a0 + a1) - (1.0 / 12.0) * (am1 + a2);
  if ((f - a0) * (a1 - f) < 0.0) {
    const double d2 = 3.0 * ((a0 - 2.0 * f) + a1);
    const double d2L = (am1 - 2.0 * a0) + a1;
    const double d2R = (a0 - 2.0 * a1) + a2;
    f = 0.5 * (a0 + a1) - cs_lim3(d2, d2L, d2R) / 6.0;
  }
  return f;
}
CTU_DEV Parab ppm_cs(double s0, double s1, double s2, double s3, double s4, double phi) {
  double aL = cs_face(s0, s1, s2, s3);
  double aR = cs_face(s1, s2, s3, s4);
  aL = phi * aL + (1.0 - phi) * s2;
  aR = phi * aR + (1.0 - phi) * s2;
  if ((aR - s2) * (s2 - aL) <= 0.0 || (s1 - s2) * (s2 - s3) <= 0.0) {
    const double d2 = -2.0 * (6.0 * s2 - 3.0 * (aL + aR));
    const double d2C = (s1 - 2.0 * s2) + s3;
    const double d2L = (s0 - 2.0 * s1) + s2;
    const double d2R = (s2 - 2.0 * s3) + s4;
    if (d2 != 0.0) {
      const double r = cs_lim4(d2, d2L, d2R, d2C) / d2;
      aL = s2 + (aL - s2) * r;
      aR = s2 + (aR - s2) * r;
    } else {
      aL = s2;
      aR = s2;
    }
  } else {
    if (fabs(aR - s2) >= 2.0 * fabs(aL - s2)) aR = s2 - 2.0 * (aL - s2);
    if (fabs(aL - s2) >= 2.0 * fabs(aR - s2)) aL = s2 - 2.0 * (aR - s2);
  }
  Parab p;
  p.aL = aL;
  p.aR = aR;
  p.da = aR - aL;
  p.a6 = 6.0 * (s2 - 0.5 * (aL + aR));
  return p;
}

// The parabola of reconstruction variant V: bit 0 the limiter (0 CW84, 1
// Colella & Sekora); bit 1 contact steepening with weight eta (CW84 only).
template <int V>
CTU_DEV Parab ppm_l(double s0, double s1, double s2, double s3, double s4, double phi, double eta = 0.0) {
  if (V & 1) return ppm_cs(s0, s1, s2, s3, s4, phi);
  if (V & 2) return ppm(s0, s1, s2, s3, s4, phi, eta);
  return ppm(s0, s1, s2, s3, s4, phi);
}

// CW84 contact detector of a density stencil r0..r4 with the neighbours'
// pressures pm, pp: eta~ = -(d2+ - d2-) / (r3 - r1) from the neighbours'
// second differences d2 = (r+1 - 2 r + r-1)/6 where they change sign and the
// jump exceeds 0.01 of the smaller neighbour; eta = clamp(20 (eta~ - 0.05),
// 0, 1); zero unless gamma K0 |r3 - r1| / min(r3, r1) >= |pp - pm| / min(pp,
// pm) with K0 = 0.1 (the pressure jump is small against the density jump).
CTU_DEV double steep_eta(double r0, double r1, double r2, double r3, double r4, double pm, double pp,
                         double gamma) {
  const double d2m = ((r2 - 2.0 * r1) + r0) / 6.0;
  const double d2p = ((r4 - 2.0 * r3) + r2) / 6.0;
  const double dr = r3 - r1;
  double eta = 0.0;
  if (d2p * d2m < 0.0 && fabs(dr) - 0.01 * dmin(fabs(r3), fabs(r1)) > 0.0) {
    const double et = -(d2p - d2m) / dr;
    eta = dmax(0.0, dmin(20.0 * (et - 0.05), 1.0));
  }
  if (gamma * 0.1 * fabs(dr) / dmin(r3, r1) < fabs(pp - pm) / dmin(pp, pm)) eta = 0.0;
  return eta;
}

// Averages of the parabola over the last sig of the cell (towards its right
// edge) and over the first sig (towards its left edge).
CTU_DEV double avg_right(const Parab& p, double sig) {
  const double C23 = 2.0 / 3.0;
  return p.aR - 0.5 * sig * (p.da - (1.0 - C23 * sig) * p.a6);
}
CTU_DEV double avg_left(const Parab& p, double sig) {
  const double C23 = 2.0 / 3.0;
  return p.aL + 0.5 * sig * (p.da + (1.0 - C23 * sig) * p.a6);
}

// Reference-state tracing of one cell to the half time level.  par[m] are the
// parabolas of the permuted primitives (rho, u_n, u_t1, u_t2, p); rho, un, c
// the cell-centre values.  trace_up gives the left state at the cell's upper
// face (families with positive speed arrive; the reference is the u+c
// family's average), trace_dn the right state at its lower face (negative
// speeds; reference from the u-c family).
CTU_DEV void trace_up(const Parab par[5], double rho, double un, double c, double dtdx, double up[5]) {
  const double lm = un - c, l0 = un, lp = un + c;
  const double sm = fabs(lm) * dtdx, s0 = fabs(l0) * dtdx, sp = fabs(lp) * dtdx;
  const double csq = c * c;
  double Im[5], I0[5], ref[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    Im[m] = lm > 0.0 ? avg_right(par[m], sm) : par[m].aR;
    I0[m] = l0 > 0.0 ? avg_right(par[m], s0) : par[m].aR;
    ref[m] = lp > 0.0 ? avg_right(par[m], sp) : par[m].aR;
  }
  const double bm = -(rho / (2.0 * c)) * (ref[1] - Im[1]) + (ref[4] - Im[4]) / (2.0 * csq);
  const double b0 = (ref[0] - I0[0]) - (ref[4] - I0[4]) / csq;
  const double bt1 = ref[2] - I0[2];
  const double bt2 = ref[3] - I0[3];
#pragma unroll
  for (int m = 0; m < 5; ++m) up[m] = ref[m];
  if (lm > 0.0) {
    up[0] = up[0] - bm;
    up[1] = up[1] - bm * (-(c / rho));
    up[4] = up[4] - bm * csq;
  }
  if (l0 > 0.0) {
    up[0] = up[0] - b0;
    up[2] = up[2] - bt1;
    up[3] = up[3] - bt2;
  }
}

CTU_DEV void trace_dn(const Parab par[5], double rho, double un, double c, double dtdx, double dn[5]) {
  const double lm = un - c, l0 = un, lp = un + c;
  const double sm = fabs(lm) * dtdx, s0 = fabs(l0) * dtdx, sp = fabs(lp) * dtdx;
  const double csq = c * c;
  double Ip[5], I0[5], ref[5];
#pragma unroll
  for (int m = 0; m < 5; ++m) {
    ref[m] = lm < 0.0 ? avg_left(par[m], sm) : par[m].aL;
    I0[m] = l0 < 0.0 ? avg_left(par[m], s0) : par[m].aL;
    Ip[m] = lp < 0.0 ? avg_left(par[m], sp) : par[m].aL;
  }
  const double bp = (rho / (2.0 * c)) * (ref[1] - Ip[1]) + (ref[4] - Ip[4]) / (2.0 * csq);
  const double b0 = (ref[0] - I0[0]) - (ref[4] - I0[4]) / csq;
  const double bt1 = ref[2] - I0[2];
  const double bt2 = ref[3] - I0[3];
#pragma unroll
  for (int m = 0; m < 5; ++m) dn[m] = ref[m];
  if (lp < 0.0) {
    dn[0] = dn[0] - bp;
    dn[1] = dn[1] - bp * (c / rho);
    dn[4] = dn[4] - bp * csq;
  }
  if (l0 < 0.0) {
    dn[0] = dn[0] - b0;
    dn[2] = dn[2] - bt1;
    dn[3] = dn[3] - bt2;
  }
}

// Which HLLC state a face flux comes from and the numbers a passive species
// needs to take the same state: kind 0 the left state, 1 the left star state,
// 2 the right star state, 3 the right state; m the mass flux of that state,
// SK its wave speed, fac the star-density factor, rK its density.
struct Wave { double m, SK, fac, rK; int kind; };

// HLLC flux between permuted primitive states L and R; F in permuted
// conserved order (mass, normal momentum, t1 momentum, t2 momentum, energy).
CTU_DEV void hllc(const double L[5], const double R[5], double g, double rgm1, double F[5], Wave& W) {
  const double rL = L[0], uL = L[1], vL = L[2], wL = L[3], pL = L[4];
  const double rR = R[0], uR = R[1], vR = R[2], wR = R[3], pR = R[4];
  const double cL = sqrt(g * pL / rL);
  const double cR = sqrt(g * pR / rR);
  const double SL = dmin(uL - cL, uR - cR);
  const double SR = dmax(uL + cL, uR + cR);
  const double EL = pL * rgm1 + 0.5 * rL * ((uL * uL + vL * vL) + wL * wL);
  const double ER = pR * rgm1 + 0.5 * rR * ((uR * uR + vR * vR) + wR * wR);
  W.SK = 0.0;
  W.fac = 0.0;
  if (SL >= 0.0) {
    const double m = rL * uL;
    F[0] = m; F[1] = m * uL + pL; F[2] = m * vL; F[3] = m * wL; F[4] = uL * (EL + pL);
    W.m = m; W.rK = rL; W.kind = 0;
    return;
  }
  const double Ss = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) /
                    (rL * (SL - uL) - rR * (SR - uR));
  if (Ss < 0.0 && !(SR > 0.0)) {
    const double m = rR * uR;
    F[0] = m; F[1] = m * uR + pR; F[2] = m * vR; F[3] = m * wR; F[4] = uR * (ER + pR);
    W.m = m; W.rK = rR; W.kind = 3;
    return;
  }
  const bool left = Ss >= 0.0;
  const double rK = left ? rL : rR, uK = left ? uL : uR, vK = left ? vL : vR;
  const double wK = left ? wL : wR, pK = left ? pL : pR, EK = left ? EL : ER;
  const double SK = left ? SL : SR;
  const double m = rK * uK;
  const double fac = rK * (SK - uK) / (SK - Ss);
  const double us4 = fac * (EK / rK + (Ss - uK) * (Ss + pK / (rK * (SK - uK))));
  F[0] = m + SK * (fac - rK);
  F[1] = (m * uK + pK) + SK * (fac * Ss - m);
  F[2] = m * vK + SK * (fac * vK - rK * vK);
  F[3] = m * wK + SK * (fac * wK - rK * wK);
  F[4] = uK * (EK + pK) + SK * (us4 - EK);
  W.m = m; W.SK = SK; W.fac = fac; W.rK = rK; W.kind = left ? 1 : 2;
}

CTU_DEV void hllc(const double L[5], const double R[5], double g, double rgm1, double F[5]) {
  Wave W;
  hllc(L, R, g, rgm1, F, W);
}

// Godunov flux of the two-shock approximate Riemann solution between permuted
// primitive states L and R (F in permuted conserved order).  Both waves on
// their shock curves: Lagrangian sound speeds C = sqrt(gamma p rho), shock
// speeds W(p) = C sqrt(1 + (gamma+1)/(2 gamma) (p/p_K - 1)); the star
// pressure from the acoustic estimate by a fixed number of Newton steps on
// u*_L(p) = u*_R(p) with curve slopes Z = 2 W^3 / (W^2 + C^2), floored; the
// contact speed from the last W.  The state at x/t = 0 is on the contact's
// upwind side K: K beyond the K wave, the star state (density from the shock
// relation) behind it, a linear blend inside a rarefaction fan that straddles
// x/t = 0; transverse velocities (and species, through W) from K.
constexpr int kTwoShockIters = 6;

CTU_DEV void twoshock(const double L[5], const double R[5], double g, double rgm1, double sd, double sp,
                      double F[5], Wave& W) {
  const double gp = (g + 1.0) / (2.0 * g);
  const double rL = L[0], uL = L[1], pL = L[4];
  const double rR = R[0], uR = R[1], pR = R[4];
  const double CL = sqrt(g * pL * rL), CR = sqrt(g * pR * rR);
  double ps = ((CR * pL + CL * pR) + CL * CR * (uL - uR)) / (CL + CR);
  ps = dmax(ps, sp);
  double WL = CL, WR = CR;
  for (int it = 0; it < kTwoShockIters; ++it) {
    WL = CL * sqrt(1.0 + gp * (ps / pL - 1.0));
    WR = CR * sqrt(1.0 + gp * (ps / pR - 1.0));
    const double ZL = 2.0 * (WL * WL * WL) / (WL * WL + CL * CL);
    const double ZR = 2.0 * (WR * WR * WR) / (WR * WR + CR * CR);
    const double usL = uL - (ps - pL) / WL;
    const double usR = uR + (ps - pR) / WR;
    ps = ps - (ZL * ZR) * (usR - usL) / (ZL + ZR);
    ps = dmax(ps, sp);
  }
  WL = CL * sqrt(1.0 + gp * (ps / pL - 1.0));
  WR = CR * sqrt(1.0 + gp * (ps / pR - 1.0));
  const double us = ((WL * uL + WR * uR) + (pL - pR)) / (WL + WR);
  const bool left = us >= 0.0;
  const double WK = left ? WL : WR;
  const double rK = left ? rL : rR, uK = left ? uL : uR, pK = left ? pL : pR;
  const double vK = left ? L[2] : R[2], wK = left ? L[3] : R[3];
  const double sgn = left ? -1.0 : 1.0;
  double rs = 1.0 / (1.0 / rK - (ps - pK) / (WK * WK));
  rs = dmax(rs, sd);
  const double cK = sqrt(g * pK / rK), cs = sqrt(g * ps / rs);
  double head, tail;
  if (ps > pK) {
    head = uK + sgn * (WK / rK);
    tail = head;
  } else {
    head = uK + sgn * cK;
    tail = us + sgn * cs;
  }
  double ri, ui, pi;
  if (left ? head >= 0.0 : head <= 0.0) {
    ri = rK; ui = uK; pi = pK;
  } else if (left ? tail <= 0.0 : tail >= 0.0) {
    ri = rs; ui = us; pi = ps;
  } else {
    const double f = (0.0 - tail) / (head - tail);
    ri = rs + f * (rK - rs);
    ui = us + f * (uK - us);
    pi = ps + f * (pK - ps);
  }
  const double m = ri * ui;
  const double Ei = pi * rgm1 + 0.5 * ri * ((ui * ui + vK * vK) + wK * wK);
  F[0] = m;
  F[1] = m * ui + pi;
  F[2] = m * vK;
  F[3] = m * wK;
  F[4] = ui * (Ei + pi);
  W.m = m;
  W.rK = ri;
  W.SK = 0.0;
  W.fac = 0.0;
  W.kind = left ? 0 : 3;
}

// Flux of a passive mass fraction (X_L, X_R at the face) for the HLLC state
// W chose: X rides the contact like a transverse velocity, so its star value
// is fac X_K.
CTU_DEV double species_flux(const Wave& W, double XL, double XR) {
  if (W.kind == 0) return W.m * XL;
  if (W.kind == 3) return W.m * XR;
  const double XK = W.kind == 1 ? XL : XR;
  return W.m * XK + W.SK * (W.fac * XK - W.rK * XK);
}

// Tracing of a passive mass fraction with parabola p: only the contact
// family (speed un) carries it, so like a transverse velocity it takes the
// reference average and subtracts the reference's excess over the contact
// family's average when that family reaches the face.  sp, s0, sm are the
// |speed| dt/dx of the u+c, u and u-c families.
CTU_DEV double species_up(const Parab& p, double lp, double l0, double sp, double s0) {
  const double ref = lp > 0.0 ? avg_right(p, sp) : p.aR;
  const double I0 = l0 > 0.0 ? avg_right(p, s0) : p.aR;
  double v = ref;
  if (l0 > 0.0) v = v - (ref - I0);
  return v;
}
CTU_DEV double species_dn(const Parab& p, double lm, double l0, double sm, double s0) {
  const double ref = lm < 0.0 ? avg_left(p, sm) : p.aL;
  const double I0 = l0 < 0.0 ? avg_left(p, s0) : p.aL;
  double v = ref;
  if (l0 < 0.0) v = v - (ref - I0);
  return v;
}

}  // namespace ctu
