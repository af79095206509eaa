// 0D boundary models on the device (FP64, one thread per boundary): the
// LV elastance with its valve and the C-infinity smoothing after closure
// (Eqs. LVE, SmoothFunction, vnew), the 3-element Windkessel in both
// coupling directions (Eqs. rightbc, rightQ), constant pressure / velocity.
// Shared by the 3D solver and the axisymmetric one.
#pragma once

#include "lbm_internal.h"

namespace lbm {

__device__ inline double smooth_S(double t, double t0, double L) {
  if (t < t0) return 1.0;
  if (t >= t0 + L) return 0.0;
  const double u = (t - t0) / L;
  return exp(2.0 * exp(-1.0 / u) / (u - 1.0));
}

// Double-Hill elastance and its time derivative at time t (steps) in the beat.
__device__ inline void elastance(const double* p, double t, double& E, double& dE) {
  const double tn = t / p[3];
  const double x1 = tn / p[7], x2 = tn / p[9];
  const double a = pow(x1, p[8]), b = pow(x2, p[10]);
  const double h1 = a / (1.0 + a), h2 = 1.0 / (1.0 + b);
  double dh1 = 0.0, dh2 = 0.0;
  if (tn > 0.0) {
    dh1 = p[8] * a / (x1 * p[7]) / ((1.0 + a) * (1.0 + a));
    dh2 = -p[10] * b / (x2 * p[9]) / ((1.0 + b) * (1.0 + b));
  }
  const double amp = (p[0] - p[1]) * p[6];
  E = amp * h1 * h2 + p[1];
  dE = amp * (dh1 * h2 + h1 * dh2) / p[3];
}

__device__ inline void zerod_update(BcDev& b, int64_t n, double Qp, double Pbar) {
  b.snap = 0;
  switch (b.kind) {
    case BC_PRESSURE:
      b.vmode = 0;
      b.pstar = b.par[0];
      break;
    case BC_VELOCITY:
      b.vmode = 1;
      b.vkind = VK_CONST;
      b.vz = b.par[0];
      break;
    case BC_WK3: {
      const double Z = b.par[0], C = b.par[1], R = b.par[2];
      if (b.par[3] == 0.0) {
        // flux-driven: C dPw/dt = Q - Pw/R, P* = Pw + Z Q
        const double Q = b.boundary == 0 ? -Qp : Qp;
        b.Pw += (Q - b.Pw / R) / C;
        b.vmode = 0;
        b.pstar = b.Pw + Z * Q;
      } else {
        // pressure-driven: C dPw/dt = (P - Pw)/Z - Pw/R, outflow (P - Pw)/Z
        b.Pw += ((Pbar - b.Pw) / Z - b.Pw / R) / C;
        const double Q = (Pbar - b.Pw) / Z;
        const double want = b.boundary == 0 ? -Q : Q;
        b.vmode = 1;
        b.vkind = VK_CORRECT;
        b.vz = (want - Qp) / (b.area > 0.0 ? b.area : 1.0);
      }
      break;
    }
    case BC_LV: {
      const double* p = b.par;
      const int64_t cyc = (int64_t)floor((double)n / p[2]);
      if (cyc != b.cycle) {
        b.cycle = cyc;
        b.Pv = p[4];
        b.open = 0;
        b.inflow = 0;
        b.Td = -1;
      }
      double E, dE;
      elastance(p, (double)n - (double)cyc * p[2], E, dE);
      // closes when the inflow turns negative after ejection has begun (the
      // residual flux of the first steps after opening does not count)
      if (b.open && b.inflow && Qp < 0.0) {
        b.open = 0;
        b.Td = n;
        b.snap = 1;
      } else if (b.open) {
        if (Qp > 0.0) b.inflow = 1;
      } else if (b.Td < 0 && b.Pv > Pbar) {
        b.open = 1;
        b.inflow = 0;
      }
      const double Q = b.open ? Qp : 0.0;
      // dPv/dt = -(C' Pv + Q)/C with C = 1/E  <=>  dPv/dt = (E'/E) Pv - E Q
      b.Pv += (dE / E) * b.Pv - E * Q;
      if (b.open) {
        b.vmode = 0;
        b.pstar = b.Pv;
      } else {
        b.vmode = 1;
        b.vkind = VK_SNAPSHOT;
        b.S = b.Td < 0 ? 0.0 : smooth_S((double)(n + 1), (double)b.Td, p[5]);
      }
      break;
    }
    default:
      break;
  }
  b.dstar = 3.0 * b.pstar;
}


}  // namespace lbm
