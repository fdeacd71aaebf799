// Free swimmer: the articulated body of Sec. III-A driven two ways with the
// fluid (the fluid's force enters the body dynamics as the external
// generalized force of Eq. (1)), for a planar chain whose joint motion is
// prescribed. With every joint prescribed, articulated-body (hybrid) dynamics
// leaves only the floating base free, and the base equations are the
// whole-body momentum balance:
//   M dV/dt = F,        d/dt (I_c theta' + L_s) = T,
// F and T the fluid's force and torque about the body's mass centre, I_c the
// chain's moment of inertia about its mass centre and L_s the angular
// momentum of its shape change. The local domain follows the mass centre
// (Sec. III-B: the frame translates with the body), so the frame's velocity is
// V and its acceleration enters the fluid through Eq. (3).
//
// Time stepping (unit steps, r = rho_fluid / rho_body, k the artificial added
// mass as a multiple of the body's):
//   (1 + k) a(n+1) = F(n)/M + (r + k) a(n),  V(n+1) = V(n) + a(n),
//   (1 + k) I_c(n+1) theta'(n+1) = L(n) + T(n) + (r I_c(n) + k I_c(n+1)) theta''(n)
//                                  - L_s(n+1) + k I_c(n+1) theta'(n),
//   L(n+1) = I_c(n+1) theta'(n+1) + L_s(n+1),  theta(n+1) = theta(n) + theta'(n+1).
// The frame acceleration of step n is needed before step n's force is known,
// hence a(n+1) from F(n). The direct-forcing force includes the reaction of
// the fluid the body encloses, carried along with it; the r terms add it back
// (enclosed fluid moving rigidly: mass r M, inertia r I_c). With k = 0 this is
// explicit coupling, stable on the swimmer tests down to rho_body / rho_fluid
// = 1.5: a reaction -m_a a(n) in the force feeds back as -(m_a / M) a(n). The
// k terms, added to both sides, turn that factor into (k M - m_a)/(M + k M),
// so a k of order one keeps neutrally buoyant bodies stable, and leave a
// steady acceleration unchanged.
//
// Host code only (no device work).
#pragma once

#include <cmath>

namespace lbmib {

struct ChainShape {
  // body frame: joints J_j (head joint at the origin), link mass centres r_j
  // and their velocities from the prescribed shape; mass centre rc, rcd
  double J[64][2], Jd[64][2];
  double rc[2], rcd[2];
  double Ic, Ls;
};

inline bool chain_shape(const lbm_swimmer *s, const double *psi, const double *psid, ChainShape &c) {
  const int nb = s->nbones;
  const double h = s->link_length;
  double M = 0.0, m1[2] = {0.0, 0.0}, m1d[2] = {0.0, 0.0};
  double r[64][2], rd[64][2];
  c.J[0][0] = c.J[0][1] = c.Jd[0][0] = c.Jd[0][1] = 0.0;
  for (int j = 0; j < nb; ++j) {
    const double cs = std::cos(psi[j]), sn = std::sin(psi[j]);
    const double a = s->com[j];
    r[j][0] = c.J[j][0] + a * cs;
    r[j][1] = c.J[j][1] + a * sn;
    rd[j][0] = c.Jd[j][0] - a * psid[j] * sn;
    rd[j][1] = c.Jd[j][1] + a * psid[j] * cs;
    if (j + 1 < nb) {
      c.J[j + 1][0] = c.J[j][0] + h * cs;
      c.J[j + 1][1] = c.J[j][1] + h * sn;
      c.Jd[j + 1][0] = c.Jd[j][0] - h * psid[j] * sn;
      c.Jd[j + 1][1] = c.Jd[j][1] + h * psid[j] * cs;
    }
    M += s->mass[j];
    for (int q = 0; q < 2; ++q) {
      m1[q] += s->mass[j] * r[j][q];
      m1d[q] += s->mass[j] * rd[j][q];
    }
  }
  if (!(M > 0.0)) return false;
  for (int q = 0; q < 2; ++q) {
    c.rc[q] = m1[q] / M;
    c.rcd[q] = m1d[q] / M;
  }
  c.Ic = 0.0;
  c.Ls = 0.0;
  for (int j = 0; j < nb; ++j) {
    const double qx = r[j][0] - c.rc[0], qy = r[j][1] - c.rc[1];
    const double vx = rd[j][0] - c.rcd[0], vy = rd[j][1] - c.rcd[1];
    c.Ic += s->inertia[j] + s->mass[j] * (qx * qx + qy * qy);
    c.Ls += s->inertia[j] * psid[j] + s->mass[j] * (qx * vy - qy * vx);
  }
  return c.Ic > 0.0;
}

inline double chain_mass(const lbm_swimmer *s) {
  double M = 0.0;
  for (int j = 0; j < s->nbones; ++j) M += s->mass[j];
  return M;
}

inline bool swimmer_ok(const lbm_swimmer *s) {
  if (!s || s->nbones < 1 || s->nbones > 64 || !s->mass || !s->com || !s->inertia || !s->joints_rest) return false;
  if (!(s->link_length > 0.0) || !(s->fluid_ratio >= 0.0) || !std::isfinite(s->fluid_ratio)) return false;
  if (!(s->added_mass >= 0.0) || !std::isfinite(s->added_mass)) return false;
  if (s->free_yaw != 0 && s->free_yaw != 1) return false;
  for (int j = 0; j < s->nbones; ++j)
    if (!(s->mass[j] > 0.0) || !(s->inertia[j] > 0.0) || !std::isfinite(s->com[j])) return false;
  return true;
}

}  // namespace lbmib
