// Energy splits psi = g(d) psi+ + psi- and their stresses (Sec. 2.1,
// eq. spectral_split, eq. amor_split, the star-convex variant), plus their
// reverse-mode derivatives for the adjoint step.
//
// Strain and stress are the independent components (xx, yy, xy) of the
// symmetric 2x2 tensors.  <x>+ = x for x > 0, else 0 (derivative 0 at 0).
// Plane stress for the vol-dev and star-convex splits: the out-of-plane
// strain s*tr (s = -nu/(1-nu)) enters the 3D trace c*tr (c = 1+s) and the
// deviatoric norm; Kc2 = K c^2 and coef = s^2 - c^2/3 carry that choice.
#pragma once

#include "pf_internal.hpp"

namespace pf {

enum { SPLIT_NONE = 0, SPLIT_SPECTRAL = 1, SPLIT_VOLDEV = 2, SPLIT_STAR = 3 };

template <typename T>
__device__ __forceinline__ T posp(T x) { return x > T(0) ? x : T(0); }
template <typename T>
__device__ __forceinline__ T negp(T x) { return x < T(0) ? x : T(0); }

// Constant P1 strain eps = sym(sum_k u_k (x) grad phi_k).  The forward and
// the adjoint kernels share this code so that psi+ is reproduced bit for bit.
template <typename T>
__device__ __forceinline__ void elem_strain(T u0x, T u0y, T u1x, T u1y, T u2x, T u2y, T g0x, T g0y, T g1x, T g1y,
                                            T g2x, T g2y, T& exx, T& eyy, T& exy) {
  exx = u0x * g0x + u1x * g1x + u2x * g2x;
  eyy = u0y * g0y + u1y * g1y + u2y * g2y;
  exy = T(0.5) * ((u0x * g0y + u0y * g0x) + (u1x * g1y + u1y * g1x) + (u2x * g2y + u2y * g2x));
}

// psi+ and the two stress parts sigma+ (sp) and sigma- (sm).
template <int S, typename T>
__device__ __forceinline__ void split_eval(T exx, T eyy, T exy, const InstP<T>& P, T& psi_p, T sp[3], T sm[3]) {
  const T tr = exx + eyy;
  if constexpr (S == SPLIT_NONE) {
    psi_p = T(0.5) * P.lam * tr * tr + P.mu * (exx * exx + eyy * eyy + T(2) * exy * exy);
    sp[0] = P.lam * tr + T(2) * P.mu * exx;
    sp[1] = P.lam * tr + T(2) * P.mu * eyy;
    sp[2] = T(2) * P.mu * exy;
    sm[0] = sm[1] = sm[2] = T(0);
  } else if constexpr (S == SPLIT_SPECTRAL) {
    const T hd = T(0.5) * (exx - eyy);
    const T R2 = hd * hd + exy * exy;
    const T R = R2 > T(0) ? sqrt(R2) : T(0);
    const T e1 = T(0.5) * tr + R;
    const T e2 = T(0.5) * tr - R;
    T px, py, pxy;   // E+ = sum_a <e_a>+ n_a n_a'
    if (e2 >= T(0)) {
      px = exx, py = eyy, pxy = exy;
    } else if (e1 <= T(0)) {
      px = py = pxy = T(0);
    } else {
      const T f = e1 / (T(2) * R);
      px = f * (exx - e2);
      py = f * (eyy - e2);
      pxy = f * exy;
    }
    const T tp = posp(tr), tm = negp(tr);
    const T p1 = posp(e1), p2 = posp(e2);
    psi_p = T(0.5) * P.lam * tp * tp + P.mu * (p1 * p1 + p2 * p2);
    sp[0] = P.lam * tp + T(2) * P.mu * px;
    sp[1] = P.lam * tp + T(2) * P.mu * py;
    sp[2] = T(2) * P.mu * pxy;
    sm[0] = P.lam * tm + T(2) * P.mu * (exx - px);
    sm[1] = P.lam * tm + T(2) * P.mu * (eyy - py);
    sm[2] = T(2) * P.mu * (exy - pxy);
  } else {
    // vol-dev (gamma = 0) and star-convex
    const T tp = posp(tr), tm = negp(tr);
    const T dev = exx * exx + eyy * eyy + T(2) * exy * exy + P.coef * tr * tr;
    psi_p = T(0.5) * P.Kc2 * (tp * tp - P.gamma * tm * tm) + P.mu * dev;
    const T iso = P.Kc2 * (tp - P.gamma * tm) + T(2) * P.mu * P.coef * tr;
    sp[0] = iso + T(2) * P.mu * exx;
    sp[1] = iso + T(2) * P.mu * eyy;
    sp[2] = T(2) * P.mu * exy;
    const T im = (T(1) + P.gamma) * P.Kc2 * tm;
    sm[0] = im;
    sm[1] = im;
    sm[2] = T(0);
  }
}

// Reverse mode of  sigma = g sp(eps) + sm(eps)  and  psi+ (eps):
// given the adjoints sb (of sigma) and pb (of psi+), return the adjoint of
// eps in eb[3] (w.r.t. the independent components xx, yy, xy) and the
// adjoint of g.  Branch choices are those of split_eval.
template <int S, typename T>
__device__ __forceinline__ void split_vjp(T exx, T eyy, T exy, T g, const T sb[3], T pb, const InstP<T>& P,
                                          T eb[3], T& gb) {
  const T tr = exx + eyy;
  // adjoint of sp and sm
  const T spb[3] = {g * sb[0], g * sb[1], g * sb[2]};
  const T smb[3] = {sb[0], sb[1], sb[2]};
  if constexpr (S == SPLIT_NONE) {
    T psi_p, sp[3], sm[3];
    split_eval<S, T>(exx, eyy, exy, P, psi_p, sp, sm);
    gb = sb[0] * sp[0] + sb[1] * sp[1] + sb[2] * sp[2];
    // psi+ gradient w.r.t. (xx, yy, xy) is (sp0, sp1, 2 sp2)
    const T trb = P.lam * (spb[0] + spb[1]);
    eb[0] = trb + T(2) * P.mu * spb[0] + pb * sp[0];
    eb[1] = trb + T(2) * P.mu * spb[1] + pb * sp[1];
    eb[2] = T(2) * P.mu * spb[2] + pb * T(2) * sp[2];
  } else if constexpr (S == SPLIT_SPECTRAL) {
    const T hd = T(0.5) * (exx - eyy);
    const T R2 = hd * hd + exy * exy;
    const T R = R2 > T(0) ? sqrt(R2) : T(0);
    const T e1 = T(0.5) * tr + R;
    const T e2 = T(0.5) * tr - R;
    const int br = (e2 >= T(0)) ? 0 : ((e1 <= T(0)) ? 1 : 2);
    T px, py, pxy, f = T(0);
    if (br == 0) {
      px = exx, py = eyy, pxy = exy;
    } else if (br == 1) {
      px = py = pxy = T(0);
    } else {
      f = e1 / (T(2) * R);
      px = f * (exx - e2);
      py = f * (eyy - e2);
      pxy = f * exy;
    }
    const T tp = posp(tr), tm = negp(tr);
    const T p1 = posp(e1), p2 = posp(e2);
    // forward stresses for the adjoint of g
    const T sp0 = P.lam * tp + T(2) * P.mu * px, sp1 = P.lam * tp + T(2) * P.mu * py, sp2 = T(2) * P.mu * pxy;
    gb = sb[0] * sp0 + sb[1] * sp1 + sb[2] * sp2;
    // adjoints of E+ (px, py, pxy): from sp (2 mu) and from sm (-2 mu)
    const T Pb0 = T(2) * P.mu * (spb[0] - smb[0]);
    const T Pb1 = T(2) * P.mu * (spb[1] - smb[1]);
    const T Pb2 = T(2) * P.mu * (spb[2] - smb[2]);
    // direct eps adjoint from sm's (exx - px) terms
    T ex = T(2) * P.mu * smb[0], ey = T(2) * P.mu * smb[1], exyb = T(2) * P.mu * smb[2];
    // tr through <tr>+ and <tr>-: sp uses lam tp, sm uses lam tm; psi+ uses lam/2 tp^2
    T trb = P.lam * ((tr > T(0) ? (spb[0] + spb[1]) : T(0)) + (tr < T(0) ? (smb[0] + smb[1]) : T(0)));
    trb += pb * P.lam * tp;
    // psi+ eigen part: mu (p1^2 + p2^2)
    T e1b = pb * T(2) * P.mu * p1;
    T e2b = pb * T(2) * P.mu * p2;
    if (br == 0) {
      ex += Pb0, ey += Pb1, exyb += Pb2;
    } else if (br == 2) {
      // px = f (exx - e2), py = f (eyy - e2), pxy = f exy, f = e1 / (2R)
      const T fb = Pb0 * (exx - e2) + Pb1 * (eyy - e2) + Pb2 * exy;
      ex += f * Pb0;
      ey += f * Pb1;
      exyb += f * Pb2;
      e2b -= f * (Pb0 + Pb1);
      e1b += fb / (T(2) * R);
      const T Rb_f = -fb * e1 / (T(2) * R * R);
      // e1 = tr/2 + R, e2 = tr/2 - R
      trb += T(0.5) * (e1b + e2b);
      const T Rb = e1b - e2b + Rb_f;
      // R = sqrt(hd^2 + exy^2)
      ex += Rb * hd / R * T(0.5);
      ey -= Rb * hd / R * T(0.5);
      exyb += Rb * exy / R;
      e1b = e2b = T(0);
    }
    if (br != 2) {
      trb += T(0.5) * (e1b + e2b);
      if (R > T(0)) {
        const T Rb = e1b - e2b;
        ex += Rb * hd / R * T(0.5);
        ey -= Rb * hd / R * T(0.5);
        exyb += Rb * exy / R;
      }
    }
    eb[0] = ex + trb;
    eb[1] = ey + trb;
    eb[2] = exyb;
  } else {
    const T tp = posp(tr), tm = negp(tr);
    const T iso = P.Kc2 * (tp - P.gamma * tm) + T(2) * P.mu * P.coef * tr;
    const T sp0 = iso + T(2) * P.mu * exx, sp1 = iso + T(2) * P.mu * eyy, sp2 = T(2) * P.mu * exy;
    gb = sb[0] * sp0 + sb[1] * sp1 + sb[2] * sp2;
    const T isob = spb[0] + spb[1];
    const T imb = smb[0] + smb[1];
    // d iso / d tr = Kc2 (1[tr>0] - gamma 1[tr<0]) + 2 mu coef;  d im / d tr = (1+gamma) Kc2 1[tr<0]
    const T dtp = tr > T(0) ? T(1) : T(0), dtm = tr < T(0) ? T(1) : T(0);
    T trb = isob * (P.Kc2 * (dtp - P.gamma * dtm) + T(2) * P.mu * P.coef) + imb * (T(1) + P.gamma) * P.Kc2 * dtm;
    // psi+ = Kc2/2 (tp^2 - gamma tm^2) + mu (exx^2 + eyy^2 + 2 exy^2 + coef tr^2)
    trb += pb * (P.Kc2 * (tp - P.gamma * tm) + T(2) * P.mu * P.coef * tr);
    eb[0] = trb + T(2) * P.mu * spb[0] + pb * T(2) * P.mu * exx;
    eb[1] = trb + T(2) * P.mu * spb[1] + pb * T(2) * P.mu * eyy;
    eb[2] = T(2) * P.mu * spb[2] + pb * T(4) * P.mu * exy;
  }
}

}  // namespace pf
