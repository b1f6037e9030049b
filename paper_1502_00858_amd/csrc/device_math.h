// Small FP64 device helpers shared by several kernel files.
#pragma once

#include <hip/hip_runtime.h>

namespace calib {

// Unitary polar factor of a 2x2 complex matrix in closed form: with A = W S V^H and
// e^{i phi} = det A / |det A|, A + e^{i phi} adj(A)^H = (s1 + s2) W V^H.
__device__ inline void polar2(const double *a, double *u) {
  const double ar = a[0], ai = a[1], br = a[2], bi = a[3], cr = a[4], ci = a[5], dr = a[6], di = a[7];
  double detr = ar * dr - ai * di - (br * cr - bi * ci);
  double deti = ar * di + ai * dr - (br * ci + bi * cr);
  const double dn = sqrt(detr * detr + deti * deti);
  double er = 1.0, ei = 0.0;
  if (dn > 0.0) { er = detr / dn; ei = deti / dn; }
  // adj(A)^H = [[conj d, -conj c], [-conj b, conj a]]
  const double hr[4] = {dr, -cr, -br, ar}, hi[4] = {-di, ci, bi, -ai};
  double m[8];
  const double src[8] = {ar, ai, br, bi, cr, ci, dr, di};
  double s = 0.0;
  for (int e = 0; e < 4; ++e) {
    m[2 * e] = src[2 * e] + er * hr[e] - ei * hi[e];
    m[2 * e + 1] = src[2 * e + 1] + er * hi[e] + ei * hr[e];
    s += m[2 * e] * m[2 * e] + m[2 * e + 1] * m[2 * e + 1];
  }
  const double scale = (s > 0.0) ? sqrt(2.0 / s) : 0.0;
  for (int e = 0; e < 8; ++e) u[e] = m[e] * scale;
}

}  // namespace calib
