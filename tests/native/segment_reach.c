/* Test helper (not part of the library): which Gaussians can reach a segment.
 *
 * For segments from points c[k] to x, marks hit[k * n + i] = 1 when the sphere of radius r[i]
 * around mu[i] meets the segment (distance from mu[i] to the closest point of the segment
 * <= r[i]).  The parity tests use it to cut a scene down to the Gaussians that can contribute
 * to an opacity-field query along each view's ray, before the float64 oracle runs on that
 * sub-scene.  Plain double precision, one OpenMP thread per block of Gaussians. */
#include <stdint.h>

void segment_reach(const double* mu, const double* r, int64_t n, const double* c, const double* x, int32_t n_seg,
                   uint8_t* hit) {
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < n; ++i) {
    const double m0 = mu[3 * i], m1 = mu[3 * i + 1], m2 = mu[3 * i + 2], rr = r[i] * r[i];
    for (int32_t k = 0; k < n_seg; ++k) {
      const double s0 = x[0] - c[3 * k], s1 = x[1] - c[3 * k + 1], s2 = x[2] - c[3 * k + 2];
      const double q0 = m0 - c[3 * k], q1 = m1 - c[3 * k + 1], q2 = m2 - c[3 * k + 2];
      const double ss = s0 * s0 + s1 * s1 + s2 * s2;
      double t = ss > 0.0 ? (q0 * s0 + q1 * s1 + q2 * s2) / ss : 0.0;
      t = t < 0.0 ? 0.0 : (t > 1.0 ? 1.0 : t);
      const double d0 = q0 - t * s0, d1 = q1 - t * s1, d2 = q2 - t * s2;
      hit[(int64_t)k * n + i] = (d0 * d0 + d1 * d1 + d2 * d2) <= rr ? 1 : 0;
    }
  }
}
