/* Oracle direct sums (test infrastructure; FP64, plain loops).
 *
 * oracle_near_traction: the near-image single-layer traction sum of the
 * periodic Green's function split (Sec. 4.2, definition of G_near, with the
 * 3x3 image set of every particle) evaluated with the traction kernel
 * G^t(x,y;n) = -(1/pi) r r^T (r.n) / |r|^4, r = x - y (Sec. 4.1, eq. Gt):
 *
 *   T(x_i) = sum_j sum_s G^t(x_i, y_j + s; n_i) f_j,    skipping j == self[i] for s == (0,0)
 *
 * Targets are shifted instead of sources: G^t(x, y+s) = G^t(x-s, y).
 * No blocking, no reordering beyond the plain loops; OpenMP over targets only.
 */
#include <stdint.h>
#include <math.h>

void oracle_near_traction(int64_t nt, const double* x1, const double* x2,
                          const double* n1, const double* n2,
                          int64_t ns, const double* y1, const double* y2,
                          const double* f1, const double* f2,
                          int32_t nshift, const double* s1, const double* s2,
                          const int64_t* self_idx, double* t1, double* t2)
{
    const double c = -1.0 / M_PI;
    #pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < nt; ++i) {
        double a1 = 0.0, a2 = 0.0;
        for (int32_t s = 0; s < nshift; ++s) {
            const int zero_shift = (s1[s] == 0.0 && s2[s] == 0.0);
            const double xs1 = x1[i] - s1[s], xs2 = x2[i] - s2[s];
            for (int64_t j = 0; j < ns; ++j) {
                if (zero_shift && self_idx != 0 && j == self_idx[i]) continue;
                const double r1 = xs1 - y1[j], r2 = xs2 - y2[j];
                const double rr = r1 * r1 + r2 * r2;
                const double rn = r1 * n1[i] + r2 * n2[i];
                const double rf = r1 * f1[j] + r2 * f2[j];
                const double k = c * rn * rf / (rr * rr);
                a1 += k * r1;
                a2 += k * r2;
            }
        }
        t1[i] = a1;
        t2[i] = a2;
    }
}

/* Stokeslet velocity and vorticity at targets from point forces f_j at the
 * shifted sources y_j + s (Sec. 4.1 eq. Gv; the vorticity of G f is
 * -(r1 f2 - r2 f1) / (2 pi mu |r|^2)). No self-skip: used for targets off the
 * source set only.
 */
void oracle_stokeslet_velocity(int64_t nt, const double* x1, const double* x2,
                               int64_t ns, const double* y1, const double* y2,
                               const double* f1, const double* f2,
                               int32_t nshift, const double* s1, const double* s2,
                               double mu, double* u1, double* u2, double* vort)
{
    const double cu = 1.0 / (4.0 * M_PI * mu);
    const double cw = -1.0 / (2.0 * M_PI * mu);
    #pragma omp parallel for schedule(dynamic, 4)
    for (int64_t i = 0; i < nt; ++i) {
        double a1 = 0.0, a2 = 0.0, aw = 0.0;
        for (int32_t s = 0; s < nshift; ++s) {
            const double xs1 = x1[i] - s1[s], xs2 = x2[i] - s2[s];
            for (int64_t j = 0; j < ns; ++j) {
                const double r1 = xs1 - y1[j], r2 = xs2 - y2[j];
                const double rr = r1 * r1 + r2 * r2;
                const double rf = r1 * f1[j] + r2 * f2[j];
                const double lg = -0.5 * log(rr);
                a1 += cu * (lg * f1[j] + r1 * rf / rr);
                a2 += cu * (lg * f2[j] + r2 * rf / rr);
                aw += cw * (r1 * f2[j] - r2 * f1[j]) / rr;
            }
        }
        u1[i] = a1;
        u2[i] = a2;
        vort[i] = aw;
    }
}
