/*
 * Plain FP64 CPU oracle of the Piacsek-Williams (PW) momentum-advection stencil.
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load or call this file.  It shares no code,
 * header, table or helper with the HIP library, and the HIP library never
 * calls it.
 *
 * What it computes (Brown, "Accelerating advection for atmospheric modelling
 * on Xilinx and Intel FPGAs", Sec. II-A):
 *
 *   su  Listing 1 exactly: an x flux term, a y flux term and a vertical term,
 *       for k = 2 .. nz, with the upper vertical flux dropped at k = nz.
 *   sv  not printed in the paper (it names the three source terms and counts
 *       21 operations per field, Sec. III).  Reading used here: the x<->y
 *       mirror of su on the same staggered (Arakawa C) grid that Listing 1's
 *       indices imply -- v sits on y faces, u on x faces, w on z faces, and
 *       each flux is (advected value at the neighbour) times (sum of the two
 *       advecting velocities that straddle the face).
 *   sw  not printed either; same staggering rule applied to w, with its own
 *       vertical coefficients tzd1, tzd2, for k = 2 .. nz-1.  sw(nz) = 0
 *       (rigid lid; w itself is 0 there).
 *   k = 1 is not computed by the paper's loop; this oracle writes 0 there for
 *   all three outputs so that every interior column is fully defined.
 *
 * Evaluation order is the textual order of Listing 1: each output is
 * accumulated as ((x-term + y-term) + lower vertical) - upper vertical, each
 * product is left-associated ((coef * a) * (b + c)), and the horizontal
 * coefficient multiplies the bracketed difference last.  sv accumulates its
 * own-direction (y) term first, mirroring su.  Build with -ffp-contract=off
 * (no fused multiply-add) so the order above is also the rounding order.
 *
 * Layout: element (k, j, i), k in 1..nz, j in 0..ny+1, i in 0..nx+1 (one-point
 * halo in x and y, none in z) lives at offset (k-1) + j*sy + i*sx.  Halo
 * columns of the inputs must be filled by the caller; halo columns of the
 * outputs are never written.
 */
#include <stddef.h>
#include <stdint.h>

#define AT(a, k, j, i) (a)[(ptrdiff_t)((k) - 1) + (ptrdiff_t)(j) * sy + (ptrdiff_t)(i) * sx]

/*
 * Returns 0 on success, -1 on an invalid shape (nx < 1, ny < 1, nz < 2, or
 * strides too small to hold the halo'd extents).  `nthreads` > 1 splits the
 * outer i loop over OpenMP threads when built with -fopenmp; the arithmetic of
 * every point is the same whatever the thread count.
 */
int pw_oracle_f64(int32_t nx, int32_t ny, int32_t nz, int64_t sy, int64_t sx,
                  const double *u, const double *v, const double *w,
                  double *su, double *sv, double *sw,
                  double tcx, double tcy,
                  const double *tzc1, const double *tzc2,
                  const double *tzd1, const double *tzd2,
                  int32_t nthreads)
{
    if (nx < 1 || ny < 1 || nz < 2 || sy < nz || sx < (int64_t)(ny + 2) * sy)
        return -1;
    (void)nthreads;
#ifdef _OPENMP
#pragma omp parallel for schedule(static) num_threads(nthreads > 0 ? nthreads : 1)
#endif
    for (int32_t i = 1; i <= nx; ++i) {
        for (int32_t j = 1; j <= ny; ++j) {
            AT(su, 1, j, i) = 0.0;
            AT(sv, 1, j, i) = 0.0;
            AT(sw, 1, j, i) = 0.0;
            for (int32_t k = 2; k <= nz; ++k) {
                double s;

                /* su: Listing 1. */
                s = tcx * (AT(u, k, j, i - 1) * (AT(u, k, j, i) + AT(u, k, j, i - 1))
                           - AT(u, k, j, i + 1) * (AT(u, k, j, i) + AT(u, k, j, i + 1)));
                s = s + tcy * (AT(u, k, j - 1, i) * (AT(v, k, j - 1, i) + AT(v, k, j - 1, i + 1))
                               - AT(u, k, j + 1, i) * (AT(v, k, j, i) + AT(v, k, j, i + 1)));
                if (k < nz)
                    s = s + tzc1[k - 1] * AT(u, k - 1, j, i) * (AT(w, k - 1, j, i) + AT(w, k - 1, j, i + 1))
                          - tzc2[k - 1] * AT(u, k + 1, j, i) * (AT(w, k, j, i) + AT(w, k, j, i + 1));
                else
                    s = s + tzc1[k - 1] * AT(u, k - 1, j, i) * (AT(w, k - 1, j, i) + AT(w, k - 1, j, i + 1));
                AT(su, k, j, i) = s;

                /* sv: x<->y mirror of su (own-direction y term first). */
                s = tcy * (AT(v, k, j - 1, i) * (AT(v, k, j, i) + AT(v, k, j - 1, i))
                           - AT(v, k, j + 1, i) * (AT(v, k, j, i) + AT(v, k, j + 1, i)));
                s = s + tcx * (AT(v, k, j, i - 1) * (AT(u, k, j, i - 1) + AT(u, k, j + 1, i - 1))
                               - AT(v, k, j, i + 1) * (AT(u, k, j, i) + AT(u, k, j + 1, i)));
                if (k < nz)
                    s = s + tzc1[k - 1] * AT(v, k - 1, j, i) * (AT(w, k - 1, j, i) + AT(w, k - 1, j + 1, i))
                          - tzc2[k - 1] * AT(v, k + 1, j, i) * (AT(w, k, j, i) + AT(w, k, j + 1, i));
                else
                    s = s + tzc1[k - 1] * AT(v, k - 1, j, i) * (AT(w, k - 1, j, i) + AT(w, k - 1, j + 1, i));
                AT(sv, k, j, i) = s;

                /* sw: w on z faces, advected by u, v (averaged to the face) and by w itself. */
                if (k < nz) {
                    s = tcx * (AT(w, k, j, i - 1) * (AT(u, k, j, i - 1) + AT(u, k + 1, j, i - 1))
                               - AT(w, k, j, i + 1) * (AT(u, k, j, i) + AT(u, k + 1, j, i)));
                    s = s + tcy * (AT(w, k, j - 1, i) * (AT(v, k, j - 1, i) + AT(v, k + 1, j - 1, i))
                                   - AT(w, k, j + 1, i) * (AT(v, k, j, i) + AT(v, k + 1, j, i)));
                    s = s + tzd1[k - 1] * AT(w, k - 1, j, i) * (AT(w, k, j, i) + AT(w, k - 1, j, i))
                          - tzd2[k - 1] * AT(w, k + 1, j, i) * (AT(w, k, j, i) + AT(w, k + 1, j, i));
                    AT(sw, k, j, i) = s;
                } else {
                    AT(sw, k, j, i) = 0.0;
                }
            }
        }
    }
    return 0;
}
