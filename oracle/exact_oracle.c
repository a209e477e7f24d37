/*
 * EXACT CPU oracle -- TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT.
 *
 * Only the tests, the smoke check and the benchmark's CPU-baseline leg may
 * load or call this library.  It shares no source, header or table with the
 * HIP implementation under paper_2503_19925_amd/.
 *
 * A plain, slow, obviously correct implementation of what the hot path of
 * EXACT computes (Lou, Verchand, Fridovich-Keil, Pananjady, "Accurate,
 * provable and fast polychromatic tomographic reconstruction: a variational
 * inequality approach", arXiv 2503.19925).  Citations below name the paper's
 * section and equation label.
 *
 * Definitions implemented (all loops, no blocking or reordering):
 *
 *  Geometry.  N x N square image of pixels of side dpix centred at the
 *  origin; pixel (iy, ix) (iy = 0 the bottom row, p = iy*N + ix) has centre
 *  ((ix-c) dpix, (iy-c) dpix), c = (N-1)/2.  Parallel beam: view v at angle
 *  theta_v = half_turns*pi*v/V; detector bin b at u_b = (b-(B-1)/2) dbin; ray
 *  i = v*B + b is the line {p : p . (cos theta, sin theta) = u_b}.  The paper
 *  only asks for nonnegative entries derived from the Radon transform
 *  (Sec. 1, forward model eq. referenceforwardmodel and its bullet list on
 *  A_{i,k}); the projector is Joseph's: rows of A hold linear-interpolation
 *  (tent) weights on the image lines crossed by the ray, scaled by the path
 *  length per line, dpix/|cos| for row-stepping views (|cos| >= |sin|, ties
 *  at 45 and 135 degrees broken by an integer test) and dpix/|sin| otherwise.
 *  Pixels outside the image contribute nothing.
 *
 *  Spectral model (Sec. 1, eq. model:multi-material with M = 1; Sec. 1.2,
 *  eq. model-pre and eq. function-h-plus).  With I[j][k] = Ibar_j s_{jk}
 *  (window j, energy bin k) the expected counts on ray i are
 *  sum_k I[j][k] exp(-mu_k max(<a_i,x>, 0)).
 *
 *  Known materials (appendix, model underlying the experiment in the
 *  introduction's figure): when the other materials of the scan are known,
 *  with line integral bg_i on ray i, each ray gets the reparametrised window
 *  spectrum Ibar'_ij = sum_k I[j][k] exp(-mu_k bg_i), s'_ijk = I[j][k]
 *  exp(-mu_k bg_i) / Ibar'_ij, and the single-material model applies with
 *  those.  Every entry point below takes bg as an optional argument.
 *
 *  Operator (Sec. 1.2, eq. operator, summed over windows as in the
 *  multi-window model): F(x) = (1/n) sum_i [sum_j y[j][i] - sum_j sum_k
 *  I[j][k] exp(-mu_k <a_i,x>_+)] a_i = (1/n) A^T r, n = number of rays.
 *
 *  Projected extragradient (Sec. 1.2, eq. extragrad-method), with the
 *  projection onto the nonnegative orthant of Sec. 3.1 (keep positive
 *  entries, zero the rest).  Both half-steps start from x_t.
 *
 *  Averaged iterate and stopping rule of the experiments (Sec. 5,
 *  comparison of methods): xbar_s is the mean of x_j over the last half of
 *  the indices, j = floor(s/2)+1 .. s; the run stops at the first s with
 *  ||xbar_s - xbar_{s-1}||_2 <= tol and reports xbar_s.
 *
 *  Constraint set of the experiments (Sec. 5): X = TV ball intersected with
 *  the orthant.  TV is the isotropic total variation with forward
 *  differences; the TV-ball projection is approximated by the
 *  TV-regularized point (eq. TV-regularization) whose weight is found by
 *  binary search to |TV - tau| <= tv_tol, the regularized point itself by
 *  the fast gradient projection method on the dual of TV denoising (Beck and
 *  Teboulle 2009) with a fixed number of steps; the intersection by
 *  Dykstra's algorithm (eq. projection-intersection).
 *
 *  Dense measurements (the Gaussian measurement model, Sec. 2.2, and its
 *  experiment in Sec. 5): the same model and operator with an explicit
 *  matrix A of n rows a_i; EG over a ball centred at the origin (the
 *  bounded set of Assumption assump-X) or the whole space.
 *
 *  Step size (Theorem 2, Sec. 2.1; Lipschitz bound in Sec. 4.2):
 *  L <= lambda_max(Sigma) * sum_k J_k mu_k with Sigma = A^T A / n and
 *  J_k = sum_j I[j][k]; gamma = c / L.  lambda_max comes from ora_power.
 *
 * The same text is compiled for REAL = double (the oracle), long double (its
 * own rounding error) and float (the inherent single-precision sensitivity),
 * with suffixes _f64, _ld and _f32.  Every array crossing the interface is
 * double; conversion happens on entry and exit only.
 */
#include <stdlib.h>
#include <tgmath.h>

typedef struct {
    int n_pix, n_views, n_bins, half_turns;
    double pixel_cm, bin_cm;
} ora_geom;

#define ORA_PI 3.14159265358979323846264338327950288L

#define REAL double
#define FN(name) name##_f64
#include "exact_oracle_impl.h"
#undef REAL
#undef FN

#define REAL long double
#define FN(name) name##_ld
#include "exact_oracle_impl.h"
#undef REAL
#undef FN

#define REAL float
#define FN(name) name##_f32
#include "exact_oracle_impl.h"
#undef REAL
#undef FN
