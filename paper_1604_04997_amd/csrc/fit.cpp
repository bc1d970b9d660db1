// Relative-error least-squares fit of the model weights (Sec. 4.3), FP64,
// on the host.
//
// Rows are measured variants, columns their features; each row is divided
// by the variant's measured time, so minimising ||A alpha - 1||_2 minimises
// sum_j (1 - sum_i alpha_i f_ji / T_j)^2.  Columns that are zero in every
// row are left out (weight 0).  The kept columns are scaled to unit norm
// (the solution is unscaled afterwards) and factorised by Householder QR
// with column pivoting; the numerical rank is the number of pivots above
// max(m, p) * eps * |R_00|, and a rank-deficient system gets the basic
// solution on the leading pivots (predictions inside the column space do
// not depend on which least-squares solution is taken).
#include <cfloat>
#include <cmath>
#include <vector>

#include "pm.h"
#include "fit.h"
#include "desc.h"

namespace pm {

int fit_model(const pm_counts *P, const double *T, size_t m, uint32_t proj,
              pm_model *out, double *cond, double *resid, uint32_t *rank_out) {
    int nf = nfeat(proj);
    if (nf < 0 || m == 0 || !P || !T || !out) return PM_EINVAL;
    for (size_t j = 0; j < m; j++)
        if (!(T[j] > 0.0) || !std::isfinite(T[j])) return PM_EINVAL;
    std::vector<double> A(m * nf);
    for (size_t j = 0; j < m; j++) {
        double f[PM_NFEAT_MAX];
        features(P[j].c, proj, f);
        for (int i = 0; i < nf; i++) A[j * nf + i] = f[i] / T[j];
    }
    std::vector<int> keep;
    for (int i = 0; i < nf; i++) {
        bool nz = false;
        for (size_t j = 0; j < m && !nz; j++) nz = A[j * nf + i] != 0.0;
        if (nz) keep.push_back(i);
    }
    const int p = (int)keep.size();
    out->proj = proj;
    out->nfeat = (uint32_t)nf;
    for (int i = 0; i < PM_NFEAT_MAX; i++) out->alpha[i] = 0.0;
    if (p == 0) return PM_ERANK;

    // column-major working copy of the kept columns, unit-norm scaled
    std::vector<double> M((size_t)m * p), scale(p);
    for (int c = 0; c < p; c++) {
        double s = 0;
        for (size_t j = 0; j < m; j++) s += A[j * nf + keep[c]] * A[j * nf + keep[c]];
        scale[c] = std::sqrt(s);
        for (size_t j = 0; j < m; j++) M[(size_t)c * m + j] = A[j * nf + keep[c]] / scale[c];
    }
    std::vector<double> b(m, 1.0);
    std::vector<int> perm(p);
    for (int c = 0; c < p; c++) perm[c] = c;
    const int kmax = (int)(m < (size_t)p ? m : (size_t)p);
    std::vector<double> rdiag(kmax, 0.0);
    int k = 0;
    for (; k < kmax; k++) {
        // pivot: the remaining column with the largest norm below row k
        int best = k;
        double bn = -1;
        for (int c = k; c < p; c++) {
            double s = 0;
            for (size_t j = k; j < m; j++) s += M[(size_t)c * m + j] * M[(size_t)c * m + j];
            if (s > bn) {
                bn = s;
                best = c;
            }
        }
        if (best != k) {
            for (size_t j = 0; j < m; j++) std::swap(M[(size_t)k * m + j], M[(size_t)best * m + j]);
            std::swap(perm[k], perm[best]);
        }
        double *x = &M[(size_t)k * m];
        double nx = 0;
        for (size_t j = k; j < m; j++) nx += x[j] * x[j];
        nx = std::sqrt(nx);
        if (nx == 0.0) break;
        double alpha = x[k] > 0 ? -nx : nx;  // R_kk
        // v = x - alpha e_k, stored in place; H = I - 2 v v^T / (v^T v)
        x[k] -= alpha;
        double vtv = 0;
        for (size_t j = k; j < m; j++) vtv += x[j] * x[j];
        for (int c = k + 1; c < p; c++) {
            double *y = &M[(size_t)c * m];
            double d = 0;
            for (size_t j = k; j < m; j++) d += x[j] * y[j];
            d = 2.0 * d / vtv;
            for (size_t j = k; j < m; j++) y[j] -= d * x[j];
        }
        double d = 0;
        for (size_t j = k; j < m; j++) d += x[j] * b[j];
        d = 2.0 * d / vtv;
        for (size_t j = k; j < m; j++) b[j] -= d * x[j];
        rdiag[k] = alpha;
    }
    const int kk = k;
    int r = 0;
    const double tol = (double)(m > (size_t)p ? m : (size_t)p) * DBL_EPSILON *
                       (kk ? std::fabs(rdiag[0]) : 0.0);
    while (r < kk && std::fabs(rdiag[r]) > tol) r++;
    if (r == 0) return PM_ERANK;
    // back substitution on the leading r x r block: R_ij (i<j) lives in
    // column j rows above the diagonal; R_ii in rdiag
    std::vector<double> z(r);
    for (int i = r - 1; i >= 0; i--) {
        double s = b[i];
        for (int c = i + 1; c < r; c++) s -= M[(size_t)c * m + i] * z[c];
        z[i] = s / rdiag[i];
    }
    for (int i = 0; i < r; i++) out->alpha[keep[perm[i]]] = z[i] / scale[perm[i]];
    if (cond) *cond = std::fabs(rdiag[0]) / std::fabs(rdiag[r - 1]);
    if (rank_out) *rank_out = (uint32_t)r;
    if (resid)
        for (size_t j = 0; j < m; j++) {
            double f[PM_NFEAT_MAX];
            features(P[j].c, proj, f);
            double t = 0;
            for (int i = 0; i < nf; i++) t += out->alpha[i] * f[i];
            resid[j] = 1.0 - t / T[j];
        }
    return PM_OK;
}

}  // namespace pm
