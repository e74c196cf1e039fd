/* Brute-force neighborhoods (MLIP-3 paper, Sec. II.A) -- oracle side.
 *
 * TEST INFRASTRUCTURE ONLY: called from the Python oracle; the product
 * library never links or calls it.
 *
 * For every atom i: every atom j and every lattice translation n (integers,
 * zero along non-periodic axes) with 0 < |x_j + n H - x_i| < r_cut, where
 * the rows of H are the cell vectors.  For a pair (i, j) the admissible n_k
 * along a periodic axis are all integers with |s_j - s_i + n_k| <= r_cut/h_k
 * (s = fractional coordinates, h_k = cell height along axis k); every one of
 * them is tested, so positions need not lie inside the cell.
 * Output order: by i, then j, then n lexicographically.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>

static void inv3(const double *H, double *Hi) {
    double a = H[0], b = H[1], c = H[2], d = H[3], e = H[4], f = H[5], g = H[6], h = H[7], k = H[8];
    double det = a * (e * k - f * h) - b * (d * k - f * g) + c * (d * h - e * g);
    Hi[0] = (e * k - f * h) / det; Hi[1] = (c * h - b * k) / det; Hi[2] = (b * f - c * e) / det;
    Hi[3] = (f * g - d * k) / det; Hi[4] = (a * k - c * g) / det; Hi[5] = (c * d - a * f) / det;
    Hi[6] = (d * h - e * g) / det; Hi[7] = (b * g - a * h) / det; Hi[8] = (a * e - b * d) / det;
}

static double height(const double *H, int k) {
    const double *u = H + 3 * ((k + 1) % 3), *v = H + 3 * ((k + 2) % 3), *w = H + 3 * k;
    double cx = u[1] * v[2] - u[2] * v[1], cy = u[2] * v[0] - u[0] * v[2], cz = u[0] * v[1] - u[1] * v[0];
    double vol = fabs(w[0] * cx + w[1] * cy + w[2] * cz);
    return vol / sqrt(cx * cx + cy * cy + cz * cz);
}

/* Scans atom i; if out_j != NULL writes up to cap pairs; returns the count. */
static int64_t scan_atom(int64_t n, const double *pos, const double *H, const double *Hi,
                         const int *pbc, double r_cut, int64_t i,
                         int32_t *out_j, int32_t *out_shift, int64_t cap) {
    double hk[3], si[3];
    for (int k = 0; k < 3; ++k) hk[k] = height(H, k);
    for (int k = 0; k < 3; ++k)
        si[k] = pos[3 * i] * Hi[k] + pos[3 * i + 1] * Hi[3 + k] + pos[3 * i + 2] * Hi[6 + k];
    int64_t cnt = 0;
    for (int64_t j = 0; j < n; ++j) {
        long lo[3], hi[3];
        for (int k = 0; k < 3; ++k) {
            double sj = pos[3 * j] * Hi[k] + pos[3 * j + 1] * Hi[3 + k] + pos[3 * j + 2] * Hi[6 + k];
            double d = sj - si[k];
            if (pbc[k]) {
                lo[k] = (long)ceil(-d - r_cut / hk[k]) - 1;
                hi[k] = (long)floor(-d + r_cut / hk[k]) + 1;
            } else {
                lo[k] = hi[k] = 0;
            }
        }
        for (long a = lo[0]; a <= hi[0]; ++a)
            for (long b = lo[1]; b <= hi[1]; ++b)
                for (long c = lo[2]; c <= hi[2]; ++c) {
                    if (j == i && a == 0 && b == 0 && c == 0) continue;
                    double r[3], rr = 0.0;
                    for (int k = 0; k < 3; ++k) {
                        r[k] = pos[3 * j + k] + a * H[k] + b * H[3 + k] + c * H[6 + k] - pos[3 * i + k];
                        rr += r[k] * r[k];
                    }
                    if (sqrt(rr) < r_cut) {
                        if (out_j && cnt < cap) {
                            out_j[cnt] = (int32_t)j;
                            out_shift[3 * cnt] = (int32_t)a;
                            out_shift[3 * cnt + 1] = (int32_t)b;
                            out_shift[3 * cnt + 2] = (int32_t)c;
                        }
                        ++cnt;
                    }
                }
    }
    return cnt;
}

/* Counts per atom (counts[n]); returns the total. */
int64_t oracle_nbr_count(int64_t n, const double *pos, const double *cell, const int *pbc,
                         double r_cut, int64_t *counts) {
    double Hi[9];
    inv3(cell, Hi);
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 16) reduction(+ : total)
    for (int64_t i = 0; i < n; ++i) {
        counts[i] = scan_atom(n, pos, cell, Hi, pbc, r_cut, i, NULL, NULL, 0);
        total += counts[i];
    }
    return total;
}

/* Fills pairs; offsets[n+1] is the exclusive scan of the counts. */
void oracle_nbr_fill(int64_t n, const double *pos, const double *cell, const int *pbc,
                     double r_cut, const int64_t *offsets, int32_t *out_j, int32_t *out_shift) {
    double Hi[9];
    inv3(cell, Hi);
#pragma omp parallel for schedule(dynamic, 16)
    for (int64_t i = 0; i < n; ++i)
        scan_atom(n, pos, cell, Hi, pbc, r_cut, i, out_j + offsets[i], out_shift + 3 * offsets[i],
                  offsets[i + 1] - offsets[i]);
}

/* Neighbors of selected atoms only (for spot checks in large systems). */
int64_t oracle_nbr_count_sel(int64_t n, const double *pos, const double *cell, const int *pbc,
                             double r_cut, int64_t n_sel, const int64_t *sel, int64_t *counts) {
    double Hi[9];
    inv3(cell, Hi);
    int64_t total = 0;
#pragma omp parallel for schedule(dynamic, 4) reduction(+ : total)
    for (int64_t s = 0; s < n_sel; ++s) {
        counts[s] = scan_atom(n, pos, cell, Hi, pbc, r_cut, sel[s], NULL, NULL, 0);
        total += counts[s];
    }
    return total;
}

void oracle_nbr_fill_sel(int64_t n, const double *pos, const double *cell, const int *pbc,
                         double r_cut, int64_t n_sel, const int64_t *sel, const int64_t *offsets,
                         int32_t *out_j, int32_t *out_shift) {
    double Hi[9];
    inv3(cell, Hi);
#pragma omp parallel for schedule(dynamic, 4)
    for (int64_t s = 0; s < n_sel; ++s)
        scan_atom(n, pos, cell, Hi, pbc, r_cut, sel[s], out_j + offsets[s], out_shift + 3 * offsets[s],
                  offsets[s + 1] - offsets[s]);
}
