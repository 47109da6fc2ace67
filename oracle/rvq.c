/*
 * Oracle for residual vector quantization (R-VQ), Sec. 3.4 eqs. (14)-(15).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
 * benchmark's CPU-baseline leg may load this file's library.  It shares no
 * code with the HIP path.
 *
 * eq. (14): stage l picks, for each vector x_n, the code of C^l nearest to the
 *   residual r^l_n = x_n - xhat^{l-1}_n, where xhat^l_n = sum_{k<=l} C^k[i^k_n]
 *   and xhat^0 = 0.  The stages run in order: each residual depends on the
 *   codes picked before it.
 * eq. (15): L = 1/(N P) sum_l sum_n || sg[r^l_n] - C^l[i^l_n] ||^2, P the
 *   codebook size; sg stops the gradient, so only the codes receive one:
 *   dL/dC^l[k] = 2/(N P) sum_{n : i^l_n = k} (C^l[k] - r^l_n).
 *
 * The argmin decides an integer, so it is taken in binary32, in the order the
 * kernel uses (readings in the design notes):
 *   |c|^2  = c_0*c_0, then fmaf(c_j, c_j, .) for j = 1..D-1;
 *   e_k    = |c_k|^2, then fmaf(-2 c_kj, r_j, .) for j = 0..D-1
 *            (|c - r|^2 less the constant |r|^2);
 *   i      = the first k with the smallest e_k;
 *   xhat_j = xhat_j + c_ij and r_j = x_j - xhat_j, both in binary32.
 * Everything that reaches the loss and the code gradient is binary64 from
 * those binary32 residuals and codes.
 *
 * Build: gcc -O2 -ffp-contract=off -fno-fast-math -shared -fPIC.
 */
#include <math.h>
#include <stdint.h>
#include <string.h>

static float code_norm2(const float* c, int dim)
{
    float s = c[0] * c[0];
    for (int j = 1; j < dim; ++j) s = fmaf(c[j], c[j], s);
    return s;
}

/*
 * books  [stages][codes][dim] binary32
 * x      [n][dim] binary32
 * idx    [stages][n] out
 * recon  [n][dim] out: xhat after the last stage
 * loss   out: eq. (15)
 * dbooks [stages][codes][dim] out (overwritten): dL/dC
 */
void orc_rvq(int64_t n, int dim, int stages, int codes, const float* books, const float* x, int32_t* idx,
             float* recon, double* loss, double* dbooks)
{
    float xhat[64], r[64];
    double total = 0.0;
    memset(dbooks, 0, sizeof(double) * (size_t)stages * codes * dim);
    for (int64_t v = 0; v < n; ++v) {
        const float* xv = x + v * dim;
        for (int j = 0; j < dim; ++j) xhat[j] = 0.0f;
        for (int l = 0; l < stages; ++l) {
            const float* C = books + (size_t)l * codes * dim;
            for (int j = 0; j < dim; ++j) r[j] = xv[j] - xhat[j];
            int best = 0;
            float best_e = 0.0f;
            for (int k = 0; k < codes; ++k) {
                const float* c = C + (size_t)k * dim;
                float e = code_norm2(c, dim);
                for (int j = 0; j < dim; ++j) e = fmaf(-2.0f * c[j], r[j], e);
                if (k == 0 || e < best_e) {
                    best = k;
                    best_e = e;
                }
            }
            idx[(size_t)l * n + v] = best;
            const float* c = C + (size_t)best * dim;
            double* g = dbooks + ((size_t)l * codes + best) * dim;
            for (int j = 0; j < dim; ++j) {
                const double d = (double)r[j] - (double)c[j];
                total += d * d;
                g[j] -= 2.0 * d;
                xhat[j] = xhat[j] + c[j];
            }
        }
        for (int j = 0; j < dim; ++j) recon[v * dim + j] = xhat[j];
    }
    const double scale = (n > 0) ? 1.0 / ((double)n * codes) : 0.0;
    *loss = total * scale;
    for (size_t i = 0; i < (size_t)stages * codes * dim; ++i) dbooks[i] *= scale;
}
