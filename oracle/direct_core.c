/* Oracle direct-summation core (TEST INFRASTRUCTURE ONLY).
 *
 * Plain FP64 loops for one patch of the product-convolution sum (eq. (2.5))
 * and of its adjoint (eq. (1.6)).  Arrays are row-major boxes in up to three
 * dimensions; unused trailing axes have extent 1.  No FFT, no blocking: every
 * output is the straight sum over the kernel offsets in ascending row-major
 * order.  OpenMP splits the independent output points across threads.
 */
#include <stdint.h>

/* out[y] += sum_x t[x] * K[y - x]  for the output points y of a window
 *   t   : input box of extent m[3] starting at Omega point tlo[3]
 *   K   : kernel box of extent kn[3] starting at offset zlo[3]
 *   out : the window of Omega starting at olo[3] with extent on[3]
 *         (the whole domain: olo = 0, on = n)
 * Every output point of the window reached by (t box + K box) is visited
 * once. */
void oracle_conv_add(const double* t, const int64_t* tlo, const int64_t* m,
                     const double* K, const int64_t* zlo, const int64_t* kn,
                     double* out, const int64_t* olo, const int64_t* on)
{
    int64_t ylo[3], yhi[3];
    for (int i = 0; i < 3; ++i) {
        ylo[i] = tlo[i] + zlo[i];
        yhi[i] = tlo[i] + m[i] - 1 + zlo[i] + kn[i] - 1;
        if (ylo[i] < olo[i]) ylo[i] = olo[i];
        if (yhi[i] > olo[i] + on[i] - 1) yhi[i] = olo[i] + on[i] - 1;
        if (ylo[i] > yhi[i]) return;
    }
    #pragma omp parallel for collapse(2) schedule(static)
    for (int64_t y0 = ylo[0]; y0 <= yhi[0]; ++y0)
    for (int64_t y1 = ylo[1]; y1 <= yhi[1]; ++y1)
    for (int64_t y2 = ylo[2]; y2 <= yhi[2]; ++y2) {
        double s = 0.0;
        for (int64_t z0 = 0; z0 < kn[0]; ++z0) {
            int64_t x0 = y0 - (zlo[0] + z0) - tlo[0];
            if (x0 < 0 || x0 >= m[0]) continue;
            for (int64_t z1 = 0; z1 < kn[1]; ++z1) {
                int64_t x1 = y1 - (zlo[1] + z1) - tlo[1];
                if (x1 < 0 || x1 >= m[1]) continue;
                for (int64_t z2 = 0; z2 < kn[2]; ++z2) {
                    int64_t x2 = y2 - (zlo[2] + z2) - tlo[2];
                    if (x2 < 0 || x2 >= m[2]) continue;
                    s += t[(x0 * m[1] + x1) * m[2] + x2] * K[(z0 * kn[1] + z1) * kn[2] + z2];
                }
            }
        }
        out[((y0 - olo[0]) * on[1] + (y1 - olo[1])) * on[2] + (y2 - olo[2])] += s;
    }
}

/* c[x] = sum_z K[z] * g[x + z] over x + z in Omega, for x in the box
 * starting at tlo with extent m. */
void oracle_corr(const double* g, const int64_t* n,
                 const double* K, const int64_t* zlo, const int64_t* kn,
                 double* c, const int64_t* tlo, const int64_t* m)
{
    #pragma omp parallel for collapse(2) schedule(static)
    for (int64_t x0 = 0; x0 < m[0]; ++x0)
    for (int64_t x1 = 0; x1 < m[1]; ++x1)
    for (int64_t x2 = 0; x2 < m[2]; ++x2) {
        double s = 0.0;
        for (int64_t z0 = 0; z0 < kn[0]; ++z0) {
            int64_t y0 = tlo[0] + x0 + zlo[0] + z0;
            if (y0 < 0 || y0 >= n[0]) continue;
            for (int64_t z1 = 0; z1 < kn[1]; ++z1) {
                int64_t y1 = tlo[1] + x1 + zlo[1] + z1;
                if (y1 < 0 || y1 >= n[1]) continue;
                for (int64_t z2 = 0; z2 < kn[2]; ++z2) {
                    int64_t y2 = tlo[2] + x2 + zlo[2] + z2;
                    if (y2 < 0 || y2 >= n[2]) continue;
                    s += K[(z0 * kn[1] + z1) * kn[2] + z2] * g[(y0 * n[1] + y1) * n[2] + y2];
                }
            }
        }
        c[(x0 * m[1] + x1) * m[2] + x2] = s;
    }
}
