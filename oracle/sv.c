/* FP64 state-vector kernels for the oracle (test infrastructure only).
 *
 * Paper Sec. 2.2: the state-vector method tracks all 2^n amplitudes and
 * applies each gate in circuit order.  Storage: 2^n complex doubles, real and
 * imaginary parts interleaved.  Qubit q is bit (n-1-q) of the index
 * (qubit 0 is the most significant bit).
 *
 * Each routine is the plain definition: for every group of amplitudes that
 * differ only in the gate's qubits, multiply that small vector by the gate
 * matrix.  OpenMP splits the groups across threads; every output element is
 * computed by exactly one thread from the same operands, so results do not
 * depend on the thread count.
 */
#include <stdint.h>
#include <string.h>

static inline int64_t insert_zero(int64_t k, int pos) {
    int64_t lo = k & ((((int64_t)1) << pos) - 1);
    return ((k >> pos) << (pos + 1)) | lo;
}

void sv_zero_state(double *psi, int n) {
    int64_t len = ((int64_t)2) << n;
    memset(psi, 0, (size_t)len * sizeof(double));
    psi[0] = 1.0;
}

/* m: 2x2 complex row-major, interleaved (re, im). */
void sv_apply_1q(double *psi, int n, int q, const double *m) {
    int pos = n - 1 - q;
    int64_t bit = ((int64_t)1) << pos;
    int64_t half = ((int64_t)1) << (n - 1);
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < half; k++) {
        int64_t i0 = insert_zero(k, pos), i1 = i0 | bit;
        double ar = psi[2 * i0], ai = psi[2 * i0 + 1];
        double br = psi[2 * i1], bi = psi[2 * i1 + 1];
        psi[2 * i0]     = m[0] * ar - m[1] * ai + m[2] * br - m[3] * bi;
        psi[2 * i0 + 1] = m[0] * ai + m[1] * ar + m[2] * bi + m[3] * br;
        psi[2 * i1]     = m[4] * ar - m[5] * ai + m[6] * br - m[7] * bi;
        psi[2 * i1 + 1] = m[4] * ai + m[5] * ar + m[6] * bi + m[7] * br;
    }
}

/* m: 4x4 complex row-major in the basis |q1 q2> (q1 most significant). */
void sv_apply_2q(double *psi, int n, int q1, int q2, const double *m) {
    int p1 = n - 1 - q1, p2 = n - 1 - q2;
    int plo = p1 < p2 ? p1 : p2, phi = p1 < p2 ? p2 : p1;
    int64_t b1 = ((int64_t)1) << p1, b2 = ((int64_t)1) << p2;
    int64_t quarter = ((int64_t)1) << (n - 2);
    #pragma omp parallel for schedule(static)
    for (int64_t k = 0; k < quarter; k++) {
        int64_t base = insert_zero(insert_zero(k, plo), phi);
        int64_t idx[4] = {base, base | b2, base | b1, base | b1 | b2};
        double vr[4], vi[4];
        for (int a = 0; a < 4; a++) { vr[a] = psi[2 * idx[a]]; vi[a] = psi[2 * idx[a] + 1]; }
        for (int r = 0; r < 4; r++) {
            double sr = 0.0, si = 0.0;
            for (int c = 0; c < 4; c++) {
                double mr = m[2 * (4 * r + c)], mi = m[2 * (4 * r + c) + 1];
                sr += mr * vr[c] - mi * vi[c];
                si += mr * vi[c] + mi * vr[c];
            }
            psi[2 * idx[r]] = sr;
            psi[2 * idx[r] + 1] = si;
        }
    }
}

/* out[j] = psi[index[j]] (complex). */
void sv_gather(const double *psi, int64_t count, const int64_t *index, double *out) {
    for (int64_t j = 0; j < count; j++) {
        out[2 * j] = psi[2 * index[j]];
        out[2 * j + 1] = psi[2 * index[j] + 1];
    }
}
