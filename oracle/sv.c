/* Plain FP64 Schroedinger-style statevector core (oracle; test-only).
 *
 * Sec. II-A of the paper: a state of n qubits is an array of 2^n complex
 * amplitudes with index i = sum_q i_q 2^q, and a gate is applied as a
 * matrix-vector product on the amplitudes that differ only in the gate's
 * qubits.  One gate per pass, no fusion, no blocking.
 *
 * Matrices are row-major 2^k x 2^k complex128; the gate's qubit q[0] is the
 * most significant bit of the matrix index.  Matrices need not be unitary
 * (Schmidt factors are not).
 */
#include <complex.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* Insert a zero bit at each of the (ascending) positions in pos[0..k). */
static inline uint64_t spread(uint64_t r, const int *pos_sorted, int k) {
    for (int j = 0; j < k; ++j) {
        uint64_t low = r & ((1ull << pos_sorted[j]) - 1ull);
        r = ((r >> pos_sorted[j]) << (pos_sorted[j] + 1)) | low;
    }
    return r;
}

int sv_apply(cplx *psi, int n, const int *q, int k, const cplx *m) {
    if (k < 1 || k > 8 || k > n) return -1;
    int sorted[8];
    for (int j = 0; j < k; ++j) {
        if (q[j] < 0 || q[j] >= n) return -2;
        sorted[j] = q[j];
    }
    for (int a = 0; a < k; ++a)
        for (int b = a + 1; b < k; ++b)
            if (sorted[b] < sorted[a]) { int t = sorted[a]; sorted[a] = sorted[b]; sorted[b] = t; }
    for (int j = 1; j < k; ++j)
        if (sorted[j] == sorted[j - 1]) return -3;
    const int64_t d = 1ll << k;
    const int64_t groups = 1ll << (n - k);
#pragma omp parallel for schedule(static)
    for (int64_t g = 0; g < groups; ++g) {
        uint64_t base = spread((uint64_t)g, sorted, k);
        uint64_t idx[256];
        cplx v[256];
        for (int64_t j = 0; j < d; ++j) {
            uint64_t x = base;
            for (int b = 0; b < k; ++b)
                if ((j >> (k - 1 - b)) & 1) x |= 1ull << q[b];
            idx[j] = x;
            v[j] = psi[x];
        }
        for (int64_t i = 0; i < d; ++i) {
            cplx s = 0;
            for (int64_t j = 0; j < d; ++j) s += m[i * d + j] * v[j];
            psi[idx[i]] = s;
        }
    }
    return 0;
}

/* out = <l| (m on qubits q) |r> = sum_x conj(l[x]) (M r)[x] (the plain
 * definition of a matrix element between two states, Sec. II-A indexing),
 * one read-only pass over both states: the adjoint gradient's inner product
 * without a temporary copy of the state. */
int sv_braket(const cplx *l, const cplx *r, int n, const int *q, int k, const cplx *m, double *out) {
    if (k < 1 || k > 8 || k > n) return -1;
    int sorted[8];
    for (int j = 0; j < k; ++j) {
        if (q[j] < 0 || q[j] >= n) return -2;
        sorted[j] = q[j];
    }
    for (int a = 0; a < k; ++a)
        for (int b = a + 1; b < k; ++b)
            if (sorted[b] < sorted[a]) { int t = sorted[a]; sorted[a] = sorted[b]; sorted[b] = t; }
    for (int j = 1; j < k; ++j)
        if (sorted[j] == sorted[j - 1]) return -3;
    const int64_t d = 1ll << k;
    const int64_t groups = 1ll << (n - k);
    double re = 0.0, im = 0.0;
#pragma omp parallel for schedule(static) reduction(+:re, im)
    for (int64_t g = 0; g < groups; ++g) {
        uint64_t base = spread((uint64_t)g, sorted, k);
        uint64_t idx[256];
        cplx v[256];
        for (int64_t j = 0; j < d; ++j) {
            uint64_t x = base;
            for (int b = 0; b < k; ++b)
                if ((j >> (k - 1 - b)) & 1) x |= 1ull << q[b];
            idx[j] = x;
            v[j] = r[x];
        }
        for (int64_t i = 0; i < d; ++i) {
            cplx s = 0;
            for (int64_t j = 0; j < d; ++j) s += m[i * d + j] * v[j];
            cplx t = conj(l[idx[i]]) * s;
            re += creal(t);
            im += cimag(t);
        }
    }
    out[0] = re;
    out[1] = im;
    return 0;
}

/* Apply a list of gates in order.  qs holds the qubits of all gates back to
 * back, ks their sizes, moff the offset of each matrix in mats. */
int sv_run(cplx *psi, int n, int64_t n_ops, const int *qs, const int *ks,
           const int64_t *moff, const cplx *mats) {
    int64_t qo = 0;
    for (int64_t g = 0; g < n_ops; ++g) {
        int rc = sv_apply(psi, n, qs + qo, ks[g], mats + moff[g]);
        if (rc) return rc;
        qo += ks[g];
    }
    return 0;
}

/* Run the same op list on `count` independent states of n qubits laid out
 * back to back (paths of a plain HSF are independent, Sec. II-B).  Each op
 * may carry several matrices; op g uses matrix sel[s * n_ops + g] for state s
 * (an index into mats via moff), so factor slots pick their Schmidt term. */
int sv_run_many(cplx *psi, int n, int64_t count, int64_t n_ops, const int *qs, const int *ks,
                const int64_t *moff, const int64_t *sel, const cplx *mats) {
    int rc_all = 0;
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t s = 0; s < count; ++s) {
        cplx *st = psi + (s << n);
        int64_t qo = 0;
        for (int64_t g = 0; g < n_ops; ++g) {
            int k = ks[g];
            int sorted[8];
            for (int j = 0; j < k; ++j) sorted[j] = qs[qo + j];
            for (int a = 0; a < k; ++a)
                for (int b = a + 1; b < k; ++b)
                    if (sorted[b] < sorted[a]) { int t = sorted[a]; sorted[a] = sorted[b]; sorted[b] = t; }
            const cplx *m = mats + moff[sel[s * n_ops + g]];
            const int64_t d = 1ll << k;
            const int64_t groups = 1ll << (n - k);
            for (int64_t gi = 0; gi < groups; ++gi) {
                uint64_t base = spread((uint64_t)gi, sorted, k);
                uint64_t idx[256];
                cplx v[256];
                for (int64_t j = 0; j < d; ++j) {
                    uint64_t x = base;
                    for (int b = 0; b < k; ++b)
                        if ((j >> (k - 1 - b)) & 1) x |= 1ull << qs[qo + b];
                    idx[j] = x;
                    v[j] = st[x];
                }
                for (int64_t i = 0; i < d; ++i) {
                    cplx acc = 0;
                    for (int64_t j = 0; j < d; ++j) acc += m[i * d + j] * v[j];
                    st[idx[i]] = acc;
                }
            }
            qo += k;
        }
    }
    return rc_all;
}
