/*
 * Oracle: plain, slow, obviously correct state-vector evolution in complex128.
 *
 * TEST INFRASTRUCTURE ONLY.  Nothing on the product path links, loads or calls
 * this file; only the tests, the smoke check and the CPU-baseline leg of the
 * benchmark do.  It shares no code, header or table with the HIP library.
 *
 * What it computes is the plain definition of state-vector simulation (paper,
 * Simulations and State Vector sections): psi_out = U_G ... U_1 psi_in, each
 * gate applied once, in list order, as a matrix-vector product on the amplitude
 * groups it touches.  No fusion, no reordering, no skipping.
 *
 * Conventions (the paper's Grover example fixes the bit order, see the Python
 * side): amplitude index i holds the qubit at position p in bit p; a k-qubit
 * matrix M has local index m whose most significant bit belongs to q[0].
 */
#include <complex.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

typedef double complex cplx;

/* O2, initial product state (Initial and Final State Specification section):
 * tokens '0', '1', '+', '-'; token j describes the qubit at position n-1-j.
 * Amplitude i is the product over positions p of a_p[bit p of i].
 * Returns 0, or -1 on an unknown token. */
int ref_product_state(int n, const char *tokens, double *psi_out)
{
    cplx (*a)[2] = malloc(sizeof(cplx[2]) * (size_t)(n > 0 ? n : 1));
    const double r = 0.70710678118654752440;
    for (int j = 0; j < n; ++j) {
        int p = n - 1 - j;
        switch (tokens[j]) {
        case '0': a[p][0] = 1.0; a[p][1] = 0.0; break;
        case '1': a[p][0] = 0.0; a[p][1] = 1.0; break;
        case '+': a[p][0] = r;   a[p][1] = r;   break;
        case '-': a[p][0] = r;   a[p][1] = -r;  break;
        default: free(a); return -1;
        }
    }
    cplx *psi = (cplx *)psi_out;
    uint64_t N = (uint64_t)1 << n;
    for (uint64_t i = 0; i < N; ++i) {
        cplx v = 1.0;
        for (int p = 0; p < n; ++p)
            v *= a[p][(i >> p) & 1];
        psi[i] = v;
    }
    free(a);
    return 0;
}

/* O3, apply one k-qubit gate (State Vector section: a matrix-vector product
 * between the gate and the state).  For every base b that has zeros at all of
 * q[0..k-1], gather v[m] = psi[b + sum_j bit_{k-1-j}(m) 2^{q_j}], then write
 * psi[idx(m)] = sum_{m'} M[m][m'] v[m'], summing m' in ascending order.
 * M is 2^k x 2^k, row-major, complex128 stored as (re, im) pairs. */
void ref_apply(int n, double *psi_io, int k, const int *q, const double *m_in)
{
    cplx *psi = (cplx *)psi_io;
    const cplx *M = (const cplx *)m_in;
    const uint64_t N = (uint64_t)1 << n;
    const int D = 1 << k;
    uint64_t tmask = 0;
    for (int j = 0; j < k; ++j)
        tmask |= (uint64_t)1 << q[j];

#pragma omp parallel for schedule(static)
    for (int64_t bs = 0; bs < (int64_t)N; ++bs) {
        uint64_t b = (uint64_t)bs;
        if (b & tmask)
            continue; /* not a base: it has a one at some target position */
        uint64_t idx[64];
        cplx v[64];
        for (int mm = 0; mm < D; ++mm) {
            uint64_t off = 0;
            for (int j = 0; j < k; ++j)
                if ((mm >> (k - 1 - j)) & 1)
                    off += (uint64_t)1 << q[j];
            idx[mm] = b + off;
            v[mm] = psi[idx[mm]];
        }
        for (int mm = 0; mm < D; ++mm) {
            cplx acc = 0.0;
            for (int mp = 0; mp < D; ++mp)
                acc += M[mm * D + mp] * v[mp];
            psi[idx[mm]] = acc;
        }
    }
}

/* O5, a whole circuit: apply the G gates in list order.  Gate g acts on
 * ks[g] qubits listed at qs[qoff[g] ..] with its matrix at ms[moff[g] ..]
 * (offsets counted in doubles). */
void ref_run(int n, double *psi_io, int G, const int *ks, const int *qs,
             const int64_t *qoff, const double *ms, const int64_t *moff)
{
    for (int g = 0; g < G; ++g)
        ref_apply(n, psi_io, ks[g], qs + qoff[g], ms + moff[g]);
}

/* Plain inner product <a|b> = sum_i conj(a_i) b_i, accumulated in index order
 * with Kahan-compensated sums of the real and imaginary parts. */
void ref_inner(int n, const double *a_in, const double *b_in, double *re, double *im)
{
    const cplx *a = (const cplx *)a_in, *b = (const cplx *)b_in;
    uint64_t N = (uint64_t)1 << n;
    double sr = 0, cr = 0, si = 0, ci = 0;
    for (uint64_t i = 0; i < N; ++i) {
        cplx t = conj(a[i]) * b[i];
        double y = creal(t) - cr, s = sr + y;
        cr = (s - sr) - y; sr = s;
        y = cimag(t) - ci; s = si + y;
        ci = (s - si) - y; si = s;
    }
    *re = sr;
    *im = si;
}
