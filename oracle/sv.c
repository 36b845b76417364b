/* In-place state-vector gate application in plain C (oracle; test infrastructure only).
 *
 * The same three operations as the numpy simulator in statevector.py, written out as
 * loops over the 2^n complex128 amplitudes so that a 30-qubit state (16 GiB) is updated in
 * place, without the copies numpy.tensordot makes, and on every host core (OpenMP).
 * Qubit q is bit n-1-q of the amplitude index (qubit 0 is the most significant bit).
 *
 *   sv_apply_1q(psi, n, q, u)          psi <- U_q psi, u[2*out + in] (row-major 2x2)
 *   sv_apply_2q(psi, n, qa, qb, g)     psi <- G_{qa,qb} psi, g[((oa*2+ob)*2+ia)*2+ib]
 *                                      (four-way tensor G[out_a, out_b, in_a, in_b])
 *   sv_project(psi, n, q, v)           psi <- |v><v|_q psi (amplitudes with s_q != v zeroed)
 *
 * The simulator loop (cycles, the single-qubit layer, then the fSim layer; Eq. (1) for the
 * fSim entries; slicing and holes as projectors) stays in statevector.py, shared by both
 * backends; this file only holds the per-gate arithmetic.
 */
#include <complex.h>
#include <stdint.h>

typedef double complex cplx;

/* i with a zero bit inserted at bit position b (the bits from b upwards move up by one) */
static inline int64_t insert_zero(int64_t i, int b) {
  const int64_t low = i & ((((int64_t)1) << b) - 1);
  return ((i - low) << 1) | low;
}

void sv_apply_1q(cplx* psi, int n, int q, const cplx* u) {
  const int b = n - 1 - q;
  const int64_t half = ((int64_t)1) << (n - 1), step = ((int64_t)1) << b;
  const cplx u00 = u[0], u01 = u[1], u10 = u[2], u11 = u[3];
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < half; ++i) {
    const int64_t i0 = insert_zero(i, b), i1 = i0 | step;
    const cplx a0 = psi[i0], a1 = psi[i1];
    psi[i0] = u00 * a0 + u01 * a1;
    psi[i1] = u10 * a0 + u11 * a1;
  }
}

void sv_apply_2q(cplx* psi, int n, int qa, int qb, const cplx* g) {
  const int ba = n - 1 - qa, bb = n - 1 - qb;
  const int blo = ba < bb ? ba : bb, bhi = ba < bb ? bb : ba;
  const int64_t quarter = ((int64_t)1) << (n - 2);
  const int64_t sa = ((int64_t)1) << ba, sb = ((int64_t)1) << bb;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < quarter; ++i) {
    const int64_t base = insert_zero(insert_zero(i, blo), bhi);
    int64_t idx[4];
    cplx x[4];
    for (int ia = 0; ia < 2; ++ia)
      for (int ib = 0; ib < 2; ++ib) {
        idx[2 * ia + ib] = base | (ia ? sa : 0) | (ib ? sb : 0);
        x[2 * ia + ib] = psi[idx[2 * ia + ib]];
      }
    for (int o = 0; o < 4; ++o) {
      cplx s = 0;
      for (int in = 0; in < 4; ++in) s += g[4 * o + in] * x[in];
      psi[idx[o]] = s;
    }
  }
}

void sv_project(cplx* psi, int n, int q, int v) {
  const int b = n - 1 - q;
  const int64_t half = ((int64_t)1) << (n - 1), step = ((int64_t)1) << b;
#pragma omp parallel for schedule(static)
  for (int64_t i = 0; i < half; ++i) {
    const int64_t i0 = insert_zero(i, b);
    psi[v ? i0 : (i0 | step)] = 0;
  }
}
