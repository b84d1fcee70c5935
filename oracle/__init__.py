"""CPU FP64 oracle for the Chebyshev-based Nystrom (CBIE) MFIE system.

TEST INFRASTRUCTURE ONLY.  Plain, slow, obviously correct NumPy/SciPy code in
float64 / complex128 that computes what the GPU path computes, written from
the paper (arXiv 2408.17116) and checked against closed forms.  Only the tests,
the smoke check and the CPU-baseline leg of the benchmark may import it; the
product library never does, and it shares no code with the HIP path.

Modules
-------
cheb      Fejer-1 rule, Chebyshev coefficient map (eq. 13), interpolation basis
geometry  cube-sphere ellipsoid patches, covariant/contravariant bases
          (eqs. 11, 14, 17, 18)
mfie      PEC MFIE (eq. 10, second row) discretized by CBIE (eqs. 15-20, 22):
          far entries by plain Fejer quadrature, self/near entries as exact
          integrals against the Chebyshev basis by an independent Duffy/sinh
          rule, plane-wave right-hand side
dense     dense complex128 solve (LAPACK partial pivoting) and a hand-written
          partial-pivot LU for small systems
post      surface current, radiation integral and bistatic RCS
mie       Mie series for the PEC sphere (surface current, S1/S2, RCS)
aca       partial-pivot adaptive cross approximation (the paper's ref. [22])
mlp       8-64-64-1 rank-predictor network, forward/backward/Adam in float64
"""
