"""FP64 CPU oracle for the Monte Carlo - rigorous Mie photon walk.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call, link
or execute anything in this package: only the tests, the smoke check and the
benchmark's CPU-baseline leg use it.  It shares no code with the HIP library
(no common kernels, headers, tables or helpers); the only module both sides
read is ``workloads`` (input parameters, no arithmetic of the method).

Contents
  mie     Mie coefficients (Bohren-Huffman downward log-derivative recurrence,
          Sec. 2.5), Q_ext/Q_sca/g (Eqs. 12-13), amplitudes S1/S2 (Eqs. 5-6),
          phase function (Eqs. 9-10), trapezoid CDF and inverse table (Sec. 2.6,
          Sec. 3.1.2), Henyey-Greenstein closed forms (Eq. 11).
  philox  Philox4x32-10 in pure Python integers (Salmon et al., SC'11).
  walk.c  The photon walk of Sec. 3.1.3 in plain C, FP64, one photon at a time.
  walk    ctypes driver for walk.c: per-chunk images reduced in a fixed order.
"""
