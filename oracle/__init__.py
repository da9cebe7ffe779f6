"""CPU FP64 oracle for the layered BTTB sensitivity operator and the inversion built on it.

TEST INFRASTRUCTURE ONLY.  Nothing in the product package may import, call, link or
execute this package: only the test suite, the smoke check and the CPU-baseline leg
of the benchmark use it.  It shares no code with the HIP path (no kernels, headers,
tables or helpers); the two meet only through the seeded input generators in
``paper_2004_13904_amd.workloads``, which hold none of the method's arithmetic.

The oracle computes the *definitions*, never the fast method:

* ``prism``     closed-form prism integrals (gravity g_z, gravity-gradient tensor,
                induced total-field anomaly), Sec. 2.1 of the paper.
* ``geometry``  station / prism bookkeeping, padding rule of Sec. 3.2 (Table 2),
                subspace sizes t, t_p of Secs. 2.3 and 3.1.
* ``operator``  the sensitivity matrix G entry by entry (eq. blockG) and G x, G^T y
                by direct summation over its Toeplitz blocks -- no FFT anywhere.
* ``solvers``   Algorithm 1 (GKB with MGS reorthogonalization), Algorithm 2 (RSVD
                with one power iteration), the truncated UPRE and the closed-form
                Tikhonov solution eq. (constantWL).
* ``irls``      the focusing IRLS step of Secs. 2.2-2.3, depth weighting, noise model
                eq. (noisydata), chi^2 test eq. (scaledchi2), SNR and RE.

Functions whose result the tests cannot pin to anything independent of the oracle
itself say "parity unpinned" in their docstring.
"""
