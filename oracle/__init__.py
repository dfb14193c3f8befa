"""FP64 CPU oracle for the FEWHA hot path (Stadler & Ramlau, "Performance of an
iterative wavelet reconstructor for MAORY", arXiv 2202.11945).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this package: only the test suite, the smoke check and the CPU
baseline leg of the benchmark do.  It shares no code with the GPU library;
both take their inputs from the ``synthetic`` package.

The oracle is plain and slow on purpose: explicit scipy.sparse matrices for
the Shack-Hartmann operator Gamma (Sec. 2), the propagation operators P_g
(Sec. 2, NGS and LGS forms) and the wavelet transform W (Sec. 3.1, periodic
Daubechies-3), dense 1-D transform matrices for wavelet applications, and a
textbook fixed-iteration PCG (Sec. 3.3-3.4, Algorithm 1, open loop) in float64.

Readings of the paper (where it is silent, ambiguous or inconsistent) are
listed in the repository's design notes; the ones that change numbers:

* s^y stencil: the printed formula repeats phi_{i,j}; the symmetric partner
  of the s^x stencil, (phi_{i+1,j+1} - phi_{i,j+1}), is used.
* Slopes are phase differences per subaperture (no 1/d factor).
* Index (i, j) = (row = y, column = x), row-major.
* Active subaperture: centre inside the annulus [sqrt(obs) D/2, D/2].
* Layers share one centred square domain of side L; delta_l = L / n_l.
* W_l = delta_l W, so W_l^{-1} = W^T / delta_l.
* The preconditioner and the right-hand side use the tip/tilt-filtered
  noise weighting C_hat^{-1} everywhere, the system operator too.

Parity status per function:

* db3 filter, W, Gamma, P_g, A, C_hat^{-1}, M, J, PCG, warm start: pinned by
  the closed forms, invariants and brute-force checks in tests/test_oracle_*.py.
* D (the diagonal prior): the paper does not print its formula (it cites
  another paper).  The von Karman spectrum evaluated at the level frequency
  2^j / L is used.  Its level ratios are pinned in the Kolmogorov limit, and
  the spectrum's absolute scale and outer-scale term by the textbook
  Kolmogorov structure function and von Karman phase variance; which
  frequency stands for level j (2^j / L) is parity unpinned.
"""
