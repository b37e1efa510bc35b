"""CPU FP64 oracle for the short-range PM-FMM force (test infrastructure).

This package is test infrastructure only.  The GPU library never imports,
links or calls it; only the test suite, the smoke check and the CPU baseline
leg of the benchmark use it.  It shares no code with the GPU path.

Every function is a plain, slow restatement of the paper (Wang & Meng,
"PhotoNs-GPU", arXiv 2107.14008) in float64 numpy:

  * ``truncation`` - the truncation factor T of Eq. (tr), its integral form
    and Taylor table of Eq. (int), the M2L prefactors f_(n) of Sec. 2 and the
    full Cartesian derivative tensors D built from them;
  * ``direct``     - brute-force minimum-image sums over cell lists (the
    definition of the short-range acceleration and of its gradient);
  * ``tree``       - the ORB tree (Sec. 2) and the dual walk that yields the
    P2P and M2L task lists (Sec. 3), with the readings in its docstring;
  * ``fmm``        - the truncated FMM of Sec. 2 on those lists
    (P2M, M2M, M2L, L2L, L2P plus P2P);
  * ``pm``         - the long-range part of the split on a mesh (CIC, FFT,
    Gaussian-filtered Green's function) and a periodic Ewald sum that the
    short + long total is checked against;
  * ``stepping``   - a kick-drift-kick leapfrog with the split force and the
    power spectrum of the paper's precision comparison;
  * ``metrics``    - relative force error percentiles.

Parity status of each function is stated in its module docstring.
"""
