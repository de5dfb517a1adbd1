"""FP64 CPU oracle for TDVP time evolution of MPS with long-range MPOs.

TEST INFRASTRUCTURE ONLY.  Only the test suite, ``__graft_entry__.smoke()``
and the CPU-baseline leg of ``bench.py`` may import this package.  The
product path (the HIP library and its Python binding) never imports, calls
or links anything here, and nothing here imports the product path.

Everything is plain numpy/scipy in complex128, written for readability:
each function cites the part of Secular et al., "Parallel time-dependent
variational principle algorithm for matrix product states" (arXiv:1912.06127)
it follows.  Index conventions (all sites 1-based in the text, 0-based in
Python lists):

* MPS site tensor  A[a, s, b]        shape [chi_{j-1}, d, chi_j]     (Sec. II A)
* MPO site tensor  W[k, l, s', s]    shape [w_{j-1}, w_j, d, d]      (Sec. II C)
  with s' the output (bra) and s the input (ket) physical index.
* left environment  beta_j[a', k, a]  from sites 1..j-1  (Sec. III A, Fig. 3a)
* right environment gamma_j[b', l, b] from sites j+1..N  (Sec. III A, Fig. 3b)

Pin status of each module is listed in its header; every function is pinned
by a test under ``tests/test_oracle_*.py`` unless its docstring says
"parity unpinned".
"""
