"""CPU oracle for the extreme-precision Hankel LDL^T -> k x k block of H^-1 -> lambda_1
path.  TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import or run anything in this package.  The HIP library and its
Python binding never call it, and it shares no code with them: the only thing
both sides use is ``hankel_inputs`` (the moment sequence, which carries none of
the method's arithmetic).

Modules
-------
contract  the fixed-point contract step by step, in Python integers:
          scales, load, Algorithm 1 with explicit rounding points, Algorithm 4
          for the first k columns of L^-1, eq. ``equ:index`` for the block, and
          the largest eigenvalue of the block by a dense library eigen-solver,
          and (``eigen_next``) the next ones, lambda_2 and lambda_3 of Table 2.
exact     exact rational arithmetic for tiny N: LDL^T, L^-1, H^-1 block, and the
          characteristic polynomial of H_N for brute-force eigenvalues.
fit       the weighted straight-line fit of Section 6 (leading exponent) from its
          closed form, with Student-t intervals.
adjoint   the derivative of lambda_1 with respect to the moments (the adjoint
          vector mubar) and its contraction with d mu / d beta, from the
          definition, in mpmath.

Every function names the passage of the paper it follows.  Parity status of each
function is stated in its module header.
"""
