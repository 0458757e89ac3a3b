"""CPU FP64 oracle for the truncated free-space box code (TEST INFRASTRUCTURE ONLY).

This package is the checker, not the product. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it. It shares no code, tables,
constants or helpers with the HIP path under ``paper_2501_17967_amd/``; the two meet only
through the seeded input generators in ``workloads/``, which hold none of the method's
arithmetic.

What it computes (Sec. 4.2, eq. (vbulk)): the volume potential of the leaf data,

    u(x) = int_{Omega_B} G(x - y) f_h(y) dy,   G(r) = -(1/2pi) log|r|,

where Omega_B is the union of the leaf boxes of a quadtree and f_h is, on each leaf, the
order-p tensor Chebyshev interpolant of the nodal samples (Sec. 4.2.1). The paper's
v_bulk is -u (it writes v_bulk = -int Phi f with Phi = (1/2pi) log; we keep the sign that
makes -Lap u = f).

Modules
-------
nodes         node/weight convention of a leaf (first-kind Chebyshev, Fejer-1 weights)
closed_forms  uniform-square and Gaussian potentials in closed form, exterior tail
quad          the log-kernel integral of one Lagrange basis over a box (adaptive
              subdivision, plain C in ``_quad.c``), the near tables built from it, and
              the direct sum u = sum_b int_{B_b} G f_h  (the plain definition), also at
              arbitrary points and with its gradient
tree          integer box keys, tiling and 2:1-balance checks, the U/V/W/X interaction
              lists of the adaptive FMM by key arithmetic
quadtree      adaptive construction of the quadtree from samples of f (Chebyshev tail test)
              and the 2:1 balance, plain loops
strip         the strip solve of Sec. 4.3 (multidomain spectral collocation between the boundary
              and the fictitious curve), assembled densely and solved directly
fmm           a CPU machine code with complex scaled expansions (Greengard-Rokhlin), its
              exact transpose, used for full-size parity and as the CPU baseline
layer         the glue layer potentials S[sigma] - D[tau] of Sec. 4.4 on a panel-discretised
              curve, by direct summation at arbitrary targets (the plain definition that
              the FMM evaluation at the quadtree nodes approximates)

Parity pins: see tests/test_oracle_*.py. Every function here is pinned by a closed form,
a library routine, brute force or an invariant, except where its docstring says
"parity unpinned".
"""
