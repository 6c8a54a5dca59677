"""Plain, slow CPU FP64 oracle for the spherical curvelet transform.

THIS PACKAGE IS TEST INFRASTRUCTURE.  Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it.  The product path
(``paper_1511_05578_amd``) never imports, calls or links anything here, and this
package imports nothing from the product.  The two share no kernels, tables,
constants or helpers; only the seeded input generator
(``paper_1511_05578_amd/inputs.py``, which holds none of the method's
arithmetic) feeds both sides.

What it computes, and how (Chan, Leistedt, Kitching, McEwen, "Second-generation
curvelets on the sphere", IEEE TSP 65(1), 2017):

* Wigner small-d (Sec. II-A, the factorial-sum expression for d^l_mn) in exact
  multiprecision at tiny l, and for any l by the textbook three-term recurrence
  in l with closed-form edge seeds (``wigner``).  The Fourier factorisation
  through Delta = d(pi/2) that the fast path uses is NOT used here.
* Curvelet kernels (Sec. II-B): k_lambda by tanh-sinh quadrature in
  multiprecision, kappa^(j), the scaling function Phi, the directional part
  zeta obtained by explicitly rotating the unrotated zeta-tilde, and the
  curvelet coefficients Psi^(j)_ln (``kernels``).
* Spherical harmonic transforms on McEwen-Wiaux sampling (``sht``): inverse
  by direct summation of Y_lm; forward by exact Gauss-Legendre quadrature after
  exact trigonometric interpolation in theta.
* Wigner transforms on SO(3) (``so3``) and the curvelet analysis / synthesis
  (``curvelet``) straight from their definitions (Sec. II-D, the harmonic forms
  of analysis and synthesis), with exact Gauss-Legendre quadrature in beta for
  the forward direction.

Every function cites the passage it follows.  The pins that tie each function
to something other than itself live in ``tests/test_oracle_*.py``.  The
k_lambda integral has no closed form; its integrand is pinned by values the
definition fixes and by the ratio of k_lambda's slopes at two points (see
``kernels``), so every function here has a pin.
"""
