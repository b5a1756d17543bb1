"""FP64 CPU oracle of the STAMP SVGD hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  The product path (the HIP library and
its Python binding) never imports, links or executes anything here, and this
package imports nothing from the product.  The two share only the seeded input
generators in ``workloads``.

What it computes, step by step in the paper's order (Algorithm 1):

* ``sim``   -- the relaxed plan (Eq. 5: per-push softmax / argmax), the
  semi-implicit-Euler rigid-body pushing rollout with penalty-spring contacts
  (Section III-B), the block-pushing cost (Section IV-A, Appendix E-B) and its
  gradient by reverse-mode automatic differentiation over the rollout
  (Section III-B: gradients back-propagated through the whole trajectory).
* ``svgd``  -- squared pairwise distances, the median-heuristic bandwidth
  (Appendix D-B), the RBF kernel and the SVGD direction of Eq. (1), the Adam
  or plain update, and the solve loop.
* ``structured`` -- the structured pusher kernel of Appendix E-C (per-action
  RBF terms on the continuous parameters and on softmax(a_k), von Mises terms
  on angles) and the SVGD direction under it, the kernel gradient by autodiff.
* ``mlp``   -- the surrogate network (3 dense layers, GELU) with its input
  gradient and a training step, by autodiff in FP64.

All arithmetic is float64.  Parity pins live in ``tests/test_oracle_*.py``.
Functions without an external pin say "parity unpinned" in their docstring.
"""
from . import sim, structured, svgd  # noqa: F401
