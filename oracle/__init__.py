"""Plain FP64 CPU oracle of the CN / SIPG-PolyDG monodomain solve with the
two-level additive Schwarz PCG.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` may import this package.  The product path
(the C-ABI library and its Python binding) never imports or calls it, and this
package never imports the product.  The two share no code; only the seeded
input generators in ``pdg_inputs`` serve both, as data.

Modules (each function cites the passage of the paper it follows):

* :mod:`oracle.basis`       -- modal Legendre basis on element bounding boxes.
* :mod:`oracle.quadrature`  -- element and facet quadrature rules.
* :mod:`oracle.assemble`    -- mass matrix, SIPG matrix (eq. (3)), penalty (eq. (2)),
                               system matrix of Section 3.
* :mod:`oracle.ionic`       -- Barreto-Cressman-type ionic model (Section 2).
* :mod:`oracle.schwarz`     -- two-level additive Schwarz preconditioner (eq. (5)).
* :mod:`oracle.pcg`         -- PCG and the Lanczos condition-number estimate (Section 5).
* :mod:`oracle.monodomain`  -- one fully discrete time step (eq. (4)).
* :mod:`oracle.mlp`         -- the learned initial guess's network (not in the
                               paper): forward, backward, Adam, BF16 rounding.

Parity status of each function is stated in its module header.
"""
