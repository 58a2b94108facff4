"""FP64 CPU oracle for asynchrony-tolerant (AT) finite differences.

This package is TEST INFRASTRUCTURE. It is a plain, slow, direct transcription
of what Aditya & Donzis, "High-order asynchrony-tolerant finite difference
schemes for partial differential equations" (arXiv 1702.00496) define:

- ``coeffs``   exact rational solution of the Taylor order conditions
               (Sec. 3.1, eq. cond) and of the step-by-step time-level system
               (Sec. 3.3 / Sec. 3.4 Example 3);
- ``rng``      the counter-based delay generator (SplitMix64 finaliser, bins of
               Sec. 5.1 "simulate delays");
- ``solver``   the AT time step with a full-field history of past levels
               (Sec. 2, eqs. general_deriv / general_deriv_async; Sec. 3.4
               eq. cd4-at and Tables atschemes-left/right; Sec. 4.1 eqs.
               time_disc / time_ab2; Sec. 5 eq. general);
- ``analytic`` the exact decaying advected Fourier series (Sec. 5.1 eq. ana_sol);
- ``norms``    space averages of the error (Sec. 4) and ensemble statistics;
- ``adjoint``  gradients of a final-time function through torch CPU autograd
               of the forward steps.

A delay ensemble member is a single 1-D problem of ``solver`` with its own
generator key, so ensembles need no module of their own.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import anything from here. The product library never does and
shares no code with it.
"""
