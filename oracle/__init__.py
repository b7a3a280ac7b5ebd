"""CPU oracle for the Berends-Giele event-generation path (TEST INFRASTRUCTURE ONLY).

A plain, slow, double-precision (or long-double) restatement of what the method
computes, written from the paper's Sections 3 and 4:

  philox.py     counter-based generator (published Philox-4x32-10 definition)
  draws.py      how one event's 32-bit words become uniforms, helicities, ordering
  pdf.py        synthetic gluon density and its inverse-CDF sampler
  rambo.py      flat massless phase space (RAMBO) and the longitudinal boost
  cuts.py       jet cuts and the observables H_T and R_min
  helicity.py   helicity polarisation vectors
  recursion.py  the Berends-Giele recursion exactly as printed (Eqs. 3.1, 3.2),
                the amputated closure (Eq. 3.6), the Parke-Taylor closed form and
                the W-tensor form (Eqs. 3.3, 3.4) used only as checks
  weight.py     event weight (Eqs. 3.7, 3.8) and compensated summation (Sec. 4)
  event.py      whole-event pipelines and the log-weight gradient (torch autograd)

Only tests/, __graft_entry__.smoke() and bench.py's cpu_baseline leg may import this
package.  It shares no code with the HIP library and never imports it.
Everything here works on arrays batched over events; arithmetic per event is the
plain definition, with no regrouping.

Parity pins: every function is pinned by tests/test_oracle_*.py against closed
forms, invariants, brute force or an independent implementation: Philox word for
word against rocRAND's implementation of the published generator; the weight chain's
n-dependence (helicity, ordering and colour factors, the phase-space volume) by a
brute-force full-colour sum at n = 4, 5, the random-ordering identity and the
recursive factorisation of phase space (tests/test_oracle_chain.py).  The values of
non-MHV amplitudes (n >= 6) have no closed form; they are pinned by the identities
(gauge, Ward, cyclic, reflection, U(1) decoupling, scaling, Lorentz invariance), the
W-tensor form and a long-double evaluation.
"""
