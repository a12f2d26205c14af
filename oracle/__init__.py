"""CPU oracle for G-QAOA on 3-SAT (Zhang et al., arXiv 2402.02585).

TEST INFRASTRUCTURE, NOT PART OF THE PRODUCT. Only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import, call, link or run anything in this package. It shares no code with the
HIP path: it is plain numpy in complex128 / float64 (plus one plain C loop for
brute-force counting at large n), written from the paper's definitions:

  cost.py      clause cost C(z) and the level histogram (Eq. (1) and App. B)
  evolve.py    statevector and level-space ("effective space") evolution of
               Eq. (3) / Eq. (5), readouts of Eq. (4)
  grad.py      reverse-mode gradient of P_sol with respect to all 2p angles
  mlp.py       the angle-predictor MLP in float64 with bfloat16 rounding
               emulated at the storage points
  optimize.py  grid search followed by L-BFGS-B (App. C, "Optimization")
  rounds.py    rounds to reach a target success probability, Max-SAT level,
               the 1/sqrt(P) fit (Sec. III)
  xqaoa.py     the transverse-field mixer comparator (Sec. IV)
  fairness.py  fair-sampling metrics of Table I
  brute.py     ctypes wrapper of brute_count.c (plain loops) for n up to 34

Every function names the passage it follows. ``optimize.py`` is pinned on
two-level costs (Grover's optimum) and otherwise only by the properties in its
header. ``mlp.py``'s training step is built from pinned pieces (forward,
backward, Adam); training over many steps is not pinned further.
"""
