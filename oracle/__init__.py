"""CPU oracle for the accurate interface-capturing LB scheme (arXiv:2203.05230).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The
product library never loads, links or calls this package, and this package
never imports the product package.  The two share no code.

Contents:
  lbm_oracle.c  plain FP64 D2Q9 iteration (built into liboracle.so)
  lib.py        ctypes wrapper over liboracle.so
  d1q3.py       independent 1-D D1Q3 reduction of the same scheme (numpy)
  fv1d.py       finite-volume solution of the 1-D improved conservative ACE
  mlp.py        FP64 reference of the learned-closure MLP, its gradients, Adam
  closure_ref.py  restriction and flux-correction targets for the closure
"""
