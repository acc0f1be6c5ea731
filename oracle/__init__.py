"""Sequential CPU oracle for the discretised continuous-time MAP problem.

TEST INFRASTRUCTURE ONLY.  Only `tests/`, `__graft_entry__.smoke()` and the
CPU-baseline leg of `bench.py` may import, call or link anything in here.  It
shares no code, header, table or pre/post-processing with the GPU library in
`paper_2512_13319_amd/`, and neither side imports the other; both only read
the seeded inputs of `workloads/`.

  ref.py     plain PyTorch FP64: Kalman filter, RTS smoother, discretised
             Onsager--Machlup objective, Gauss--Newton iteration; gradients by
             autograd.
  kfs.c      the same filter / smoother / likelihood / objective as plain C,
             for sizes where a Python loop is too slow (`cref.py` drives it),
             and the two-filter smoother of Sec. 4.3 (eq. twofilter): the
             conditional value function of the later steps by the paper's
             combination rule, joined with the forward filter.
  models.py  the models' drift/measurement Taylor terms.
  lti.py     exact (Van Loan, scipy expm) discretisation of time-invariant
             linear models, re-expressed as terms of the implicit-Euler step.

Every function is pinned by tests under `tests/test_oracle_*.py` against
things that do not come from itself: dense Gaussian conditioning, dense least
squares, the discrete and continuous algebraic Riccati equations, central
finite differences of a dense likelihood, and nonlinear least squares; the
two-filter smoother also against the dense likelihood of the later
measurements given one state (its backward filter); the exact discretisation
against closed forms and dense conditioning with exact transitions.
"""
