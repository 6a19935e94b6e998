"""Plain FP64 CPU oracle for neural dependence fields.

TEST INFRASTRUCTURE ONLY: the slow, obviously correct reference the GPU path is
checked against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the benchmark's
CPU-baseline leg import it; the product path never does.  It shares no code with
the GPU library (``paper_2307_02203_amd``) and does not import it.

* ``oracle.direct``  : Pearson (Sec. 3.1, Eq. 1) and KSG mutual information
                       (Sec. 3.2, Eq. 2, estimator of [KSG04]) via plain C (ndf_oracle.c)
* ``oracle.ndf_net`` : the learned field (Sec. 4, Eq. 3; Sec. 4.1-4.3) forward,
                       adjoint and Adam in float64 numpy
* ``oracle.points``  : training targets at continuous positions (Sec. 4.3):
                       trilinear interpolation of the ensemble, Pearson in float64
"""
