"""FP64 CPU oracle for the contact-smoothed rope/cloth simulator.

TEST INFRASTRUCTURE ONLY.  Nothing on the product path may import, call or
execute this package: only the tests, ``__graft_entry__.smoke()`` and the
``cpu_baseline`` leg of ``bench.py`` use it.  It shares no code with the HIP
library (no kernels, headers, helpers, tables or pre/post-processing) and
never imports it; both are fed from the seeded generators in ``workloads``.

The oracle is deliberately plain and slow: numpy/scipy in float64, one
instance at a time, every step written in the order the paper gives it
(Sec. 4.1 "Differentiable Deformable Object Simulator with Contact
Smoothing"): gripper kinematics and predictor, stage 1 (eq. dynamics-first-
stage, Newton), stage 2 (eq. dynamics-second-stage with the smoothed
complementarity of the "Contact Smoothing" paragraph), and the implicit
derivatives of both stages (the two implicit-function equations and
eq. diff-sim).

Modules
-------
model        element lists, elastic energy and its first three derivatives
sdf          signed distances, normals and curvatures of the obstacles
step         one time step (stage 1 + stage 2) and rollouts
derivatives  per-step JVP / VJP, dense A_t / B_t, rollout gradient
planner      reference projected-gradient planner (cost, gradient, step, argmin)
conformal    conformal radius of the one-step model error (scores, order statistic)
apg          the step as a differentiable torch layer for analytical policy gradients
sls          output-feedback SLS stage 3: Kalman recursion and its associative scan,
             observer propagations, assembly of the closed-loop responses, tubes
"""
STATUS_OK = 0
STATUS_NEWTON_NOCONV = 1
STATUS_NOT_PD = 2
STATUS_QP_NOCONV = 3
STATUS_NONFINITE = 4
