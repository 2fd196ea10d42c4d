"""Seeded synthetic rope and cloth instances.

Shapes follow the paper's objects: a rope of about 0.8 m (perception appendix,
rope subsection) and a cloth of about 38 cm square (cloth subsection).  The
paper names no benchmark suite for its simulator, so every instance here is
synthetic; the recipes are the configurations the simulator is benchmarked on:

* ``config_c1``: one 20-node rope, 50 steps, ground + one sphere.
* ``config_c2``: 1024 ropes of 64 nodes, 100 steps, ground + 3 random spheres.
* ``config_c3``: 256 cloths of 32x32 nodes, 60 steps, ground + sphere + box.
* ``config_c4``: 4096 mixed ropes (16..256 nodes) and cloths (8x8..48x48).

Random numbers come from ``numpy.random.Generator(PCG64)``; a batch uses one
child stream per instance from ``SeedSequence(seed).spawn(B)`` so that an
instance's inputs do not depend on the batch it is drawn in.

State layout of one instance (``n`` nodes): ``s = [x_0 .. x_{n-1} | v_0 .. v_{n-1}]``
with xyz interleaved, i.e. ``6n`` floats.  Controls are gripper velocities,
``u[t] = [u_0 | u_1 | ...]`` (3 per gripper).  A cloth node ``(ix, iy)`` has
index ``iy * nx + ix``.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

ROPE = "rope"
CLOTH = "cloth"


@dataclasses.dataclass
class Instance:
    kind: str                 # "rope" | "cloth"
    nx: int                   # rope: number of nodes; cloth: nodes along x
    ny: int                   # rope: 1; cloth: nodes along y
    h: float                  # rest spacing between grid neighbours [m]
    mass: float               # lumped mass per node [kg]
    k_struct: float           # stretch / structural spring stiffness [N/m]
    k_shear: float            # cloth shear spring stiffness [N/m] (rope: unused)
    k_bend: float             # rope: discrete-curvature stiffness; cloth: bend spring [N/m]
    grip_nodes: tuple         # node held by gripper k
    ground: bool              # plane z = 0
    spheres: np.ndarray       # (ns, 4): cx, cy, cz, r
    boxes: np.ndarray         # (nb, 7): cx, cy, cz, hx, hy, hz, rounding
    dt: float
    gamma: float              # velocity damping: predictor x + dt (1 - gamma) v
    gravity: np.ndarray       # (3,)
    kappa_fwd: float          # contact relaxation used by forward rollouts [J]
    kappa_bwd: float          # contact relaxation used for derivatives [J]
    T: int                    # horizon
    s0: np.ndarray            # (n_s,) initial state [x | v] (+ [g] in penalty mode)
    u: np.ndarray             # (T, 3 * n_grip) controls
    # grasp: "dirichlet" (node held exactly) or "penalty" (gripper position
    # g_k is part of the state and pulls its node with stiffness
    # D_k = D_max * activation; smooth activation exp(-|x_j - g_k| / kappa_h)
    # if kappa_h > 0, else the indicator of |x_j - g_k| <= r_g)
    grip_mode: str = "dirichlet"
    D_max: float = 0.0        # [N/m]
    kappa_h: float = 0.0      # [m]
    r_g: float = 0.0          # [m]
    mu: float = 0.0           # friction coefficient of every contact (0: frictionless)

    @property
    def n(self) -> int:
        return self.nx * self.ny

    @property
    def penalty(self) -> bool:
        return self.grip_mode == "penalty"

    @property
    def n_s(self) -> int:
        return 6 * self.n + (3 * len(self.grip_nodes) if self.penalty else 0)

    @property
    def n_u(self) -> int:
        return 3 * len(self.grip_nodes)

    def replace(self, **kw) -> "Instance":
        return dataclasses.replace(self, **kw)


def contact_kappa(mass: float, dt: float, width: float) -> float:
    """Contact relaxation for a smoothing width: kappa = (m / dt^2) * width^2.

    With this choice an isolated particle resting on a surface (signed
    distance 0) settles at a gap equal to ``width``.
    """
    return mass / dt ** 2 * width ** 2


def _grid_positions(nx: int, ny: int, h: float, z0: float) -> np.ndarray:
    ix, iy = np.meshgrid(np.arange(nx), np.arange(ny), indexing="xy")
    pos = np.stack([ix.ravel() * h, iy.ravel() * h, np.full(nx * ny, z0)], axis=1)
    return pos.astype(np.float64)


def rope(n: int, *, length: float = 0.8, z0: float = 0.1, k: float = 500.0,
         k_bend: float = 5.0, mass: float = 0.01, dt: float = 0.005,
         gamma: float = 0.02, T: int = 50, grip_nodes=(0,), ground: bool = True,
         spheres=(), boxes=(), width: float = 1e-3, kappa_fwd=None,
         kappa_bwd=None, u=None, gravity=(0.0, 0.0, -9.81), h=None,
         s0=None) -> Instance:
    """A straight rope along +x at height ``z0``, at rest."""
    h = (length / (n - 1) if n > 1 else length) if h is None else h
    kap = contact_kappa(mass, dt, width)
    pos = _grid_positions(n, 1, h, z0)
    if s0 is None:
        s0 = np.concatenate([pos.ravel(), np.zeros(3 * n)])
    n_u = 3 * len(grip_nodes)
    if u is None:
        u = np.zeros((T, n_u))
    return Instance(
        kind=ROPE, nx=n, ny=1, h=float(h), mass=float(mass), k_struct=float(k),
        k_shear=0.0, k_bend=float(k_bend), grip_nodes=tuple(int(g) for g in grip_nodes),
        ground=bool(ground), spheres=np.asarray(spheres, dtype=np.float64).reshape(-1, 4),
        boxes=np.asarray(boxes, dtype=np.float64).reshape(-1, 7), dt=float(dt),
        gamma=float(gamma), gravity=np.asarray(gravity, dtype=np.float64),
        kappa_fwd=float(kap if kappa_fwd is None else kappa_fwd),
        kappa_bwd=float(kap if kappa_bwd is None else kappa_bwd), T=int(T),
        s0=np.asarray(s0, dtype=np.float64), u=np.asarray(u, dtype=np.float64))


def cloth(nx: int, ny: int, *, size: float = 0.38, z0: float = 0.1,
          k_struct: float = 500.0, k_shear: float = 250.0, k_bend: float = 5.0,
          mass: float = 0.01, dt: float = 0.002, gamma: float = 0.02, T: int = 60,
          grip_nodes=None, ground: bool = True, spheres=(), boxes=(),
          width: float = 1e-3, kappa_fwd=None, kappa_bwd=None, u=None,
          gravity=(0.0, 0.0, -9.81), s0=None) -> Instance:
    """A flat square-cell cloth in the plane z = ``z0``, at rest.

    By default the two corners of the ``iy = 0`` edge are gripped.
    """
    h = size / (max(nx, ny) - 1)
    if grip_nodes is None:
        grip_nodes = (0, nx - 1)
    kap = contact_kappa(mass, dt, width)
    pos = _grid_positions(nx, ny, h, z0)
    if s0 is None:
        s0 = np.concatenate([pos.ravel(), np.zeros(3 * nx * ny)])
    n_u = 3 * len(grip_nodes)
    if u is None:
        u = np.zeros((T, n_u))
    return Instance(
        kind=CLOTH, nx=nx, ny=ny, h=float(h), mass=float(mass), k_struct=float(k_struct),
        k_shear=float(k_shear), k_bend=float(k_bend),
        grip_nodes=tuple(int(g) for g in grip_nodes), ground=bool(ground),
        spheres=np.asarray(spheres, dtype=np.float64).reshape(-1, 4),
        boxes=np.asarray(boxes, dtype=np.float64).reshape(-1, 7), dt=float(dt),
        gamma=float(gamma), gravity=np.asarray(gravity, dtype=np.float64),
        kappa_fwd=float(kap if kappa_fwd is None else kappa_fwd),
        kappa_bwd=float(kap if kappa_bwd is None else kappa_bwd), T=int(T),
        s0=np.asarray(s0, dtype=np.float64), u=np.asarray(u, dtype=np.float64))


# --------------------------------------------------------------------------
# random obstacle recipes
# --------------------------------------------------------------------------

def _rope_spheres(rng: np.random.Generator, length: float, z0: float, count: int = 3,
                  clearance: float = 0.005) -> np.ndarray:
    """Spheres r ~ U[0.03, 0.08], centre x ~ U[0.1, 0.7] (scaled to the rope
    length), y ~ U[-0.1, 0.1], z ~ U[0, r]; a draw closer than r + 5 mm to
    the initial rope is rejected and redrawn."""
    out = []
    scale = length / 0.8
    while len(out) < count:
        r = rng.uniform(0.03, 0.08)
        c = np.array([rng.uniform(0.1, 0.7) * scale, rng.uniform(-0.1, 0.1),
                      rng.uniform(0.0, r)])
        xc = min(max(c[0], 0.0), length)
        dist = math.sqrt((c[0] - xc) ** 2 + c[1] ** 2 + (c[2] - z0) ** 2)
        if dist > r + clearance:
            out.append([c[0], c[1], c[2], r])
    return np.array(out, dtype=np.float64)


def _cloth_obstacles(rng: np.random.Generator, size: float, z0: float):
    """One sphere under the cloth interior (top at least 1 cm below the
    cloth) and one rounded box resting on the ground (top at least 1 cm
    below the cloth)."""
    r = rng.uniform(0.03, 0.08)
    cz = rng.uniform(0.0, max(0.0, min(r, z0 - 0.01 - r)))
    sph = np.array([[rng.uniform(0.25, 0.75) * size, rng.uniform(0.25, 0.75) * size, cz, r]])
    hx, hy = rng.uniform(0.02, 0.05, size=2)
    hz = rng.uniform(0.02, min(0.05, (z0 - 0.01) / 2.0))
    box = np.array([[rng.uniform(0.2, 0.8) * size, rng.uniform(0.2, 0.8) * size, hz,
                     hx, hy, hz, 0.005]])
    return sph, box


def _streams(seed: int, count: int):
    return [np.random.Generator(np.random.PCG64(s)) for s in np.random.SeedSequence(seed).spawn(count)]


# --------------------------------------------------------------------------
# benchmark configurations
# --------------------------------------------------------------------------

C1_GOAL = np.array([0.7, 0.2, 0.0])


def config_c1(seed: int = 1001) -> Instance:
    """Single 20-node rope, 50 steps; node 0 gripped; ground + sphere at
    (0.4, 0, 0.05), r = 0.05; controls ~ N(0, 0.05^2)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    T = 50
    u = rng.normal(0.0, 0.05, size=(T, 3))
    return rope(20, k=500.0, k_bend=5.0, mass=0.01, dt=0.005, gamma=0.02, T=T,
                spheres=[[0.4, 0.0, 0.05, 0.05]], u=u)


def penalty_grasp(inst: Instance, *, offset_scale: float = 0.003, kappa_h: float = 0.01,
                  r_g: float = 0.005, D_max: float = None, seed: int = 0) -> Instance:
    """The same instance with penalty grasps: gripper k starts near its node
    (seeded offset ~ N(0, offset_scale^2) per axis) and joins the state;
    D_max defaults to 100 m / dt^2.  kappa_h = 0 selects the hard activation
    radius r_g."""
    rng = np.random.Generator(np.random.PCG64(seed))
    n = inst.n
    x0 = np.asarray(inst.s0[:3 * n]).reshape(n, 3)
    g0 = np.array([x0[j] for j in inst.grip_nodes]) + rng.normal(0.0, offset_scale,
                                                                 size=(len(inst.grip_nodes), 3))
    D = 100.0 * inst.mass / inst.dt ** 2 if D_max is None else D_max
    s0 = np.concatenate([np.asarray(inst.s0[:6 * n]), g0.ravel()])
    return inst.replace(grip_mode="penalty", D_max=float(D), kappa_h=float(kappa_h), r_g=float(r_g), s0=s0)


def _c2_instance(rng, n=64, T=100) -> Instance:
    k = rng.uniform(300.0, 800.0)
    sph = _rope_spheres(rng, 0.8, 0.1)
    u = rng.normal(0.0, 0.05, size=(T, 3))
    return rope(n, k=k, k_bend=5.0, mass=0.01, dt=0.005, gamma=0.02, T=T,
                spheres=sph, u=u)


def config_c2(B: int = 1024, seed: int = 1002, n: int = 64, T: int = 100):
    """Ropes of 64 nodes, 100 steps, k ~ U[300, 800], 3 random spheres."""
    return [_c2_instance(rng, n, T) for rng in _streams(seed, B)]


def _c3_instance(rng, nx=32, ny=32, T=60) -> Instance:
    sph, box = _cloth_obstacles(rng, 0.38, 0.1)
    u = rng.normal(0.0, 0.02, size=(T, 6))
    return cloth(nx, ny, k_struct=500.0, k_shear=250.0, k_bend=5.0, mass=0.01,
                 dt=0.002, gamma=0.02, T=T, spheres=sph, boxes=box, u=u)


def config_c3(B: int = 256, seed: int = 1003, nx: int = 32, ny: int = 32, T: int = 60):
    """Cloths of 32x32 nodes, 60 steps, ground + sphere + box, corners gripped."""
    return [_c3_instance(rng, nx, ny, T) for rng in _streams(seed, B)]


def config_c4(B: int = 4096, seed: int = 1004, max_cloth_side: int = 48, T_range=(30, 120)):
    """Mixed batch: rope (n log-uniform on [16, 256]) or cloth (side
    log-uniform on [8, 48]) with probability 1/2; T ~ U{30..120}.
    ``max_cloth_side`` clips the cloth side (the draw itself is unchanged)."""
    out = []
    for rng in _streams(seed, B):
        T = int(rng.integers(T_range[0], T_range[1] + 1))
        if rng.random() < 0.5:
            n = int(round(math.exp(rng.uniform(math.log(16), math.log(256)))))
            out.append(_c2_instance(rng, n, T))
        else:
            side = int(round(math.exp(rng.uniform(math.log(8), math.log(48)))))
            side = min(side, max_cloth_side)
            out.append(_c3_instance(rng, side, side, T))
    return out


def compressed_rope(n: int = 10, ratio: float = 0.75, T: int = 6, k: float = 800.0, k_bend: float = 5.0,
                    push: float = 0.02) -> Instance:
    """A vertical rope (along z, so gravity acts along its axis) held at both
    ends by grippers, its nodes spaced ``ratio`` times the rest length
    l0 = 4 cm; the top gripper pushes down along the axis at ``push`` m/s.
    No obstacles: the rope stays exactly straight while compressed (the
    compression-guard case)."""
    l0 = 0.04
    z = 0.05 + ratio * l0 * np.arange(n)
    pos = np.stack([np.zeros(n), np.zeros(n), z], axis=1)
    s0 = np.concatenate([pos.ravel(), np.zeros(3 * n)])
    u = np.zeros((T, 6))
    u[:, 5] = -push
    return rope(n, k=k, k_bend=k_bend, mass=0.01, dt=0.005, gamma=0.02, T=T, grip_nodes=(0, n - 1),
                ground=False, h=l0, s0=s0, u=u)


def calibration_set(count: int, n: int = 11, seed: int = 1007, rho: float = 0.002, dt: float = 0.01):
    """Perceived-state transitions (q_i, u_i, q_i+) of a rope of n nodes
    (0.8 m, the paper's hardware rope has 11), for conformal calibration.
    The paper's calibration data are hardware transitions that are not
    available; these are synthetic: q_i is a random planar chain (link
    lengths within 2 % of rest, turning angles ~ N(0, 0.3^2), height
    U[0.05, 0.3] m), u_i ~ N(0, 0.05^2) moves the gripped node 0, and q_i+
    is q_i dragged kinematically (node j by dt u_i exp(-j / 3)) and dropped
    by dt^2 g; both q_i and q_i+ carry perception noise drawn uniformly
    from the ball |e|_2 <= rho over the whole configuration.  Returns a
    list of (Instance with T = 1, quasi-static gamma = 1 and the chain as
    s0, q_next (n, 3))."""
    out = []
    length = 0.8
    l0 = length / (n - 1)
    for rng in _streams(seed, count):
        ang = np.cumsum(rng.normal(0.0, 0.3, size=n - 1))
        seg = l0 * (1.0 + rng.uniform(-0.02, 0.02, size=n - 1))
        q = np.zeros((n, 3))
        q[1:, 0] = np.cumsum(seg * np.cos(ang))
        q[1:, 1] = np.cumsum(seg * np.sin(ang))
        q[:, 2] = rng.uniform(0.05, 0.3)
        u = rng.normal(0.0, 0.05, size=3)
        drag = dt * u[None, :] * np.exp(-np.arange(n) / 3.0)[:, None]
        qn = q + drag + dt * dt * np.array([0.0, 0.0, -9.81])[None, :]

        def ball(d):
            v = rng.normal(size=d)
            return rho * rng.uniform() ** (1.0 / d) * v / np.linalg.norm(v)
        qp = q + ball(3 * n).reshape(n, 3)
        qnp = qn + ball(3 * n).reshape(n, 3)
        s0 = np.concatenate([qp.ravel(), np.zeros(3 * n)])
        inst = rope(n, length=length, dt=dt, gamma=1.0, T=1, s0=s0, u=u[None, :])
        out.append((inst, qnp))
    return out


def lift_rope_envs(B: int, n: int = 12, seed: int = 1008, kappa_fwd: float = 0.0):
    """Environments of a synthetic lift-rope task (the paper's first task: a
    pair of grippers must make contact with the rope to activate the
    holonomic constraint, then lift it).  Each is a rope of n nodes (0.5 m)
    lying just above the ground (z = 2 mm, seeded lateral waviness
    N(0, (5 mm)^2)), with penalty grippers for nodes 0 and n - 1 that start
    U[1.5, 3] cm above their nodes (activation exp(-|c| / 1 cm), so the grasp
    is weak until a gripper comes down), one step per instance (T = 1: a
    policy closes the loop between steps), hard contact forward
    (kappa_fwd = 0) and smoothed gradients (kappa_bwd from a 1 mm width):
    the paper's surrogate-gradient mode."""
    out = []
    for rng in _streams(seed, B):
        y = rng.normal(0.0, 0.005, size=n)
        base = rope(n, length=0.5, z0=0.002, T=1, grip_nodes=(0, n - 1), kappa_fwd=kappa_fwd)
        x = base.s0[:3 * n].reshape(n, 3).copy()
        x[:, 1] = y
        g0 = x[[0, n - 1]] + np.stack([np.zeros(2), np.zeros(2), rng.uniform(0.015, 0.03, size=2)], axis=1)
        s0 = np.concatenate([x.ravel(), np.zeros(3 * n), g0.ravel()])
        inst = base.replace(grip_mode="penalty", D_max=100.0 * base.mass / base.dt ** 2, kappa_h=0.01,
                            r_g=0.005, s0=s0)
        out.append(inst)
    return out


def small_rope_batch(B: int, n: int, T: int, seed: int):
    """C2-style ropes at a smaller size (parity tests)."""
    return [_c2_instance(rng, n, T) for rng in _streams(seed, B)]


def small_cloth_batch(B: int, nx: int, ny: int, T: int, seed: int):
    """C3-style cloths at a smaller size (parity tests)."""
    return [_c3_instance(rng, nx, ny, T) for rng in _streams(seed, B)]


def random_cotangent(size: int, seed: int) -> np.ndarray:
    """A seeded unit vector used as the terminal-state cotangent."""
    rng = np.random.Generator(np.random.PCG64(seed))
    w = rng.normal(size=size)
    return w / np.linalg.norm(w)


def serve_trace(rate: float = 200.0, duration: float = 60.0, seed: int = 1005, T: int = 30):
    """Planning requests with Poisson arrivals: a list of
    (arrival_time_s, Instance, goal_node, goal_point).  Each request is a rope
    (n ~ U{48..128}) or a cloth (side ~ U{16..32}) with probability 1/2,
    horizon T, C2/C3-style material, obstacles and warm-start controls; the
    goal is the last node, steered to a point drawn near its rest position."""
    rng = np.random.Generator(np.random.PCG64(seed))
    out = []
    t = 0.0
    k = 0
    while True:
        t += rng.exponential(1.0 / rate)
        if t >= duration:
            break
        sub = np.random.Generator(np.random.PCG64(np.random.SeedSequence([seed, k])))
        if sub.random() < 0.5:
            n = int(sub.integers(48, 129))
            inst = _c2_instance(sub, n, T)
        else:
            side = int(sub.integers(16, 33))
            inst = _c3_instance(sub, side, side, T)
        x = inst.s0[:3 * inst.n].reshape(-1, 3)
        goal = x[-1] + np.array([sub.uniform(-0.1, 0.1), sub.uniform(-0.1, 0.1), sub.uniform(0.0, 0.1)])
        out.append((t, inst, inst.n - 1, goal))
        k += 1
    return out


def sls_system(B: int, N: int, n: int, m: int, seed: int = 1016, r: float = 0.05, rho: float = 0.1):
    """Seeded inputs of the output-feedback SLS stage (float32, C = I): per
    instance and step a linearization A_j = I + 0.15 G / sqrt(n) (spectral
    radius near 1, like a time step of a damped mass-spring system), input
    matrices B_j (n x m), disturbance scalings E_j = r (I + 0.2 G / sqrt(n))
    and F_j = rho (I + 0.2 G / sqrt(n)), a state-feedback gain K_j (m x n,
    j = 0 .. N) of scale 0.2 / sqrt(n), and Xi = 3 rho (I + 0.2 G / sqrt(n)),
    with G standard normal.  Returns dict(A, E, F, Xi, Bm, K)."""
    rng = np.random.default_rng(seed)
    I = np.eye(n)
    s = 1.0 / np.sqrt(n)

    def near_identity(scale, lead):
        return scale * (I + 0.2 * s * rng.normal(size=lead + (n, n)))

    A = I + 0.15 * s * rng.normal(size=(B, N, n, n))
    E = near_identity(r, (B, N))
    F = near_identity(rho, (B, N))
    Xi = near_identity(3 * rho, (B,))
    Bm = s * rng.normal(size=(B, N, n, m))
    K = -0.2 * s * rng.normal(size=(B, N + 1, m, n))
    f32 = lambda x: np.ascontiguousarray(x, dtype=np.float32)  # noqa: E731
    return dict(A=f32(A), E=f32(E), F=f32(F), Xi=f32(Xi), Bm=f32(Bm), K=f32(K))


def friction_ropes(B: int, n: int = 12, T: int = 10, seed: int = 1021, hard: bool = False):
    """Ropes dragged over the ground with friction: n nodes, 0.4 m, lying at
    z = 1 mm (inside the smoothing width of the ground), some with a sphere
    half sunk in the ground on their path; node 0 held by the gripper, whose
    velocity is mostly along the rope (N(0.15, 0.05^2), N(0, 0.05^2), 0) so
    that the rope slides; mu ~ U[0.2, 0.8].  hard: kappa_fwd = 0 (the
    paper's forward mode), gradients smoothed."""
    out = []
    for rng in _streams(seed, B):
        mu = float(rng.uniform(0.2, 0.8))
        spheres = [[float(rng.uniform(0.15, 0.3)), float(rng.uniform(-0.05, 0.05)), -0.02, 0.03]] \
            if rng.uniform() < 0.5 else []
        u = np.stack([rng.normal(0.15, 0.05, T), rng.normal(0.0, 0.05, T), np.zeros(T)], axis=1)
        inst = rope(n, length=0.4, z0=0.001, T=T, grip_nodes=(0,), spheres=spheres, u=u)
        inst = inst.replace(mu=mu)
        if hard:
            inst = inst.replace(kappa_fwd=0.0)
        out.append(inst)
    return out


def friction_cloths(B: int, side: int = 8, T: int = 6, seed: int = 1028):
    """Square cloths (side x side nodes, 0.2 m) lying at z = 1 mm on the
    ground with friction mu ~ U[0.3, 0.7], the two corners of one edge
    gripped and dragged along the ground (u ~ N(0.1, 0.03^2) along x and
    N(0, 0.03^2) along y for both grippers, 0 vertically)."""
    out = []
    for rng in _streams(seed, B):
        mu = float(rng.uniform(0.3, 0.7))
        u = np.zeros((T, 6))
        for g in range(2):
            u[:, 3 * g] = rng.normal(0.1, 0.03, T)
            u[:, 3 * g + 1] = rng.normal(0.0, 0.03, T)
        inst = cloth(side, side, size=0.2, z0=0.001, T=T, u=u)
        out.append(inst.replace(mu=mu))
    return out
