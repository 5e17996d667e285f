"""Seeded synthetic scene generators.

This module produces *inputs only*: body masses, inertias, poses, joint anchors and
axes, contact candidate points, the subsystem partition and the interface table.  It
holds none of the solver's arithmetic (no dynamics matrices, Jacobians, errors,
factorisations or projections); both the CPU oracle and the HIP path consume the
arrays it returns.

Scenes are shaped after the examples of the paper's Sec. IV (rigid bodies and
articulated chains in contact with the ground, a co-rotated FEM body split into
pieces joined by hard constraints), at the sizes of the workloads this library is
measured on.  Every generator takes an explicit seed and uses numpy's PCG64.

Conventions shared with the solver's interface description:

* Rigid body velocity is ``(v_lin in world frame, omega in body frame)``; the body
  frame is the principal frame of the box, so the inertia is diagonal.
* ``rot`` is world-from-body, row-major 3x3.
* A revolute joint between bodies ``a`` and ``b`` lists its anchor in each body's
  frame, an orthonormal frame ``(h, u, v)`` in body ``a``'s frame (``h`` the hinge
  axis, ``u, v`` spanning its orthogonal plane; rows of ``joint_frame_a``) and the
  hinge axis in body ``b``'s frame.
* A link lists its type (0 linear: anchor-point velocities; 1 angular: angular
  velocities), bodies ``a`` and ``b`` (``b = -1`` for rows on one body), anchors in each
  body's frame and up to three row directions in ``a``'s frame (rows of ``link_frame``);
  its interface carries the kind (soft with gain ``if_k`` and ``if_alpha``, equality,
  hard inequality, or contact with ``if_mu``).
* Interfaces of a scene are listed joints first (construction order), then links, then
  contacts; all subsystems and interfaces of one scene are contiguous.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.spatial.transform import Rotation

KIND_EQUALITY = 0
KIND_CONTACT = 1
KIND_HARD_INEQ = 2
KIND_SOFT = 3

JOINT_DIM = 5
CONTACT_DIM = 3

SEED_BASE = 2302014344
GRAVITY = 9.81


def config_seed(config: int, variant: int = 0) -> int:
    """Seed of variant ``variant`` of workload ``config`` (1-based, as listed)."""
    return SEED_BASE + 1000 * config + variant


@dataclass
class RigidScenes:
    """A batch of independent rigid/articulated scenes (maximal coordinates)."""

    n_scenes: int
    # bodies
    mass: np.ndarray          # (nb,)
    inertia: np.ndarray       # (nb,3) principal, body frame
    half: np.ndarray          # (nb,3) box half extents
    pos: np.ndarray           # (nb,3)
    rot: np.ndarray           # (nb,3,3) world-from-body
    vel: np.ndarray           # (nb,3) world frame
    omega: np.ndarray         # (nb,3) body frame
    body_sub: np.ndarray      # (nb,) subsystem index
    body_local: np.ndarray    # (nb,) 6-DOF block index inside its subsystem
    # subsystems
    sub_scene: np.ndarray     # (ns,)
    sub_nbody: np.ndarray     # (ns,)
    # joints
    joint_body: np.ndarray    # (nj,2)
    joint_anchor: np.ndarray  # (nj,2,3)
    joint_frame_a: np.ndarray  # (nj,3,3) rows h_a, u_a, v_a
    joint_axis_b: np.ndarray  # (nj,3)
    joint_if: np.ndarray      # (nj,) interface index
    # contacts
    contact_body: np.ndarray  # (nc,)
    contact_point: np.ndarray  # (nc,3) body frame
    contact_mu: np.ndarray    # (nc,)
    contact_if: np.ndarray    # (nc,)
    # interfaces
    if_kind: np.ndarray       # (ni,)
    if_dim: np.ndarray        # (ni,)
    if_nsub: np.ndarray       # (ni,)
    if_sub: np.ndarray        # (ni,2), -1 when unused
    if_mu: np.ndarray         # (ni,)
    dt: float = 1e-3
    gravity: float = GRAVITY
    baumgarte: float = 0.2
    meta: dict = field(default_factory=dict)
    # links: rows between two bodies (or on one body) along directions fixed in body a's
    # frame, for interfaces of kind soft, equality, hard inequality or contact
    link_type: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))   # (nl,) 0 linear, 1 angular
    link_body: np.ndarray = field(default_factory=lambda: np.zeros((0, 2), np.int32))  # (nl,2), b = -1: one body
    link_anchor: np.ndarray = field(default_factory=lambda: np.zeros((0, 2, 3)))   # (nl,2,3) body frames
    link_frame: np.ndarray = field(default_factory=lambda: np.zeros((0, 3, 3)))    # (nl,3,3) rows f_k, a's frame
    link_if: np.ndarray = field(default_factory=lambda: np.zeros(0, np.int32))     # (nl,) interface, -1: folded
    # rows of each link; gain k and alpha of Eq. 3 for a soft link folded into its subsystem's
    # dynamics (both bodies in one subsystem, no interface): A_i += k alpha J^T J,
    # b_i -= k J^T phi (0 for links with an interface, whose soft parameters sit on it)
    link_dim: np.ndarray = None
    link_k: np.ndarray = None
    link_alpha: np.ndarray = None
    if_k: np.ndarray = None       # (ni,) soft interfaces: gain k of Eq. 3 (0 elsewhere)
    if_alpha: np.ndarray = None   # (ni,) soft interfaces: alpha of Eq. 3 (0 elsewhere)

    def __post_init__(self):
        ni = int(self.if_kind.shape[0])
        if self.if_k is None:
            self.if_k = np.zeros(ni)
        if self.if_alpha is None:
            self.if_alpha = np.zeros(ni)
        nl = int(self.link_type.shape[0])
        if self.link_dim is None:
            self.link_dim = np.array([self.if_dim[j] for j in self.link_if], np.int32).reshape(nl)
        if self.link_k is None:
            self.link_k = np.zeros(nl)
        if self.link_alpha is None:
            self.link_alpha = np.zeros(nl)

    @property
    def n_bodies(self) -> int:
        return int(self.mass.shape[0])

    @property
    def n_sub(self) -> int:
        return int(self.sub_scene.shape[0])

    @property
    def n_if(self) -> int:
        return int(self.if_kind.shape[0])

    @property
    def sub_ndof(self) -> np.ndarray:
        return (6 * self.sub_nbody).astype(np.int32)

    def state(self):
        return (self.pos.copy(), self.rot.copy(), self.vel.copy(), self.omega.copy())

    def with_state(self, pos, rot, vel, omega) -> "RigidScenes":
        import copy
        s = copy.copy(self)
        s.pos, s.rot, s.vel, s.omega = (np.ascontiguousarray(pos, np.float64), np.ascontiguousarray(rot, np.float64),
                                        np.ascontiguousarray(vel, np.float64), np.ascontiguousarray(omega, np.float64))
        return s


def _box_inertia(m: float, half) -> np.ndarray:
    a, b, c = 2.0 * np.asarray(half, dtype=np.float64)
    return m / 12.0 * np.array([b * b + c * c, a * a + c * c, a * a + b * b])


def _corners(half) -> np.ndarray:
    hx, hy, hz = half
    return np.array([[sx * hx, sy * hy, sz * hz] for sx in (-1, 1) for sy in (-1, 1) for sz in (-1, 1)])


def _perp_frame(h: np.ndarray) -> np.ndarray:
    """Rows (h, u, v): an orthonormal frame whose first row is the unit vector h."""
    h = h / np.linalg.norm(h)
    ref = np.array([1.0, 0.0, 0.0]) if abs(h[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    u = np.cross(h, ref)
    u /= np.linalg.norm(u)
    v = np.cross(h, u)
    return np.stack([h, u, v])


class _SceneBuilder:
    """Accumulates bodies/joints/contacts of one scene before the partition is known."""

    def __init__(self):
        self.mass, self.half, self.pos, self.rot = [], [], [], []
        self.inertia = []     # principal moments per body, or None for the box's
        self.joints = []      # (a, b, anchor_a, anchor_b, h_body_a, h_body_b)
        self.links = []       # (type, a, b, anchor_a, anchor_b, frame rows (d x 3), kind, k, alpha, mu)
        self.contacts = []    # (body, point, mu)

    def add_link(self, ty, a, b, anchor_a, anchor_b, frame, kind, k=0.0, alpha=0.0, mu=0.0):
        self.links.append((int(ty), a, b, np.asarray(anchor_a, float), np.asarray(anchor_b, float),
                           np.atleast_2d(np.asarray(frame, float)), int(kind), float(k), float(alpha), float(mu)))

    def add_body(self, m, half, p, R, inertia=None) -> int:
        self.inertia.append(None if inertia is None else np.asarray(inertia, dtype=np.float64))
        self.mass.append(float(m))
        self.half.append(np.asarray(half, dtype=np.float64))
        self.pos.append(np.asarray(p, dtype=np.float64))
        self.rot.append(np.asarray(R, dtype=np.float64))
        return len(self.mass) - 1

    def add_joint(self, a, b, anchor_a, anchor_b, h_a, h_b):
        self.joints.append((a, b, np.asarray(anchor_a, float), np.asarray(anchor_b, float),
                            np.asarray(h_a, float), np.asarray(h_b, float)))

    def lowest_corner_z(self, bodies=None) -> float:
        zs = []
        for k in (range(len(self.mass)) if bodies is None else bodies):
            c = _corners(self.half[k]) @ self.rot[k].T + self.pos[k]
            zs.append(c[:, 2].min())
        return float(min(zs))

    def shift_z(self, dz):
        for k in range(len(self.pos)):
            self.pos[k] = self.pos[k] + np.array([0.0, 0.0, dz])


def _assemble(scenes, partitions, dt, meta, fold_soft=False) -> RigidScenes:
    """Concatenate per-scene builders into one RigidScenes batch.

    ``partitions[s]`` maps each body of scene ``s`` to a scene-local group index; groups
    are numbered in order of first appearance and become subsystems.  ``fold_soft``: soft
    links between two bodies of one subsystem become part of that subsystem's own dynamics
    (no interface; ``link_if`` -1) instead of one-member soft interfaces.
    """
    mass, inertia, half, pos, rot = [], [], [], [], []
    body_sub, body_local, sub_scene, sub_nbody = [], [], [], []
    jb, ja, jf, jh, jif = [], [], [], [], []
    lt, lb, la, lf, lif, ld, lk, lal = [], [], [], [], [], [], [], []
    cb, cp, cm, cif = [], [], [], []
    ik, idim, ins, isub, imu, ikk, ial = [], [], [], [], [], [], []
    b0 = 0
    s0 = 0
    for s, (sc, part) in enumerate(zip(scenes, partitions)):
        ng = int(max(part)) + 1
        counts = np.zeros(ng, dtype=np.int64)
        for k in range(len(sc.mass)):
            g = part[k]
            body_sub.append(s0 + g)
            body_local.append(int(counts[g]))
            counts[g] += 1
            mass.append(sc.mass[k])
            half.append(sc.half[k])
            given = sc.inertia[k] if k < len(sc.inertia) else None
            inertia.append(_box_inertia(sc.mass[k], sc.half[k]) if given is None else given)
            pos.append(sc.pos[k])
            rot.append(sc.rot[k])
        for g in range(ng):
            sub_scene.append(s)
            sub_nbody.append(int(counts[g]))
        for (a, b, ra, rb, ha, hb) in sc.joints:
            jb.append((b0 + a, b0 + b))
            ja.append((ra, rb))
            jf.append(_perp_frame(ha))
            jh.append(hb / np.linalg.norm(hb))
            jif.append(len(ik))
            ga, gb = s0 + part[a], s0 + part[b]
            ik.append(KIND_EQUALITY)
            idim.append(JOINT_DIM)
            if ga == gb:
                ins.append(1)
                isub.append((ga, -1))
            else:
                ins.append(2)
                isub.append((ga, gb))
            imu.append(0.0)
            ikk.append(0.0)
            ial.append(0.0)
        for (ty, a, b, ra, rb, fr, kind, kk, al, mu) in sc.links:
            lt.append(ty)
            lb.append((b0 + a, b0 + b if b >= 0 else -1))
            la.append((ra, rb))
            F = np.zeros((3, 3))
            F[:fr.shape[0]] = fr
            lf.append(F)
            ld.append(fr.shape[0])
            ga = s0 + part[a]
            gb = s0 + part[b] if b >= 0 else ga
            if fold_soft and kind == KIND_SOFT and b >= 0 and ga == gb:
                lif.append(-1)
                lk.append(kk)
                lal.append(al)
                continue
            lif.append(len(ik))
            lk.append(0.0)
            lal.append(0.0)
            ik.append(kind)
            idim.append(fr.shape[0])
            if ga == gb:
                ins.append(1)
                isub.append((ga, -1))
            else:
                ins.append(2)
                isub.append((ga, gb))
            imu.append(mu)
            ikk.append(kk)
            ial.append(al)
        for (k, pt, mu) in sc.contacts:
            cb.append(b0 + k)
            cp.append(pt)
            cm.append(mu)
            cif.append(len(ik))
            ik.append(KIND_CONTACT)
            idim.append(CONTACT_DIM)
            ins.append(1)
            isub.append((s0 + part[k], -1))
            imu.append(mu)
            ikk.append(0.0)
            ial.append(0.0)
        b0 += len(sc.mass)
        s0 += ng
    nb = len(mass)
    f64 = np.float64
    i32 = np.int32
    return RigidScenes(
        n_scenes=len(scenes),
        mass=np.array(mass, f64), inertia=np.array(inertia, f64).reshape(nb, 3),
        half=np.array(half, f64).reshape(nb, 3), pos=np.array(pos, f64).reshape(nb, 3),
        rot=np.array(rot, f64).reshape(nb, 3, 3), vel=np.zeros((nb, 3)), omega=np.zeros((nb, 3)),
        body_sub=np.array(body_sub, i32), body_local=np.array(body_local, i32),
        sub_scene=np.array(sub_scene, i32), sub_nbody=np.array(sub_nbody, i32),
        joint_body=np.array(jb, i32).reshape(-1, 2), joint_anchor=np.array(ja, f64).reshape(-1, 2, 3),
        joint_frame_a=np.array(jf, f64).reshape(-1, 3, 3), joint_axis_b=np.array(jh, f64).reshape(-1, 3),
        joint_if=np.array(jif, i32),
        contact_body=np.array(cb, i32), contact_point=np.array(cp, f64).reshape(-1, 3),
        contact_mu=np.array(cm, f64), contact_if=np.array(cif, i32),
        if_kind=np.array(ik, i32), if_dim=np.array(idim, i32), if_nsub=np.array(ins, i32),
        if_sub=np.array(isub, i32).reshape(-1, 2), if_mu=np.array(imu, f64),
        dt=dt, meta=meta,
        link_type=np.array(lt, i32), link_body=np.array(lb, i32).reshape(-1, 2),
        link_anchor=np.array(la, f64).reshape(-1, 2, 3), link_frame=np.array(lf, f64).reshape(-1, 3, 3),
        link_if=np.array(lif, i32), link_dim=np.array(ld, i32), link_k=np.array(lk, f64),
        link_alpha=np.array(lal, f64), if_k=np.array(ikk, f64), if_alpha=np.array(ial, f64))


# --------------------------------------------------------------------------------------
# Serial chain of boxes (small plain-method workload)
# --------------------------------------------------------------------------------------

def chain_scene(seed: int, n_links: int = 8, links_per_sub: int = 2, mu: float = 0.5,
                planar: bool = False, clearance: float = 0.005, contact_links=None,
                dt: float = 1e-3) -> RigidScenes:
    """Serial chain of ``n_links`` boxes 0.1x0.1x0.3 m joined end to end by revolute joints.

    Long axis is body z; joints sit at +-0.15 m along it.  Hinge axes alternate body y, x,
    y, ... (all body y when ``planar``; the chain then moves in the world xz plane).  Joint
    angles are U[-0.5, 0.5] rad, masses U[0.5, 2] kg, zero velocity; the lowest corner of
    the chain is ``clearance`` above the plane z = 0.  Subsystems group ``links_per_sub``
    consecutive links.  One contact candidate per listed link (default: the lowest link
    of each subsystem) at its lowest corner (lowest bottom-edge midpoint when ``planar``,
    which keeps the scene symmetric about the xz plane).
    """
    rng = np.random.Generator(np.random.PCG64(seed))
    half = np.array([0.05, 0.05, 0.15])
    masses = rng.uniform(0.5, 2.0, n_links)
    angles = rng.uniform(-0.5, 0.5, n_links - 1)
    sc = _SceneBuilder()
    R = Rotation.from_rotvec([0.0, np.pi / 2, 0.0])
    p = np.zeros(3)
    sc.add_body(masses[0], half, p, R.as_matrix())
    for k in range(n_links - 1):
        h = np.array([0.0, 1.0, 0.0]) if (planar or k % 2 == 0) else np.array([1.0, 0.0, 0.0])
        Rn = R * Rotation.from_rotvec(h * angles[k])
        pn = p + R.apply([0.0, 0.0, half[2]]) - Rn.apply([0.0, 0.0, -half[2]])
        sc.add_body(masses[k + 1], half, pn, Rn.as_matrix())
        sc.add_joint(k, k + 1, [0.0, 0.0, half[2]], [0.0, 0.0, -half[2]], h, h)
        R, p = Rn, pn
    sc.shift_z(clearance - sc.lowest_corner_z())
    if contact_links is None:
        contact_links = []
        for g0 in range(0, n_links, links_per_sub):
            grp = list(range(g0, min(g0 + links_per_sub, n_links)))
            contact_links.append(min(grp, key=lambda k: sc.lowest_corner_z([k])))
    for k in contact_links:
        if planar:
            cands = np.array([[sx * half[0], 0.0, sz * half[2]] for sx in (-1, 1) for sz in (-1, 1)])
        else:
            cands = _corners(half)
        wz = (cands @ sc.rot[k].T + sc.pos[k])[:, 2]
        sc.contacts.append((k, cands[int(np.argmin(wz))], mu))
    part = [k // links_per_sub for k in range(n_links)]
    return _assemble([sc], [part], dt, {"kind": "chain", "seed": seed, "planar": planar})


# --------------------------------------------------------------------------------------
# Legged articulated scenes (batched workload)
# --------------------------------------------------------------------------------------

def _legged_scene(rng):
    sc = _SceneBuilder()
    torso_half = np.array([0.2, 0.125, 0.05])
    torso = sc.add_body(rng.uniform(4.0, 8.0), torso_half, np.zeros(3), np.eye(3))
    n_limb = int(rng.integers(4, 7))
    per_side = (n_limb + 1) // 2
    xs = np.linspace(-0.15, 0.15, per_side) if per_side > 1 else np.zeros(1)
    limbs = []
    for li in range(n_limb):
        side = 1.0 if li % 2 == 0 else -1.0
        hip = np.array([xs[li // 2], side * 0.1, -torso_half[2]])
        n_link = int(rng.integers(2, 5))
        parent, parent_anchor = torso, hip
        Rp = Rotation.identity()
        pp = np.zeros(3)
        chain = []
        for k in range(n_link):
            L = rng.uniform(0.1, 0.25)
            m = rng.uniform(0.5, 2.0)
            half = np.array([0.025, 0.025, L / 2])
            if k == 0:
                h = np.array([1.0, 0.0, 0.0]) if li % 2 == 0 else np.array([0.0, 1.0, 0.0])
            else:
                h = np.array([0.0, 1.0, 0.0])
            # the hinge axis is expressed in the parent's frame; the child starts aligned
            # with the parent, rotated about the hinge
            ang = rng.uniform(-0.5, 0.5)
            Rc = Rp * Rotation.from_rotvec(h * ang)
            pc = pp + Rp.apply(parent_anchor) - Rc.apply([0.0, 0.0, L / 2])
            c = sc.add_body(m, half, pc, Rc.as_matrix())
            sc.add_joint(parent, c, parent_anchor, [0.0, 0.0, L / 2], h, h)
            chain.append(c)
            parent, parent_anchor, Rp, pp = c, np.array([0.0, 0.0, -L / 2]), Rc, pc
        limbs.append(chain)
    return sc, limbs


def _partition_tree(sc, rng, p_cut=0.72, max_group=8):
    """Walk the joint list (parent before child); cut each joint with probability
    ``p_cut``, and always once the parent's group holds ``max_group`` bodies."""
    part = [-1] * len(sc.mass)
    part[0] = 0
    sizes = [1]
    for (a, b, *_rest) in sc.joints:
        g = part[a]
        if rng.random() < p_cut or sizes[g] >= max_group:
            part[b] = len(sizes)
            sizes.append(1)
        else:
            part[b] = g
            sizes[g] += 1
    return part


def legged_scenes(n_scenes: int = 1024, seed: int = None, dt: float = 1e-3,
                  p_cut: float = 0.72) -> RigidScenes:
    """Batch of legged, tree-structured articulated scenes.

    Torso box 0.4x0.25x0.1 m (U[4,8] kg); U{4..6} limbs of U{2..4} links; link boxes
    0.05x0.05xL, L~U[0.1,0.25] m, m~U[0.5,2] kg; hip hinges alternate x/y, knees y;
    joint angles U[-0.5,0.5]; lowest point U[0,5] mm above ground; U{2..16} ground
    contacts at the lowest link-box corners (at most two per link), mu~U[0.3,1.0].
    Joints are cut into subsystem boundaries with probability ``p_cut`` and always once a
    group holds 8 bodies (6 to 48 DOF per subsystem).
    """
    if seed is None:
        seed = config_seed(2)
    rng = np.random.Generator(np.random.PCG64(seed))
    scenes, parts = [], []
    for _ in range(n_scenes):
        sc, limbs = _legged_scene(rng)
        sc.shift_z(rng.uniform(0.0, 0.005) - sc.lowest_corner_z())
        m_s = int(rng.integers(2, 17))
        cands = []
        for chain in limbs:
            for k in chain:
                c = _corners(sc.half[k])
                wz = (c @ sc.rot[k].T + sc.pos[k])[:, 2]
                order = np.argsort(wz, kind="stable")[:2]
                for o in order:
                    cands.append((wz[o], k, c[o]))
        cands.sort(key=lambda t: (t[0], t[1]))
        for (_, k, pt) in cands[:m_s]:
            sc.contacts.append((k, pt, float(rng.uniform(0.3, 1.0))))
        parts.append(_partition_tree(sc, rng, p_cut=p_cut))
        scenes.append(sc)
    return _assemble(scenes, parts, dt, {"kind": "legged", "seed": seed})


# --------------------------------------------------------------------------------------
# Co-rotated FEM body split into blocks (the deformable-body workload)
# --------------------------------------------------------------------------------------

# --------------------------------------------------------------------------------------
# Cable carried by two wheeled bases (stand-in for the paper's cable example)
# --------------------------------------------------------------------------------------

LINK_LINEAR = 0
LINK_ANGULAR = 1
LINK_SPHERE = 2   # sphere contact: normal along the centres (two bodies) or a world plane (one body)


def cable_scene(seed: int = None, n_segments: int = 640, seg_per_sub: int = 4, length: float = 1.2,
                diameter: float = 0.008, young: float = 1e5, poisson: float = 0.49, density: float = 1200.0,
                mu: float = 0.5, base_mass: float = 50.0, base_half=(0.25, 0.2, 0.1), wheel_mu: float = 0.8,
                base_speed: float = 0.2, dt: float = 1e-2, gravity: bool = True,
                contacts: bool = True, fold_soft: bool = False, ang_scale: float = None) -> RigidScenes:
    """A cable of ``n_segments`` rigid segments (length ``length``, diameter ``diameter``,
    Young's modulus and Poisson ratio of the paper's cable) held at its ends by two wheeled
    bases, shaped after the paper's cable-transport example with the bases standing in for
    its mobile manipulators.

    * Segments are boxes of ``length / n_segments`` x ``diameter`` x ``diameter`` (density
      ``density``), initially straight along x at the height of the bases' tops, with small
      seeded velocities N(0, 1 cm/s).  ``seg_per_sub`` consecutive segments form a
      subsystem; each base is a subsystem of its own.
    * Neighbouring segments are coupled by four soft interfaces (Eq. 3, Cosserat-like,
      rest pose straight): stretch (linear row along the axis, k = E A / l), shear (two
      linear rows, k = G A / l), twist (angular row along the axis, k = G J / l) and bend
      (two angular rows, k = E I / l), alpha = t/2 (the spring force at the step's
      midpoint), where A = pi r^2, I = pi r^4 / 4, J = 2 I, G = E / (2 (1 + nu)).
    * Each base (``base_mass``, half extents ``base_half``, heading +y at ``base_speed``)
      holds one cable end with a ball joint (equality, three linear rows), rolls on four
      ground contacts at its bottom corners (``wheel_mu``) and may not slide sideways: a
      one-body linear row along its body x at the axle centre, an equality with zero
      error (non-holonomic).
    * Each segment has one ground-contact candidate at the bottom of its cross-section
      (``mu``).
    * The angular rows are written in length units: their directions have the length
      ``ang_scale`` (default: a segment's radius of gyration about a transverse axis) and their
      gains are divided by its square, which leaves the couplings unchanged and only rescales
      the row's lambda.  With unit directions the angular rows are weighed against the
      segments' tiny moments of inertia through a penalty (Eq. 23) set by their mass, and the
      iteration barely moves them (a 16-segment cable: 7e-1 relative error in v_hat after 60
      iterations, against 6e-6 with the scaled rows).
    * ``fold_soft``: the couplings between segments of one subsystem are part of its own
      dynamics (A_i, b_i: the other option of the remark after Eq. 6) instead of one-member
      soft interfaces; only the couplings between groups remain interfaces.  With the penalty
      of Eq. 23 the stiff folded springs raise beta_i and the iteration converges more slowly
      (the 16-segment cable: 2e-2 after 60 iterations), so the default keeps every coupling an
      interface.
    """
    if seed is None:
        seed = config_seed(6)
    rng = np.random.Generator(np.random.PCG64(seed))
    sc = _SceneBuilder()
    l = length / n_segments
    r = 0.5 * diameter
    hb = np.asarray(base_half, float)
    z = 2.0 * hb[2] + 1e-4
    m = density * l * diameter * diameter
    seg_half = np.array([0.5 * l, r, r])
    I3 = np.eye(3)
    for k in range(n_segments):
        sc.add_body(m, seg_half, [-0.5 * length + (k + 0.5) * l, 0.0, z], I3)
    bases = []
    for side in (-1, 1):
        x = side * (0.5 * length + hb[0])
        bases.append(sc.add_body(base_mass, hb, [x, 0.0, hb[2] + 1e-4], I3))
    A = np.pi * r * r
    Iy = 0.25 * np.pi * r ** 4
    G = young / (2.0 * (1.0 + poisson))
    alpha = 0.5 * dt
    ex, ey, ez = I3
    # angular rows in length units: directions of length ls with the gains divided by ls^2 (the
    # same couplings, lambda per row scaled by 1/ls), ls the segment's radius of gyration
    ls = float(ang_scale) if ang_scale is not None else float(np.sqrt((3.0 * r * r + l * l) / 12.0))
    for k in range(n_segments - 1):
        a, b = k, k + 1
        pa, pb = [0.5 * l, 0, 0], [-0.5 * l, 0, 0]
        sc.add_link(LINK_LINEAR, a, b, pa, pb, [ex], KIND_SOFT, young * A / l, alpha)
        sc.add_link(LINK_LINEAR, a, b, pa, pb, [ey, ez], KIND_SOFT, G * A / l, alpha)
        sc.add_link(LINK_ANGULAR, a, b, pa, pb, [ls * ex], KIND_SOFT, G * 2.0 * Iy / l / ls ** 2, alpha)
        sc.add_link(LINK_ANGULAR, a, b, pa, pb, [ls * ey, ls * ez], KIND_SOFT, young * Iy / l / ls ** 2, alpha)
    ends = (0, n_segments - 1)
    for side, base, seg in zip((-1, 1), bases, ends):
        # ball joint: the base's top edge centre facing the cable and the segment's outer end
        sc.add_link(LINK_LINEAR, base, seg, [-side * hb[0], 0.0, hb[2]], [side * 0.5 * l, 0.0, 0.0], I3,
                    KIND_EQUALITY)
        # no sideways slip at the axle centre (non-holonomic, velocity rows only)
        sc.add_link(LINK_LINEAR, base, -1, [0.0, 0.0, -hb[2]], [0.0, 0.0, 0.0], [ex], KIND_EQUALITY)
    vel = np.zeros((len(sc.mass), 3))
    vel[:n_segments] = rng.normal(0.0, 0.01, (n_segments, 3))
    for base in bases:
        vel[base, 1] = base_speed
    if contacts:
        for k in range(n_segments):
            sc.contacts.append((k, np.array([0.0, 0.0, -r]), mu))
        for base in bases:
            for sx in (-1, 1):
                for sy in (-1, 1):
                    sc.contacts.append((base, np.array([sx * 0.8 * hb[0], sy * 0.8 * hb[1], -hb[2]]), wheel_mu))
    part = [k // seg_per_sub for k in range(n_segments)]
    ng = (n_segments + seg_per_sub - 1) // seg_per_sub
    part += [ng, ng + 1]
    out = _assemble([sc], [part], dt, {"kind": "cable", "seed": seed, "n_segments": n_segments},
                    fold_soft=fold_soft)
    out.vel = vel
    if not gravity:
        out.gravity = 0.0
    return out


@dataclass
class FemScenes:
    """Linear-tetrahedron elastic bodies, each split into blocks (one subsystem per
    block).  Every block holds its own copies of the nodes on its faces; coincident
    copies of neighbouring blocks are tied by nodal equality interfaces (dim 3, two
    members), bottom-face copies touch the ground plane z = 0 (contact, one member).

    Node arrays list the nodes of subsystem 0, then subsystem 1, ...; a subsystem's DOF
    vector is its nodes' (x, y, z) in that order, so ``pos``/``vel`` flattened are the
    position and velocity vectors of the whole batch."""

    n_scenes: int
    sub_scene: np.ndarray     # (ns,)
    sub_nodes: np.ndarray     # (ns,) nodes per subsystem
    rest: np.ndarray          # (nn,3) rest positions
    pos: np.ndarray           # (nn,3)
    vel: np.ndarray           # (nn,3)
    tets: np.ndarray          # (nt,4) node indices (all four in one subsystem), positive rest volume
    tet_sub: np.ndarray       # (nt,)
    young: np.ndarray         # (ns,) Pa
    poisson: np.ndarray       # (ns,)
    density: float
    if_kind: np.ndarray       # (ni,)
    if_dim: np.ndarray        # (ni,)
    if_nsub: np.ndarray       # (ni,)
    if_sub: np.ndarray        # (ni,2)
    if_mu: np.ndarray         # (ni,)
    if_node: np.ndarray       # (ni,2) node of each member (-1 when unused)
    dt: float = 2e-3
    gravity: float = GRAVITY
    baumgarte: float = 0.2
    meta: dict = field(default_factory=dict)

    @property
    def n_sub(self) -> int:
        return int(self.sub_scene.shape[0])

    @property
    def n_if(self) -> int:
        return int(self.if_kind.shape[0])

    @property
    def n_nodes(self) -> int:
        return int(self.rest.shape[0])

    @property
    def n_tets(self) -> int:
        return int(self.tets.shape[0])

    @property
    def sub_ndof(self) -> np.ndarray:
        return (3 * self.sub_nodes).astype(np.int32)

    @property
    def node_off(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.sub_nodes)]).astype(np.int64)

    def with_state(self, pos, vel) -> "FemScenes":
        import copy
        s = copy.copy(self)
        s.pos = np.ascontiguousarray(np.asarray(pos, np.float64).reshape(-1, 3))
        s.vel = np.ascontiguousarray(np.asarray(vel, np.float64).reshape(-1, 3))
        return s


def _kuhn_tets():
    """Six tetrahedra of the unit cube sharing the diagonal from corner 0 to corner 7
    (corner index = x + 2y + 4z): conforming between neighbouring cubes."""
    import itertools
    out = []
    for perm in itertools.permutations(range(3)):
        c = [0]
        cur = 0
        for ax in perm:
            cur |= 1 << ax
            c.append(cur)
        out.append(c)
    return np.array(out, np.int64)


def fem_scene(seed: int = None, blocks=(8, 8, 8), nodes_per_block: int = 5, h: float = 0.01,
              jitter: float = 0.05, density: float = 1000.0, young=(1e5, 1e7), poisson=(0.3, 0.45),
              mu: float = 0.5, clearance: float = 0.05, dt: float = 2e-3, n_bodies: int = 1,
              contacts: bool = True) -> FemScenes:
    """Lattice bodies of ``blocks`` x ``nodes_per_block`` nodes per axis (one count for all
    axes, or one per axis; adjacent blocks' facing node planes coincide), lattice spacing
    ``h``, every cube split into six Kuhn
    tetrahedra.  Node positions are jittered U[-jitter, jitter] h per axis per lattice
    position (coincident copies share it); the lowest node sits ``clearance`` h above the
    ground.  Young's modulus U[young] and Poisson ratio U[poisson] per block; density in
    kg/m^3.  Coincident copies are chained by equality interfaces in block order; every
    bottom-layer copy gets a ground contact with friction ``mu``.  ``n_bodies`` bodies
    (one scene each) are placed side by side along x, at rest."""
    if seed is None:
        seed = config_seed(3)
    rng = np.random.Generator(np.random.PCG64(seed))
    bx, by, bz = (int(b) for b in blocks)
    qx, qy, qz = (int(v) for v in np.broadcast_to(np.asarray(nodes_per_block), (3,)))
    cx, cy, cz = qx - 1, qy - 1, qz - 1
    gx, gy, gz = bx * cx + 1, by * cy + 1, bz * cz + 1
    nq = qx * qy * qz
    kuhn = _kuhn_tets()
    corner = np.array([[c & 1, (c >> 1) & 1, (c >> 2) & 1] for c in range(8)], np.int64)
    rest, tets, tet_sub, sub_scene, sub_nodes, young_s, nu_s = [], [], [], [], [], [], []
    ik, idim, ins, isub, imu, inode = [], [], [], [], [], []
    n_node = 0
    n_sub = 0
    for body in range(n_bodies):
        jit = rng.uniform(-jitter, jitter, (gx, gy, gz, 3)) * h
        base = np.array([body * (gx + 2) * h, 0.0, 0.0])
        lattice = np.stack(np.meshgrid(np.arange(gx), np.arange(gy), np.arange(gz), indexing="ij"), -1) * h
        P = lattice + jit + base
        P[..., 2] += clearance * h - P[..., 2].min()
        copies = {}       # lattice position -> list of (subsystem, node)
        for kb in range(bz):
            for jb in range(by):
                for ib in range(bx):
                    s = n_sub
                    n_sub += 1
                    sub_scene.append(body)
                    sub_nodes.append(nq)
                    young_s.append(rng.uniform(*young))
                    nu_s.append(rng.uniform(*poisson))
                    for k in range(qz):
                        for j in range(qy):
                            for i in range(qx):
                                g = (ib * cx + i, jb * cy + j, kb * cz + k)
                                rest.append(P[g])
                                copies.setdefault(g, []).append((s, n_node + i + qx * (j + qy * k)))
                    for k in range(cz):
                        for j in range(cy):
                            for i in range(cx):
                                for t in kuhn:
                                    c = corner[t]
                                    ids = [n_node + (i + c[m, 0]) + qx * ((j + c[m, 1]) + qy * (k + c[m, 2]))
                                           for m in range(4)]
                                    tets.append(ids)
                                    tet_sub.append(s)
                    n_node += nq
        for g in sorted(copies):
            lst = copies[g]
            for a, b in zip(lst[:-1], lst[1:]):
                ik.append(KIND_EQUALITY)
                idim.append(3)
                ins.append(2)
                isub.append((a[0], b[0]))
                imu.append(0.0)
                inode.append((a[1], b[1]))
        if contacts:
            for g in sorted(copies):
                if g[2] != 0:
                    continue
                for (s, nd) in copies[g]:
                    ik.append(KIND_CONTACT)
                    idim.append(3)
                    ins.append(1)
                    isub.append((s, -1))
                    imu.append(mu)
                    inode.append((nd, -1))
    rest = np.array(rest, np.float64)
    tets = np.array(tets, np.int64)
    # positive rest volume: swap two vertices of any negatively oriented tetrahedron
    d = rest[tets[:, 1:]] - rest[tets[:, :1]]
    neg = np.linalg.det(d) < 0
    tets[neg, 2], tets[neg, 3] = tets[neg, 3].copy(), tets[neg, 2].copy()
    return FemScenes(
        n_scenes=n_bodies, sub_scene=np.array(sub_scene, np.int32), sub_nodes=np.array(sub_nodes, np.int32),
        rest=rest, pos=rest.copy(), vel=np.zeros_like(rest), tets=tets.astype(np.int32),
        tet_sub=np.array(tet_sub, np.int32), young=np.array(young_s), poisson=np.array(nu_s), density=float(density),
        if_kind=np.array(ik, np.int32), if_dim=np.array(idim, np.int32), if_nsub=np.array(ins, np.int32),
        if_sub=np.array(isub, np.int32).reshape(-1, 2), if_mu=np.array(imu), if_node=np.array(inode, np.int32).reshape(-1, 2),
        dt=dt, meta={"kind": "fem", "seed": seed, "blocks": (bx, by, bz), "nodes_per_block": (qx, qy, qz), "h": h})


def beam_scene(seed: int = None, pieces: int = 20, nodes_per_piece=(3, 5, 5), size=(0.5, 0.05, 0.05),
               young: float = 1e7, poisson: float = 0.45, density: float = 1000.0, mu: float = 0.5,
               dt: float = 1e-2, jitter: float = 0.0, speed: float = 0.2) -> FemScenes:
    """Stand-in of the paper's FEM beam (Sec. IV-A: a 0.05 x 0.05 x 0.5 m co-rotational beam,
    Young's modulus 10 MPa, Poisson ratio 0.45, split into 20 subsystems): ``pieces`` lattice
    blocks along x, ``nodes_per_piece`` nodes per axis in each, the lattice spacing set by the
    cross-section, just above the ground plane (friction ``mu``) and moving along its axis at
    ``speed`` (the insertion direction), so that friction acts from the first contact on.
    The paper's mesh and the
    inserting arm are not available: a regular lattice of the same size, material and piece
    count stands in (20 x 75 nodes, 4500 DOF, against the paper's 1591 nodes and 4780 DOF)."""
    if seed is None:
        seed = config_seed(7)
    q = np.broadcast_to(np.asarray(nodes_per_piece), (3,)).astype(int)
    h = float(size[1]) / (q[1] - 1)
    fs = fem_scene(seed=seed, blocks=(pieces, 1, 1), nodes_per_block=tuple(q), h=h, jitter=jitter,
                   density=density, young=(young, young), poisson=(poisson, poisson), mu=mu, dt=dt)
    fs.vel[:, 0] = speed
    fs.meta.update(kind="beam", pieces=pieces, length=h * pieces * (q[0] - 1), speed=speed)
    return fs


# --------------------------------------------------------------------------------------
# Point mass on a plane (closed-form test case)
# --------------------------------------------------------------------------------------

def point_mass_scene(m: float, vel, height: float, mu: float, dt: float = 1e-3) -> RigidScenes:
    """One small cube of mass ``m`` whose contact point is its centre (a point mass on the
    plane z = 0 at the given height), one subsystem, one contact."""
    sc = _SceneBuilder()
    half = np.array([0.01, 0.01, 0.01])
    sc.add_body(m, half, [0.0, 0.0, height], np.eye(3))
    sc.contacts.append((0, np.zeros(3), mu))
    out = _assemble([sc], [[0]], dt, {"kind": "point_mass"})
    out.vel[0] = np.asarray(vel, dtype=np.float64)
    return out


# --------------------------------------------------------------------------------------
# Random assembled problems (generic solve entry)
# --------------------------------------------------------------------------------------

@dataclass
class AssembledProblem:
    """Per-step data of Eq. (6)-(8) given directly: dense A_i, b_i, J_c,i and e_j."""

    sub_ndof: np.ndarray
    sub_scene: np.ndarray
    if_kind: np.ndarray
    if_dim: np.ndarray
    if_nsub: np.ndarray
    if_sub: np.ndarray
    if_mu: np.ndarray
    A: np.ndarray   # concatenated row-major n_i x n_i blocks
    b: np.ndarray   # concatenated n_i
    J: np.ndarray   # concatenated row-major nc_i x n_i blocks (slot order)
    e: np.ndarray   # concatenated d_j
    if_k: np.ndarray = None      # soft interfaces (kind 3): gain k_j of Eq. (3), else 0
    if_alpha: np.ndarray = None  # soft interfaces: alpha_j > 0 of Eq. (3), else 0

    @property
    def n_sub(self):
        return int(self.sub_ndof.shape[0])

    @property
    def n_if(self):
        return int(self.if_kind.shape[0])


def slot_counts(sub_ndof, if_dim, if_nsub, if_sub):
    """Number of slot rows per subsystem (sum of d_j over the interfaces it belongs to)."""
    nc = np.zeros(len(sub_ndof), dtype=np.int64)
    for j in range(len(if_dim)):
        for m in range(if_nsub[j]):
            nc[if_sub[j, m]] += if_dim[j]
    return nc


def random_assembled(seed: int, n_scenes: int = 1, subs_per_scene=(2, 4), ndof=(3, 8),
                     n_if_per_scene=(2, 6), kinds=(KIND_EQUALITY, KIND_CONTACT),
                     eq_dim=(1, 3), mu=(0.0, 1.0), cond: float = 10.0,
                     e_scale: float = 1.0, b_scale: float = 1.0, soft_k=(0.2, 2.0),
                     soft_alpha=(0.1, 1.0), max_members: int = 2) -> AssembledProblem:
    """Random well-posed assembled problems: SPD A_i with condition number ``cond``,
    Gaussian b_i, J rows and e_j.  Contact interfaces have dimension 3; soft interfaces
    (kind 3) take the equality dimensions and a gain and alpha drawn from the ranges.
    ``max_members`` > 2: coupling interfaces join 2 to ``max_members`` subsystems of their
    scene (|S_j| of Sec. III-B; the member table is then (n_if, max_members))."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sub_ndof, sub_scene, ik, idim, ins, isub, imu = [], [], [], [], [], [], []
    s0 = 0
    for s in range(n_scenes):
        ns = int(rng.integers(subs_per_scene[0], subs_per_scene[1] + 1))
        for _ in range(ns):
            sub_ndof.append(int(rng.integers(ndof[0], ndof[1] + 1)))
            sub_scene.append(s)
        ni = int(rng.integers(n_if_per_scene[0], n_if_per_scene[1] + 1))
        for _ in range(ni):
            k = int(kinds[int(rng.integers(0, len(kinds)))])
            ik.append(k)
            idim.append(3 if k == KIND_CONTACT else int(rng.integers(eq_dim[0], eq_dim[1] + 1)))
            if ns > 1 and rng.random() < 0.6:
                a, b = rng.choice(ns, size=2, replace=False)
                mem = [s0 + int(a), s0 + int(b)]
                if max_members > 2 and ns > 2:
                    # a second generator, so that two-member problems are unchanged
                    rm = np.random.Generator(np.random.PCG64(seed * 7 + 104729 + len(ik)))
                    nm = int(rm.integers(2, min(max_members, ns) + 1))
                    rest = [q for q in range(ns) if s0 + q not in mem]
                    mem += [s0 + int(q) for q in rm.choice(rest, size=nm - 2, replace=False)]
                ins.append(len(mem))
                isub.append(tuple(mem))
            else:
                ins.append(1)
                isub.append((s0 + int(rng.integers(0, ns)),))
            imu.append(float(rng.uniform(*mu)) if k == KIND_CONTACT else 0.0)
        s0 += ns
    sub_ndof = np.array(sub_ndof, np.int32)
    if_dim = np.array(idim, np.int32)
    if_nsub = np.array(ins, np.int32)
    width = max(2, max_members)
    if_sub = np.full((len(isub), width), -1, np.int32)
    for j, mem in enumerate(isub):
        if_sub[j, :len(mem)] = mem
    nc = slot_counts(sub_ndof, if_dim, if_nsub, if_sub)
    A, b, J = [], [], []
    for i, n in enumerate(sub_ndof):
        Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
        ev = np.exp(rng.uniform(0.0, np.log(cond), n))
        ev[0], ev[-1] = 1.0, cond
        scale = np.exp(rng.uniform(-1.0, 1.0))
        A.append(((Q * ev) @ Q.T * scale).ravel())
        b.append(rng.standard_normal(n) * b_scale)
        J.append(rng.standard_normal((int(nc[i]), n)).ravel())
    e = rng.standard_normal(int(if_dim.sum())) * e_scale
    # soft interfaces: gain and alpha from a generator of their own, so that problems
    # without soft interfaces are unchanged
    if_kind = np.array(ik, np.int32)
    if_k = np.zeros(len(ik))
    if_alpha = np.zeros(len(ik))
    if (if_kind == KIND_SOFT).any():
        rs = np.random.Generator(np.random.PCG64(seed + 7919))
        for j in np.nonzero(if_kind == KIND_SOFT)[0]:
            if_k[j] = rs.uniform(*soft_k)
            if_alpha[j] = rs.uniform(*soft_alpha)
    return AssembledProblem(sub_ndof=sub_ndof, sub_scene=np.array(sub_scene, np.int32),
                            if_kind=if_kind, if_dim=if_dim, if_nsub=if_nsub,
                            if_sub=if_sub, if_mu=np.array(imu, np.float64),
                            A=np.concatenate(A), b=np.concatenate(b),
                            J=np.concatenate(J) if J else np.zeros(0), e=e, if_k=if_k, if_alpha=if_alpha)


# --------------------------------------------------------------------------------------
# Boxes stacked around controlled arms (the large mixed workload, rigid part)
# --------------------------------------------------------------------------------------

def mixed_scenes(n_scenes: int = 64, grid=(8, 4), layers: int = 2, n_arm_links: int = 7, seed: int = None,
                 dt: float = 1e-3, arm_gain: float = 2e3, arm_damping: float = 0.02, fold_arm: bool = True,
                 gap: float = 1e-3) -> RigidScenes:
    """Boxes stacked in columns next to a position-controlled arm, ``n_scenes`` scenes.

    * Boxes: a ``grid`` of columns of ``layers`` boxes, footprint half extents U[0.025, 0.15] m
      per column (sizes U[0.05, 0.3] m), heights U[0.05, 0.3] m, density U[500, 2000] kg/m^3,
      each box one subsystem.  Contacts (mu U[0.2, 1.0] each): the bottom layer's four bottom
      corners on the ground plane (one member); each upper box on the one below at its four
      bottom corners (two-member contact links, normal +z); neighbouring bottom-layer columns
      face to face at the middle of the facing sides (two-member contact links).  Columns stand
      ``gap`` apart, upper boxes ``gap`` above the lower ones, the bottom layer U[0, gap] above
      the ground.
    * Arm: ``n_arm_links`` links (boxes 0.06 x 0.06 x 0.2 m, U[1, 3] kg) joined by revolute
      joints with hinge axes alternating z and y, standing upright beside the first column;
      the base link is held still by velocity rows on it alone (three linear, three angular);
      every joint is held at its initial angle by a soft angular coupling (Eq. 3, gain
      ``arm_gain`` N m/rad, alpha ``arm_damping`` s), the controller of a position-controlled
      arm; the whole arm is one subsystem, its couplings folded into its dynamics when
      ``fold_arm`` (the remark after Eq. 6).  The second link touches the first column's
      bottom box side (a two-member contact link).
    """
    if seed is None:
        seed = config_seed(5)
    rng = np.random.Generator(np.random.PCG64(seed))
    gx, gy = (int(g) for g in grid)
    scenes, parts = [], []
    ex, ey, ez = np.eye(3)
    for _ in range(n_scenes):
        sc = _SceneBuilder()
        part = []
        hxy = rng.uniform(0.025, 0.15, (gx, gy, 2))
        wx = hxy[..., 0].max(axis=1)   # widest half extent of each grid row / column
        wy = hxy[..., 1].max(axis=0)
        cx = np.concatenate([[0.0], np.cumsum(wx[:-1] + wx[1:] + gap)])
        cy = np.concatenate([[0.0], np.cumsum(wy[:-1] + wy[1:] + gap)])
        col = {}
        for i in range(gx):
            for j in range(gy):
                z0 = rng.uniform(0.0, gap)
                below = None
                for k in range(layers):
                    hz = rng.uniform(0.025, 0.15)
                    half = np.array([hxy[i, j, 0], hxy[i, j, 1], hz])
                    m = rng.uniform(500.0, 2000.0) * 8.0 * half.prod()
                    b = sc.add_body(m, half, [cx[i], cy[j], z0 + hz], np.eye(3))
                    part.append(len(part))
                    if below is None:
                        for c in _corners(half):
                            if c[2] < 0:
                                sc.contacts.append((b, c, float(rng.uniform(0.2, 1.0))))
                    else:
                        hb = sc.half[below]
                        for sx in (-1, 1):
                            for sy in (-1, 1):
                                sc.add_link(LINK_LINEAR, b, below, [sx * half[0], sy * half[1], -hz],
                                            [sx * half[0], sy * half[1], hb[2]], [ez, ex, ey], KIND_CONTACT,
                                            mu=float(rng.uniform(0.2, 1.0)))
                    if k == 0:
                        col[(i, j)] = b
                    z0 += 2.0 * hz + gap
                    below = b
        for i in range(gx):
            for j in range(gy):
                a = col[(i, j)]
                ha = sc.half[a]
                if i + 1 < gx:
                    b = col[(i + 1, j)]
                    hb = sc.half[b]
                    h = min(ha[2], hb[2])
                    sc.add_link(LINK_LINEAR, a, b, [ha[0], 0.0, h - ha[2]], [-hb[0], 0.0, h - hb[2]], [-ex, ey, ez],
                                KIND_CONTACT, mu=float(rng.uniform(0.2, 1.0)))
                if j + 1 < gy:
                    b = col[(i, j + 1)]
                    hb = sc.half[b]
                    h = min(ha[2], hb[2])
                    sc.add_link(LINK_LINEAR, a, b, [0.0, ha[1], h - ha[2]], [0.0, -hb[1], h - hb[2]], [-ey, ez, ex],
                                KIND_CONTACT, mu=float(rng.uniform(0.2, 1.0)))
        # the arm, upright beside column (0, 0)
        b00 = col[(0, 0)]
        h00 = sc.half[b00]
        ah = np.array([0.03, 0.03, 0.1])
        base_xy = np.array([cx[0] - h00[0] - ah[0] - gap, cy[0]])
        arm_part = len(part)
        prev = None
        for k in range(n_arm_links):
            z = 2.0 * ah[2] * k + ah[2] + 1e-3
            b = sc.add_body(rng.uniform(1.0, 3.0), ah, [base_xy[0], base_xy[1], z], np.eye(3))
            part.append(arm_part)
            if prev is None:
                sc.add_link(LINK_LINEAR, b, -1, [0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [ex, ey, ez], KIND_EQUALITY)
                sc.add_link(LINK_ANGULAR, b, -1, [0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [ex, ey, ez], KIND_EQUALITY)
            else:
                h = ez if k % 2 == 1 else ey
                sc.add_joint(prev, b, [0.0, 0.0, ah[2]], [0.0, 0.0, -ah[2]], h, h)
                sc.add_link(LINK_ANGULAR, prev, b, [0.0, 0.0, 0.0], [0.0, 0.0, 0.0], [h], KIND_SOFT, arm_gain,
                            arm_damping)
            if k == 1:
                # the arm's second link against the side of column (0, 0)'s bottom box
                zc = min(z, 2.0 * h00[2]) - 0.5 * min(ah[2], h00[2])
                sc.add_link(LINK_LINEAR, b00, b, [-h00[0], 0.0, zc - h00[2]], [ah[0], 0.0, zc - z], [ex, ey, ez],
                            KIND_CONTACT, mu=float(rng.uniform(0.2, 1.0)))
            prev = b
        scenes.append(sc)
        parts.append(part)
    out = _assemble(scenes, parts, dt, {"kind": "mixed", "seed": seed, "grid": (gx, gy), "layers": layers},
                    fold_soft=fold_arm)
    return out


# --------------------------------------------------------------------------------------
# Granular stirring stand-in (spheres in a box, an arm with a stirrer)
# --------------------------------------------------------------------------------------

def stir_scene(seed: int = None, n_side: int = 6, radius: float = 0.01, mass: float = 0.004, gap: float = 2e-4,
               mu: float = 0.5, n_arm_links: int = 7, arm_gain: float = 50.0, arm_damping: float = 0.02,
               stirrer_radius: float = 0.02, stirrer_mass: float = 0.05, spin: float = 3.0, reach: float = 0.02,
               dt: float = 1e-2) -> RigidScenes:
    """Stand-in of the paper's granular stirring (Sec. IV-A: 216 spheres of 1 cm radius and 4 g
    stirred by an arm's end effector in a box, each sphere and the robot one subsystem, 10 ms
    steps).

    * ``n_side``^3 spheres on a cubic lattice of pitch 2 r + ``gap`` in a box (the ground plane
      and four walls ``gap`` beyond the outer spheres); sphere contacts (link type
      ``LINK_SPHERE``, mu ``mu``) between lattice neighbours and between boundary spheres and the
      ground or a wall (a fixed contact set: the candidates of the packed start).
    * The arm: ``n_arm_links`` boxes 0.04 x 0.04 x 0.1 m (0.2 kg) hanging from a base above the
      box centre, held still by velocity rows on the base, revolute joints alternating z and y,
      each held at its angle by a soft angular coupling (``arm_gain`` N m/rad, alpha
      ``arm_damping`` s) folded into the arm subsystem; a stirrer sphere (``stirrer_radius``,
      ``stirrer_mass``) on a ball joint at the last link's end, resting on the top layer, with
      sphere contacts to the granular spheres within reach.  The arm starts turning about its
      first joint at ``spin`` rad/s, so the stirrer sweeps through the spheres and the
      controller's springs swing it back.
    The paper's robot, end effector and box are not available; this scene has their counts
    (217 subsystems) and the spheres' size and mass."""
    if seed is None:
        seed = config_seed(8)
    rng = np.random.Generator(np.random.PCG64(seed))
    sc = _SceneBuilder()
    I3 = np.eye(3)
    ex, ey, ez = I3
    pitch = 2.0 * radius + gap
    c0 = -0.5 * (n_side - 1) * pitch
    inertia = np.full(3, 0.4 * mass * radius * radius)
    grid = {}
    for k in range(n_side):
        for j in range(n_side):
            for i in range(n_side):
                p = [c0 + i * pitch, c0 + j * pitch, radius + gap + k * pitch]
                p = np.asarray(p) + rng.uniform(-0.05, 0.05, 3) * gap
                grid[(i, j, k)] = sc.add_body(mass, [radius] * 3, p, I3, inertia=inertia)
    n_sph = len(grid)
    wall = -c0 + radius + gap
    for (i, j, k), b in grid.items():
        for di, dj, dk in ((1, 0, 0), (0, 1, 0), (0, 0, 1)):
            nb = grid.get((i + di, j + dj, k + dk))
            if nb is not None:
                sc.add_link(LINK_SPHERE, b, nb, [radius, 0, 0], [radius, 0, 0], I3, KIND_CONTACT, mu=mu)
        planes = []
        if k == 0:
            planes.append((ez, ex, ey, 0.0))
        if i == 0:
            planes.append((ex, ey, ez, -wall))
        if i == n_side - 1:
            planes.append((-ex, ey, ez, -wall))
        if j == 0:
            planes.append((ey, ez, ex, -wall))
        if j == n_side - 1:
            planes.append((-ey, ez, ex, -wall))
        for (nrm, t1, t2, off) in planes:
            sc.add_link(LINK_SPHERE, b, -1, [radius, 0, 0], [off, 0, 0], [nrm, t1, t2], KIND_CONTACT, mu=mu)
    # the arm, hanging straight above the box and tilted by ``tilt`` about y (base included),
    # so that turning about the first joint's (tilted) axis sweeps the stirrer round a cone;
    # every joint then sits at its controller's rest angle; the stirrer rests on the top layer
    # at ``reach`` from the box centre
    ah = np.array([0.02, 0.02, 0.05])
    top = radius + gap + (n_side - 1) * pitch
    z_stir = top + radius + gap + stirrer_radius
    tilt = 0.5
    R_t = Rotation.from_rotvec([0.0, tilt, 0.0])
    rots, cents = [], []
    end = np.zeros(3)   # the top anchor of the current link, relative to the base link's top
    for k in range(n_arm_links):
        R = R_t
        c = end + R.apply([0.0, 0.0, -ah[2]])
        rots.append(R)
        cents.append(c)
        end = end + R.apply([0.0, 0.0, -2.0 * ah[2]])
    stir_rel = end + rots[-1].apply([0.0, 0.0, -stirrer_radius])
    anchor = np.array([reach - stir_rel[0], -stir_rel[1], z_stir - stir_rel[2]])
    links = []
    for k in range(n_arm_links):
        b = sc.add_body(0.2, ah, anchor + cents[k], rots[k].as_matrix())
        if k == 0:
            sc.add_link(LINK_LINEAR, b, -1, [0, 0, 0], [0, 0, 0], I3, KIND_EQUALITY)
            sc.add_link(LINK_ANGULAR, b, -1, [0, 0, 0], [0, 0, 0], I3, KIND_EQUALITY)
        else:
            # hinge axis in the parent's frame; the tilt sits at the third joint
            h = ez if k % 2 == 1 else ey
            ha = h
            hb = (rots[k].inv() * rots[k - 1]).apply(h)
            sc.add_joint(links[-1], b, [0, 0, -ah[2]], [0, 0, ah[2]], ha, hb)
            sc.add_link(LINK_ANGULAR, links[-1], b, [0, 0, 0], [0, 0, 0], [h], KIND_SOFT, arm_gain, arm_damping)
        links.append(b)
    ms = stirrer_mass
    stir = sc.add_body(ms, [stirrer_radius] * 3, anchor + stir_rel, I3,
                       inertia=np.full(3, 0.4 * ms * stirrer_radius ** 2))
    sc.add_link(LINK_LINEAR, links[-1], stir, [0, 0, -ah[2]], R_t.apply([0.0, 0.0, stirrer_radius]), I3,
                KIND_EQUALITY)
    # stirrer contacts: the granular spheres within reach of its surface
    for key, b in grid.items():
        if np.linalg.norm(sc.pos[b] - sc.pos[stir]) < stirrer_radius + radius + pitch:
            sc.add_link(LINK_SPHERE, b, stir, [radius, 0, 0], [stirrer_radius, 0, 0], I3, KIND_CONTACT, mu=mu)
    part = list(range(n_sph)) + [n_sph] * (n_arm_links + 1)
    out = _assemble([sc], [part], dt, {"kind": "stir", "seed": seed, "n_spheres": n_sph}, fold_soft=True)
    # the arm below its first joint turns about that joint's axis (the base's z axis)
    pivot = anchor + R_t.apply([0.0, 0.0, -2.0 * ah[2]])
    omega_w = spin * R_t.apply([0.0, 0.0, 1.0])
    for b in links[1:] + [stir]:
        out.vel[b] = np.cross(omega_w, out.pos[b] - pivot)
        out.omega[b] = out.rot[b].T @ omega_w
    return out
