"""Seeded synthetic inputs: voxel phase images, phase tables and load paths.

This module generates inputs only. It holds none of the solver's arithmetic
(no transforms, symbols, projections, constitutive updates or Krylov steps),
so the GPU library and the independent CPU checker can both be fed from it.

Geometry follows the periodic voxel RVEs of the paper's numerical examples
(Sec. 4.1: one circular inclusion in a square cell; Sec. 4.2: non-overlapping
random spheres in a cubic cell).  Voxel centres sit at (n + 1/2) h
(Sec. 3.2.1, discretization); a voxel belongs to an inclusion when the
periodic minimum-image distance from its centre to the inclusion centre is
strictly less than the radius.

Phase tables are lists of plain dicts with the keys
  model   : 'elastic' | 'j2_damage' | 'elastic_cracking' | 'gtn'
  E, nu   : Young's modulus [MPa] and Poisson ratio
  sy, H   : initial yield stress and linear plastic hardening modulus [MPa]
            (flow stress sy + H * eps_p, Sec. 2.1.2 / Sec. 4)
  dfield  : index of the non-local field that drives this phase's damage,
            -1 if the phase does not damage
  dC, dR, dmax : damage law thresholds and cap
  ell     : list with one characteristic length per non-local field,
            in units of h (Sec. 2.2.1, per-phase lengths)
A 'gtn' phase (Gurson-Tvergaard-Needleman matrix, Sec. 2.1.1) also carries
  n       : exponent of the Aravas hardening law (eq. aravas)
  q1, q2, q3, fC, fF, fN, eN, sN : yield-surface, coalescence and nucleation
            parameters (eq. yield_gurson, effective_porosity, nucleation)
  fu      : cap of the effective porosity (Sec. 4)
and drives two consecutive non-local fields, dfield (matrix plastic strain)
and dfield + 1 (trace of the plastic strain).
Tensors are in Mandel order (11, 22, 33, sqrt2*23, sqrt2*13, sqrt2*12) in 3D
and (11, 22, sqrt2*12) in 2D plane strain.
"""
from __future__ import annotations

import numpy as np

MATRIX = 0
PARTICLE = 1


# ----------------------------------------------------------------------------
# geometry
# ----------------------------------------------------------------------------
def _centres(shape):
    """Voxel-centre coordinates (n + 1/2) along each numpy axis (z, y, x)."""
    return [np.arange(n, dtype=np.float64) + 0.5 for n in shape]


def _periodic_dist2(coords, centre, shape):
    d2 = 0.0
    grids = np.meshgrid(*coords, indexing="ij")
    for g, c, n in zip(grids, centre, shape):
        d = np.abs(g - c)
        d = np.minimum(d, n - d)
        d2 = d2 + d * d
    return d2


def disc_2d(shape, centre, radius):
    """2D phase image (N2, N1) with one disc of phase 1 in a matrix of phase 0.

    `centre` is given in numpy axis order (y, x), in voxel units.
    """
    shape = tuple(int(s) for s in shape)
    d2 = _periodic_dist2(_centres(shape), centre, shape)
    return (d2 < radius * radius).astype(np.uint8)


def laminate(shape, axis, fraction_b, phases=(0, 1)):
    """Layered image: voxels with index < fraction_b * n along numpy `axis` get
    phase `phases[1]`, the rest `phases[0]`."""
    shape = tuple(int(s) for s in shape)
    n = shape[axis]
    nb = int(round(fraction_b * n))
    idx = np.arange(n) < nb
    sl = [None] * len(shape)
    sl[axis] = slice(None)
    img = np.broadcast_to(idx[tuple(sl)], shape)
    return np.where(img, phases[1], phases[0]).astype(np.uint8)


def _paint_sphere(img, c, r):
    """Set to PARTICLE every voxel whose centre lies at periodic minimum-image
    distance < r from c; returns the number of voxels newly set."""
    shape = img.shape
    if 2 * (r + 1.5) >= min(shape):
        sel = (_periodic_dist2(_centres(shape), c, shape) < r * r) & (img != PARTICLE)
        img[sel] = PARTICLE
        return int(sel.sum())
    idx, off = [], []
    for ax, n in enumerate(shape):
        lo = int(np.floor(c[ax] - r - 1.0))
        hi = int(np.ceil(c[ax] + r + 1.0))
        i = np.arange(lo, hi + 1)
        idx.append(np.mod(i, n))
        off.append(i + 0.5 - c[ax])
    d2 = (off[0][:, None, None] ** 2 + off[1][None, :, None] ** 2 + off[2][None, None, :] ** 2)
    sub = img[np.ix_(*idx)]
    sel = (d2 < r * r) & (sub != PARTICLE)
    sub[sel] = PARTICLE
    img[np.ix_(*idx)] = sub
    return int(sel.sum())


def rsa_spheres(shape, seed, radius=None, radius_range=None, count=None,
                volume_fraction=None, max_tries=1_000_000):
    """Random sequential addition of non-overlapping periodic spheres.

    Centres are uniform in [0, N)^3 (numpy axis order z, y, x) drawn from
    numpy.random.default_rng(seed); a candidate is accepted when its periodic
    minimum-image distance to every accepted centre is at least r_a + r_b.
    Radii are fixed (`radius`) or uniform in `radius_range`.  Stops at `count`
    spheres, or once the voxelised volume fraction reaches `volume_fraction`.
    Returns (phase image uint8, centres (k,3), radii (k,)).
    """
    shape = tuple(int(s) for s in shape)
    rng = np.random.default_rng(seed)
    L = np.asarray(shape, dtype=np.float64)
    img = np.zeros(shape, dtype=np.uint8)
    total = img.size
    filled = 0
    centres, radii = [], []
    tries = 0
    while True:
        if count is not None and len(centres) >= count:
            break
        if volume_fraction is not None and filled / total >= volume_fraction:
            break
        if tries >= max_tries:
            raise RuntimeError("rsa_spheres: packing failed after %d tries" % tries)
        tries += 1
        c = rng.uniform(0.0, 1.0, size=3) * L
        r = float(radius) if radius is not None else float(rng.uniform(*radius_range))
        if centres:
            d = np.abs(np.asarray(centres) - c)
            d = np.minimum(d, L - d)
            if np.any(np.sqrt((d * d).sum(axis=1)) < r + np.asarray(radii)):
                continue
        centres.append(c)
        radii.append(r)
        filled += _paint_sphere(img, c, r)
    return img, np.asarray(centres).reshape(-1, 3), np.asarray(radii)


# ----------------------------------------------------------------------------
# phase tables (materials of the worked configurations; MPa)
# ----------------------------------------------------------------------------
def matrix_j2_damage(ell, dfield=0, E=70000.0, nu=0.3, sy=300.0, H=500.0,
                     dC=0.03, dR=0.2, dmax=0.99):
    return dict(model="j2_damage", E=E, nu=nu, sy=sy, H=H, dfield=dfield,
                dC=dC, dR=dR, dmax=dmax, ell=list(ell))


def matrix_gtn(ell, dfield=0, E=70000.0, nu=0.33, sy=200.0, n=0.1, q1=1.5, q2=1.0, q3=2.25,
               fC=0.15, fF=0.25, fN=0.04, eN=0.1, sN=0.05, fu=0.6):
    """Gurson matrix with the parameters of the paper's 3D examples (Sec. 4.2:
    Al alloy, Aravas hardening with n = 0.1, f* capped at 0.6).  `ell` needs
    a length for fields dfield and dfield + 1."""
    return dict(model="gtn", E=E, nu=nu, sy=sy, H=0.0, dfield=dfield, dC=0.0, dR=1.0,
                dmax=0.0, n=n, q1=q1, q2=q2, q3=q3, fC=fC, fF=fF, fN=fN, eN=eN, sN=sN,
                fu=fu, ell=list(ell))


def particle_elastic(ell, E=400000.0, nu=0.2):
    return dict(model="elastic", E=E, nu=nu, sy=0.0, H=0.0, dfield=-1,
                dC=0.0, dR=1.0, dmax=0.0, ell=list(ell))


def particle_cracking(ell, dfield=1, E=400000.0, nu=0.2, k0=1e-3, kf=1e-2, dmax=0.99):
    return dict(model="elastic_cracking", E=E, nu=nu, sy=0.0, H=0.0, dfield=dfield,
                dC=k0, dR=kf, dmax=dmax, ell=list(ell))


def elastic_phase(E, nu, ell=(0.0,)):
    return dict(model="elastic", E=E, nu=nu, sy=0.0, H=0.0, dfield=-1,
                dC=0.0, dR=1.0, dmax=0.0, ell=list(ell))


# ----------------------------------------------------------------------------
# load paths
# ----------------------------------------------------------------------------
def uniaxial_mixed(ndim, e11):
    """Macro target: E11 prescribed, every other stress component zero
    (Sec. 4.1 and Sec. 4.2 loading).  Returns (mask, E, S) in Mandel order,
    mask 1 = stress-controlled component."""
    c = 3 if ndim == 2 else 6
    mask = np.ones(c, dtype=np.uint8)
    mask[0] = 0
    E = np.zeros(c)
    E[0] = e11
    S = np.zeros(c)
    return mask, E, S


def strain_control(ndim, Emacro):
    c = 3 if ndim == 2 else 6
    return np.zeros(c, dtype=np.uint8), np.asarray(Emacro, dtype=np.float64), np.zeros(c)


# ----------------------------------------------------------------------------
# named workloads
# ----------------------------------------------------------------------------
def workload(name, seed=None):
    """Return a dict describing one of the named workloads.

    Keys: name, shape (numpy order), ndim, phase (uint8 image), table,
    nfields, load (list of per-increment (mask, E, S)), tolerances.
    """
    if name == "disc2d_32":
        # 32x32 plane strain, centred disc of radius 8 voxels, one increment
        # to E11 = 5e-3 under uniaxial mixed control, one staggered pass.
        shape = (32, 32)
        phase = disc_2d(shape, (16.0, 16.0), 8.0)
        table = [matrix_j2_damage(ell=[2.0]), particle_elastic(ell=[1.0])]
        return dict(name=name, shape=shape, ndim=2, phase=phase, table=table, nfields=1,
                    load=[uniaxial_mixed(2, 5e-3)], max_stagger=1)
    if name == "spheres64_20":
        # 64^3, 20 spheres of radius 6 (RSA, seed 2), 50 increments to 0.05.
        shape = (64, 64, 64)
        s = 2 if seed is None else seed
        phase, _, _ = rsa_spheres(shape, s, radius=6.0, count=20)
        table = [matrix_j2_damage(ell=[2.0]), particle_elastic(ell=[1.0])]
        load = [uniaxial_mixed(3, 1e-3 * (k + 1)) for k in range(50)]
        return dict(name=name, shape=shape, ndim=3, phase=phase, table=table, nfields=1,
                    load=load, max_stagger=20)
    if name == "spheres30_128":
        # 128^3, 30 identical spheres of radius 14.94 voxels (20%, RSA seed 5);
        # lengths 0.05 L in the matrix and 0.001 L in the particles; one field.
        shape = (128, 128, 128)
        s = 5 if seed is None else seed
        phase, _, _ = rsa_spheres(shape, s, radius=14.94, count=30)
        table = [matrix_j2_damage(ell=[6.4]), particle_elastic(ell=[0.128])]
        load = [uniaxial_mixed(3, 2e-3 * (k + 1)) for k in range(20)]
        return dict(name=name, shape=shape, ndim=3, phase=phase, table=table, nfields=1,
                    load=load, max_stagger=20)
    if name.startswith("gtn_spheres30_"):
        # the 30-sphere RVE (radius 0.1167 L, 20%, RSA seed 5) at n^3 with the
        # Gurson matrix of Sec. 4.2 (two non-local fields: matrix plastic
        # strain and trace of the plastic strain, lengths 0.05 L in the matrix
        # and 0.001 L in the particles); increments of 1e-3.
        n = int(name.rsplit("_", 1)[1])
        shape = (n, n, n)
        s = 5 if seed is None else seed
        phase, _, _ = rsa_spheres(shape, s, radius=14.94 * n / 128.0, count=30)
        lm, lp = 0.05 * n, 0.001 * n
        table = [matrix_gtn(ell=[lm, lm], dfield=0), particle_elastic(ell=[lp, lp])]
        load = [uniaxial_mixed(3, 1e-3 * (k + 1)) for k in range(40)]
        return dict(name=name, shape=shape, ndim=3, phase=phase, table=table, nfields=2,
                    load=load, max_stagger=20)
    if name.startswith("spheres_two_fields_"):
        # n^3 (128 for the full size), 25% spheres with radii U(4, 8) (RSA,
        # seed 3; radii scaled by n/64 below 64^3);
        # field 0: matrix ductile damage (ell 3 in matrix, 3/50 in particles),
        # field 1: particle cracking (ell 1.5 in particles, 1.5/50 in matrix);
        # 10 increments of 1e-3 to 0.01.
        n = int(name.rsplit("_", 1)[1])
        shape = (n, n, n)
        s = 3 if seed is None else seed
        f = min(1.0, n / 64.0)
        phase, _, _ = rsa_spheres(shape, s, radius_range=(4.0 * f, 8.0 * f),
                                  volume_fraction=0.25)
        table = [matrix_j2_damage(ell=[3.0, 1.5 / 50.0], dfield=0),
                 particle_cracking(ell=[3.0 / 50.0, 1.5], dfield=1)]
        load = [uniaxial_mixed(3, 1e-3 * (k + 1)) for k in range(10)]
        return dict(name=name, shape=shape, ndim=3, phase=phase, table=table, nfields=2,
                    load=load, max_stagger=20)
    raise KeyError(name)


def batch_workload(count=64, seed0=4000, sizes=(32, 48, 64, 96)):
    """A batch of independent RVEs of uneven sizes: RVE b draws, from
    numpy.random.default_rng(seed0 + b), its edge N_b uniformly from `sizes`
    and its particle volume fraction uniformly in [0.05, 0.30]; spheres have
    radii U(4, 8) voxels (random sequential addition with that generator's
    next draws).  One non-local field: J2 damage matrix (ell 2), elastic
    particles (ell 1).  Returns a list of dicts (name, shape, phase, table,
    nfields)."""
    out = []
    table = [matrix_j2_damage(ell=[2.0]), particle_elastic(ell=[1.0])]
    for b in range(count):
        rng = np.random.default_rng(seed0 + b)
        n = int(sizes[int(rng.integers(len(sizes)))])
        vf = float(rng.uniform(0.05, 0.30))
        s = int(rng.integers(2 ** 31))
        phase, _, _ = rsa_spheres((n, n, n), s, radius_range=(4.0, 8.0), volume_fraction=vf)
        out.append(dict(name="batch_%d_%d" % (b, n), shape=(n, n, n), phase=phase,
                        table=[dict(t) for t in table], nfields=1, vf_target=vf))
    return out


def random_field(shape, seed, scale=1.0, mean=0.0):
    """Seeded normal random field (float64)."""
    rng = np.random.default_rng(seed)
    return mean + scale * rng.standard_normal(shape)
