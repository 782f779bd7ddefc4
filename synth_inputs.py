"""Seeded synthetic inputs shared by the GPU path's tests and the oracle's.

This module holds none of the method's arithmetic: it only draws gauge
fields and directions from numpy's PCG64 generator.  The paper's SESAM
ensemble (16^3 x 32, N_f=2 Wilson, Sec. II) is not available; the links
below stand in for it at the same lattice shapes.

Link generator: U_mu(x) = exp(i eps H_mu(x)) with
H = sum_{a=1..8} h_a lambda_a / 2, h_a ~ N(0,1) i.i.d. (lambda_a the
Gell-Mann matrices), drawn as standard_normal((4, V, 8)) with mu-major,
lexicographic site order; the exponential is taken through the eigen-
decomposition of H, then the matrix is re-unitarised (Gram-Schmidt on rows
0 and 1, row 2 = conj(row0 x row1)) so that det U = 1 to rounding.
"""
import numpy as np

_GELL_MANN = np.zeros((8, 3, 3), dtype=np.complex128)
_GELL_MANN[0][0, 1] = _GELL_MANN[0][1, 0] = 1
_GELL_MANN[1][0, 1], _GELL_MANN[1][1, 0] = -1j, 1j
_GELL_MANN[2][0, 0], _GELL_MANN[2][1, 1] = 1, -1
_GELL_MANN[3][0, 2] = _GELL_MANN[3][2, 0] = 1
_GELL_MANN[4][0, 2], _GELL_MANN[4][2, 0] = -1j, 1j
_GELL_MANN[5][1, 2] = _GELL_MANN[5][2, 1] = 1
_GELL_MANN[6][1, 2], _GELL_MANN[6][2, 1] = -1j, 1j
_GELL_MANN[7][0, 0] = _GELL_MANN[7][1, 1] = 1 / np.sqrt(3)
_GELL_MANN[7][2, 2] = -2 / np.sqrt(3)


def volume(dims):
    return int(dims[0] * dims[1] * dims[2] * dims[3])


def _hermitian_from_coeffs(h):
    """H = sum_a h_a lambda_a / 2 for coefficient arrays h[..., 8]."""
    return np.einsum("...a,aij->...ij", h, _GELL_MANN) * 0.5


def _expi(H, eps):
    w, Q = np.linalg.eigh(H)
    ph = np.exp(1j * eps * w)
    return np.einsum("...ij,...j,...kj->...ik", Q, ph, Q.conj())


def reunitarise(U):
    """Gram-Schmidt on rows 0 and 1, row 2 = conj(row0 x row1): SU(3)."""
    U = np.array(U, dtype=np.complex128, copy=True)
    r0 = U[..., 0, :]
    r0 = r0 / np.linalg.norm(r0, axis=-1, keepdims=True)
    r1 = U[..., 1, :]
    r1 = r1 - np.sum(r0.conj() * r1, axis=-1, keepdims=True) * r0
    r1 = r1 / np.linalg.norm(r1, axis=-1, keepdims=True)
    r2 = np.cross(r0, r1).conj()
    U[..., 0, :], U[..., 1, :], U[..., 2, :] = r0, r1, r2
    return U


def random_links(dims, eps, seed):
    """Gauge field U[4][V][3][3] = reunitarised exp(i eps H), seeded by PCG64(seed)."""
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    h = rng.standard_normal((4, V, 8))
    U = _expi(_hermitian_from_coeffs(h), eps)
    return np.ascontiguousarray(reunitarise(U))


def unit_links(dims):
    """Free field U = 1."""
    V = volume(dims)
    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    U[..., 0, 0] = U[..., 1, 1] = U[..., 2, 2] = 1
    return U


def diagonal_links(dims, thetas):
    """Constant diagonal SU(3) background:
    U_mu = diag(e^{i th1}, e^{i th2}, e^{-i(th1+th2)}) for thetas[mu] = (th1, th2)."""
    V = volume(dims)
    U = np.zeros((4, V, 3, 3), dtype=np.complex128)
    for mu in range(4):
        t1, t2 = thetas[mu]
        U[mu, :, 0, 0] = np.exp(1j * t1)
        U[mu, :, 1, 1] = np.exp(1j * t2)
        U[mu, :, 2, 2] = np.exp(-1j * (t1 + t2))
    return U


def random_su3_field(V, eps, seed):
    """One SU(3) matrix per site (gauge transformation Omega[V][3][3])."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = rng.standard_normal((V, 8))
    return np.ascontiguousarray(reunitarise(_expi(_hermitian_from_coeffs(h), eps)))


def random_su3_directions(n, seed):
    """n random traceless Hermitian 3x3 matrices X (Lie-algebra directions)."""
    rng = np.random.Generator(np.random.PCG64(seed))
    h = rng.standard_normal((n, 8))
    return _hermitian_from_coeffs(h)


def random_spinors(dims, nrhs, seed):
    """Gaussian complex spinors [nrhs][V][4][3]."""
    V = volume(dims)
    rng = np.random.Generator(np.random.PCG64(seed))
    z = rng.standard_normal((nrhs, V, 4, 3, 2))
    return np.ascontiguousarray(z[..., 0] + 1j * z[..., 1])


def z4_diluted_sources(dims, comps, seed):
    """Sources [n][V][4][3] with Z4 values {1, i, -1, -i} drawn from PCG64(seed)
    on one timeslice, spin and colour each (comps = [(t, spin, colour), ...]):
    the shape and value distribution of spin-colour-time diluted Z4 noise, for
    inputs that both sides receive as given arrays."""
    V = volume(dims)
    Vs = dims[0] * dims[1] * dims[2]
    rng = np.random.Generator(np.random.PCG64(seed))
    out = np.zeros((len(comps), V, 4, 3), dtype=np.complex128)
    for k, (t, spin, col) in enumerate(comps):
        out[k, Vs * t:Vs * (t + 1), spin, col] = 1j ** rng.integers(0, 4, Vs)
    return out


def site_index(dims, x, y, z, t):
    return x + dims[0] * (y + dims[1] * (z + dims[2] * t))


def site_coords(dims, s):
    c = []
    for L in dims:
        c.append(s % L)
        s //= L
    return tuple(c)


# Workload presets: lattice, link roughness, kappa and seeds of the configurations
# the tests and the benchmark use (links seed 1000+10*c+i, noise 2000+10*c+i).
WORKLOADS = {
    "exact_4x4x4x4": dict(dims=(4, 4, 4, 4), eps=0.3, kappa=0.10, bc_t=-1, link_seed=1000,
                          noise_seed=2000),
    "exact_8x8x8x16": dict(dims=(8, 8, 8, 16), eps=0.5, kappa=0.14, bc_t=-1, link_seed=1010,
                           noise_seed=2010),
    # kappa chosen so that plain FP64 even-odd BiCGStab needs ~400 iterations to
    # reach |Dx-b|/|b| = 1e-12 on a diluted Z4 source (scan: 0.157 -> 153,
    # 0.159 -> 304, 0.1596 -> 414, 0.16 -> 1367 iterations)
    "stoch_16x16x16x32": dict(dims=(16, 16, 16, 32), eps=0.6, kappa=0.1596, bc_t=-1,
                              link_seed=1020, noise_seed=2020),
    "tsm_8x8x8x8": dict(dims=(8, 8, 8, 8), eps=0.4, kappa=0.14, bc_t=-1, link_seed=1030,
                        noise_seed=2030),
    "tsm_12x12x12x24": dict(dims=(12, 12, 12, 24), eps=0.5, kappa=0.14, bc_t=-1,
                            link_seed=1031, noise_seed=2031),
    "tsm_16x16x16x32": dict(dims=(16, 16, 16, 32), eps=0.6, kappa=0.14, bc_t=-1,
                            link_seed=1032, noise_seed=2032),
    "grad_12x12x12x24": dict(dims=(12, 12, 12, 24), eps=0.5, kappa=0.14, bc_t=-1,
                             link_seed=1040, noise_seed=2040),
}
