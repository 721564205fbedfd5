"""The largest lattices the library takes: a hop whose component arrays span
more than 2^31 bytes, checked against the free-field plane-wave symbol at
sampled sites (a closed form that holds at any size, so no oracle run on 4e8
sites is needed).

The fields are built directly in the internal layout on the device: the
canonical import of fields this large would need another copy in HBM.  The
even-odd order used to build and read them is the one include/tmhop.h
documents; the kernel computes neighbours from its own coordinates, so an
input built in any other order would not be an eigenvector of its operator.
"""

import numpy as np
import pytest
import torch

import fieldgen
import paper_1311_4521_amd as tm
from test_oracle import free_symbol

pytestmark = pytest.mark.gpu

CHUNK = 1 << 24


def eo_coords(dims, parity, i):
    """Coordinates (t, x, y, z) of even-odd index i on a parity (device ints):
    lex = 2 i + ((t + x + y + parity) & 1), LZ even."""
    L = dims
    l2 = 2 * i
    z0 = l2 % L[3]
    r = l2 // L[3]
    y = r % L[2]
    r = r // L[2]
    x = r % L[1]
    t = r // L[1]
    z = z0 + ((t + x + y + parity) & 1)
    return t, x, y, z


def plane_wave_into(buf, lat, dims, parity, p, u):
    """buf (12, S, 2) float64 <- exp(i p.x) u on the sites of one parity."""
    dev = buf.device
    uc = torch.from_numpy(u.reshape(12)).to(dev)
    for s0 in range(0, lat.Vh, CHUNK):
        i = torch.arange(s0, min(lat.Vh, s0 + CHUNK), device=dev, dtype=torch.int64)
        t, x, y, z = eo_coords(dims, parity, i)
        ph = p[0] * t.double() + p[1] * x.double() + p[2] * y.double() + p[3] * z.double()
        e = torch.polar(torch.ones_like(ph), ph)
        v = uc[:, None] * e[None, :]
        buf[:, s0:s0 + len(i), 0] = v.real
        buf[:, s0:s0 + len(i), 1] = v.imag
        del i, t, x, y, z, ph, e, v


@pytest.mark.slow
def test_free_field_plane_wave_beyond_2gib_component_arrays():
    dims = (192, 128, 128, 96)             # 301,989,888 sites, Vh * 16 B = 2.4 GB
    theta = (1.0, 0.5, 0.0, 0.25)
    n = (3, 1, 5, 2)
    kappa = 0.15
    torch.cuda.empty_cache()
    lat = tm.Lattice(dims)
    assert lat.S * 16 > 2 ** 31            # FP64 component arrays pass 2 GiB
    p = np.array([(2 * n[m] + theta[m]) * np.pi / dims[m] for m in range(4)])
    u = fieldgen.rng(971).standard_normal((4, 3)) + 1j * fieldgen.rng(972).standard_normal((4, 3))
    # unit links in two-row FP64 storage: rows (1,0,0) and (0,1,0)
    G = lat.new_gauge(tm.F64_R12, zero=True)
    G[:, :, 0, :, 0] = 1.0
    G[:, :, 4, :, 0] = 1.0
    psi = lat.new_spinor(tm.F64_R12, zero=False)
    plane_wave_into(psi, lat, dims, 1, p, u)
    out = lat.new_spinor(tm.F64_R12, zero=False)
    tm.hop_apply(lat, "eo", out, G, psi, kappa, theta, tm.F64_R12)
    torch.cuda.synchronize()
    del G, psi
    g = fieldgen.rng(973)
    Vh = lat.Vh
    sites = np.unique(np.concatenate([np.arange(64), Vh - 1 - np.arange(64),
                                      (1 << 27) + np.arange(-64, 64), g.integers(0, Vh, 4096)]))
    idx = torch.from_numpy(sites).to(out.device)
    got = out[:, idx, :].cpu().numpy()
    got = (got[..., 0] + 1j * got[..., 1]).T.reshape(-1, 4, 3)
    t, x, y, z = eo_coords(dims, 0, idx)
    c = torch.stack([t, x, y, z], 1).cpu().numpy().astype(np.float64)
    want = np.exp(1j * (c @ p))[:, None, None] * (free_symbol(p, kappa) @ u)[None]
    err = np.linalg.norm((got - want).reshape(len(sites), -1), axis=1)
    ref = np.linalg.norm(want.reshape(len(sites), -1), axis=1)
    assert np.max(err / ref) <= 1e-13
