"""Oracle pin for the non-symmetric elliptic-relaxation tensor in the velocity equation
(Eqs. 11, 27): with nu = 0, a uniform mean velocity and wp antisymmetric off the diagonal
(wp:R = 0 for isotropic R, so C0 eps = 0) the velocity update is deterministic,
U' = U + dt G (U - <U>) with G = (wp - eps/2 I) / k, which distinguishes wp_21 from wp_12."""
import numpy as np

import oracle as O
from paper_1006_0532_amd import workloads as W


def test_velocity_update_uses_all_nine_components():
    mesh = W.channel_mesh(6, 6, length=4.0, y0=-2.0, y1=2.0, stretch=1.0, jitter=0.0,
                          bottom=W.EDGE_SLIP, top=W.EDGE_SLIP)
    mu = np.array([0.3, -0.1, 0.05])
    f = W.uniform_fields(mesh, mean_u=tuple(mu), mean_omega=2.0, rey=(0.2, 0.2, 0.2, 0, 0, 0),
                         wp=(0.0, 0.0, 0.0, 0.0, 0.0, 0.0))
    mo = W.model_constants(nu=0.0)
    g = O.Grid(mesh, f, mo)
    wp = np.zeros((mesh.n_nodes, 3, 3))
    wp[:, 0, 1], wp[:, 1, 0] = 0.7, -0.7
    wp[:, 0, 2], wp[:, 2, 0] = -0.4, 0.4
    wp[:, 1, 2], wp[:, 2, 1] = 0.25, -0.25
    g.set_wp(wp)
    e = O.Ensemble(g, W.init_desc(ppe=4, u_sigma=0.5, src_r=0.0))
    st = e.export()
    keep = np.abs(st["y"]) < 1.0                      # far from the walls for one step
    dt = 1e-3
    e.step(dt)
    out = e.export()
    k = 0.3
    eps = 2.0 * k                                     # nu = 0 in Eq. (18)
    G = (wp[0] - 0.5 * eps * np.eye(3)) / k
    expect = st["u"] + dt * (st["u"] - mu) @ G.T
    assert np.allclose(out["u"][keep], expect[keep], rtol=1e-13, atol=1e-15)
    # the transposed tensor gives a different update
    wrong = st["u"] + dt * (st["u"] - mu) @ G
    assert not np.allclose(out["u"][keep], wrong[keep], rtol=1e-9, atol=1e-12)
