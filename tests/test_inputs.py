"""The device-side sphere generator (used where the host one would be too
slow) reproduces the host generator: level set at nodes and face centres
exactly, exact edge roots to an ulp."""
import numpy as np
import torch

from paper_2509_26361_amd import inputs as I


def test_sphere_shape_device_matches_host():
    for n, c, R in ((16, (0.41, 0.37, 0.52), 0.23), (24, (0.35, 0.35, 0.35), 0.15)):
        sh = I.sphere_shape(n, c, R)
        phi, faces, roots = I.sphere_shape_device(n, c, R, "cpu")
        assert np.array_equal(sh.phi_nodes, phi.numpy())
        for k in range(3):
            assert np.array_equal(sh.phi_faces[k], faces[k].numpy())
            assert np.max(np.abs(sh.s_exact[k] - roots[k].numpy())) <= 4.5e-16
