"""The Python binding checks every tensor before passing its pointer to the C ABI (which
takes raw pointers and no sizes): wrong shapes, dtypes, non-contiguous tensors, host tensors
and mixed devices raise before any library call. Host tensors suffice here because the shape
checks come before the device checks."""
import numpy as np
import pytest
import torch


@pytest.fixture(scope="module")
def efwi():
    from paper_2305_14130_amd import efwi as mod
    return mod


def _case(efwi):
    grid = efwi.make_grid(100, 200, 5.0, 5.0, 0.5e-3, 50, 20, 1e-3, 30.0, 4500.0)
    shot = efwi.Shot(50, 40, np.full(3, 50, np.int32), np.array([60, 63, 66], np.int32))
    return grid, shot


def z(*shape, dtype=torch.float32):
    return torch.zeros(shape, dtype=dtype)


def test_shape_errors_single_shot(efwi):
    grid, shot = _case(efwi)
    m, src, d = z(3, 100, 200), z(3, 50), z(3, 50)
    with pytest.raises(ValueError, match="m has shape"):
        efwi.shot_gradient(grid, shot, z(3, 100, 199), src, d)
    with pytest.raises(ValueError, match="src has shape"):
        efwi.shot_gradient(grid, shot, m, z(3, 49), d)
    with pytest.raises(ValueError, match="d_obs has shape"):
        efwi.shot_gradient(grid, shot, m, src, z(2, 50))
    with pytest.raises(ValueError, match="g has shape"):
        efwi.shot_gradient(grid, shot, m, src, d, g=z(3, 200, 100))
    with pytest.raises(TypeError, match="phi"):
        efwi.shot_gradient(grid, shot, m, src, d, phi=z(1))           # float32, not float64
    with pytest.raises(ValueError, match="phi"):
        efwi.shot_gradient(grid, shot, m, src, d, phi=z(2, dtype=torch.float64))
    with pytest.raises(ValueError, match="d_out"):
        efwi.shot_gradient(grid, shot, m, src, d, d_out=z(3, 51))
    with pytest.raises(ValueError, match="v has shape"):
        efwi.shot_jt(grid, shot, m, src, z(3, 51))
    with pytest.raises(ValueError, match="contiguous"):
        efwi.model_forward(grid, shot, z(3, 200, 100).transpose(1, 2), src)
    with pytest.raises(ValueError, match="r has shape"):
        efwi.model_adjoint(grid, shot, m, z(50, 3))
    with pytest.raises(TypeError, match="src"):
        efwi.model_forward(grid, shot, m, z(3, 50, dtype=torch.float64))


def test_host_tensors_are_refused_before_any_call(efwi):
    grid, shot = _case(efwi)
    m, src, d = z(3, 100, 200), z(3, 50), z(3, 50)
    for call in (lambda: efwi.model_forward(grid, shot, m, src),
                 lambda: efwi.model_adjoint(grid, shot, m, d),
                 lambda: efwi.shot_gradient(grid, shot, m, src, d),
                 lambda: efwi.shot_jt(grid, shot, m, src, d)):
        with pytest.raises(TypeError, match="device tensor"):
            call()


def test_batch_shape_errors(efwi):
    grid, shot = _case(efwi)
    shots = [shot, shot]
    m_ext, src, d_obs = z(2, 3, 100, 200), z(2, 3, 50), z(6, 50)
    with pytest.raises(ValueError, match="m_ext has shape"):
        efwi.batch_gradient(grid, shots, z(3, 3, 100, 200), src, d_obs)     # one component too many
    with pytest.raises(ValueError, match="src has shape"):
        efwi.batch_gradient(grid, shots, m_ext, z(1, 3, 50), d_obs)
    with pytest.raises(ValueError, match="d_obs holds"):
        efwi.batch_gradient(grid, shots, m_ext, src, z(5, 50))
    with pytest.raises(ValueError, match="phi holds"):
        efwi.batch_gradient(grid, shots, m_ext, src, d_obs, phi=z(3, dtype=torch.float64))
    with pytest.raises(ValueError, match="g_ext has shape"):
        efwi.batch_gradient(grid, shots, m_ext, src, d_obs, g_ext=z(1, 3, 100, 200))
    with pytest.raises(ValueError, match="group indices"):
        efwi.batch_gradient_grouped(grid, shots, [0, 2], m_ext, src, d_obs)
    with pytest.raises(TypeError, match="device tensor"):
        efwi.batch_gradient(grid, shots, m_ext, src, d_obs)


def test_regularizer_and_final_model_shapes(efwi):
    grid, _ = _case(efwi)
    m_ext, b, sink = z(4, 3, 100, 200), z(4, 100, 200), z(4, 100, 200, dtype=torch.uint8)
    with pytest.raises(ValueError, match="b has shape"):
        efwi.extension_regularizer(grid, m_ext, z(3, 100, 200), sink, 1.0, z(4, 3, 100, 200))
    with pytest.raises(TypeError, match="sink"):
        efwi.extension_regularizer(grid, m_ext, b, z(4, 100, 200), 1.0, z(4, 3, 100, 200))
    with pytest.raises(ValueError, match="g_ext has shape"):
        efwi.extension_regularizer(grid, m_ext, b, sink, 1.0, z(3, 3, 100, 200))
    with pytest.raises(ValueError, match="sink has shape"):
        efwi.final_model(grid, m_ext, b, z(4, 100, 199, dtype=torch.uint8))
    with pytest.raises(ValueError, match="m_out has shape"):
        efwi.final_model(grid, m_ext, b, sink, m_out=z(3, 100, 100))
    with pytest.raises(TypeError, match="device tensor"):
        efwi.final_model(grid, m_ext, b, sink)


def test_3d_model_shape(efwi):
    g3 = efwi.make_grid3d(40, 40, 40, 5.0, 5.0, 5.0, 0.5e-3, 20, 8, 1e-3, 30.0, 4500.0)
    shot = efwi.Shot(20, 20, [21], [25], src_iy=20, ch_iy=[20])
    with pytest.raises(ValueError, match="m has shape"):
        efwi.shot_gradient(g3, shot, z(3, 40, 40), z(6, 20), z(1, 20))
    with pytest.raises(ValueError, match="src has shape"):
        efwi.shot_gradient(g3, shot, z(3, 40, 40, 40), z(3, 20), z(1, 20))
