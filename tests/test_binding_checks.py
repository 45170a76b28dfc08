"""Host-side size checks of the Python binding (no GPU, no kernel launch).

The C ABI receives bare pointers, so a tensor smaller than the sizes passed
would become an out-of-bounds device access.  The binding compares every
tensor with nlos, nchan and nphi first and raises ValueError.  Here the
plan's and the network's sizes are supplied by stand-ins and the tensors are
CPU tensors: a correctly sized call gets past the size checks and stops at
the device check (TypeError), a mis-sized one raises ValueError before it.
"""
import pytest
import torch

import paper_1810_06250_amd as rs
from paper_1810_06250_amd import rmsynth as B

NCHAN, NPHI = 16, 9


@pytest.fixture(autouse=True)
def _sizes(monkeypatch):
    monkeypatch.setattr(B, "_plan_dims", lambda plan: (NCHAN, NPHI))
    monkeypatch.setattr(B, "rmsynth_mlp_info",
                        lambda mlp: dict(nchan=NCHAN, h1=64, h2=64, phi_scale=300.0))
    monkeypatch.setattr(B, "rmsynth_mlp_num_params", lambda mlp: 100)


def z(*shape, dtype=torch.float32):
    return torch.zeros(shape, dtype=dtype)


def test_execute_accepts_matching_sizes_then_needs_device_tensors():
    with pytest.raises(TypeError):
        rs.rmsynth_execute(None, z(5, NCHAN), z(5, NCHAN), 5, rs.RMSYNTH_LOS_MAJOR, rs.RMSYNTH_FP32,
                           z(5, NPHI), z(5, NPHI))
    with pytest.raises(TypeError):
        rs.rmsynth_execute(None, z(NCHAN, 5), z(NCHAN, 5), 5, rs.RMSYNTH_FREQ_MAJOR,
                           rs.RMSYNTH_FP32, z(5, NPHI), z(5, NPHI))


@pytest.mark.parametrize("case", ["short_rows", "few_los", "U_shape", "freq_transposed",
                                  "freq_more_los_than_planes", "Fq_small", "Fu_rows", "Fabs_small",
                                  "workspace_small"])
def test_execute_rejects_mismatched_sizes(case):
    Q, U = z(5, NCHAN), z(5, NCHAN)
    Fq, Fu, Fa = z(5, NPHI), z(5, NPHI), None
    layout, ws, nb = rs.RMSYNTH_LOS_MAJOR, None, 0
    if case == "short_rows":
        Q, U = z(5, NCHAN - 1), z(5, NCHAN - 1)
    elif case == "few_los":
        Q, U = z(4, NCHAN), z(4, NCHAN)
    elif case == "U_shape":
        U = z(6, NCHAN)
    elif case == "freq_transposed":
        layout = rs.RMSYNTH_FREQ_MAJOR            # a LOS-major cube passed as frequency-major
    elif case == "freq_more_los_than_planes":
        layout = rs.RMSYNTH_FREQ_MAJOR
        Q, U = z(NCHAN, 4), z(NCHAN, 4)
    elif case == "Fq_small":
        Fq = z(4, NPHI)
    elif case == "Fu_rows":
        Fu = z(5, NPHI + 1)
    elif case == "Fabs_small":
        Fa = z(3)
    elif case == "workspace_small":
        ws, nb = z(8, dtype=torch.uint8), 64
    with pytest.raises(ValueError):
        rs.rmsynth_execute(None, Q, U, 5, layout, rs.RMSYNTH_SPLIT_FP16, Fq, Fu, Fa, ws, nb)


@pytest.mark.parametrize("out", ["idx", "phi_pk", "amp", "q_pk", "u_pk"])
def test_execute_peaks_and_peaks_reject_short_outputs(out):
    vecs = {k: z(5, dtype=torch.int32 if k == "idx" else torch.float32)
            for k in ("idx", "phi_pk", "amp", "q_pk", "u_pk")}
    vecs[out] = z(4, dtype=vecs[out].dtype)
    with pytest.raises(ValueError):
        rs.rmsynth_execute_peaks(None, z(5, NCHAN), z(5, NCHAN), 5, rs.RMSYNTH_LOS_MAJOR,
                                 rs.RMSYNTH_SPLIT_BF16, z(5, NPHI), z(5, NPHI), None, vecs["idx"],
                                 vecs["phi_pk"], vecs["amp"], vecs["q_pk"], vecs["u_pk"])
    with pytest.raises(ValueError):
        rs.rmsynth_peaks(None, z(5, NPHI), z(5, NPHI), 5, vecs["idx"], vecs["phi_pk"], vecs["amp"],
                         vecs["q_pk"], vecs["u_pk"])


def test_peaks_rejects_short_spectra_and_rmsf_short_outputs():
    idx = z(5, dtype=torch.int32)
    with pytest.raises(ValueError):
        rs.rmsynth_peaks(None, z(5, NPHI - 1), z(5, NPHI - 1), 5, idx)
    with pytest.raises(ValueError):
        rs.rmsynth_rmsf(None, z(NPHI - 1), z(NPHI))
    with pytest.raises(ValueError):
        rs.rmsynth_peak_angle(None, z(5), z(5), z(4), 5, z(5))


def test_network_calls_reject_mismatched_sizes():
    with pytest.raises(ValueError):
        rs.rmsynth_mlp_infer(None, z(5, NCHAN + 1), z(5, NCHAN + 1), 5, z(5), z(5))
    with pytest.raises(ValueError):
        rs.rmsynth_mlp_infer(None, z(5, NCHAN), z(5, NCHAN), 5, z(4), z(5))
    with pytest.raises(ValueError):
        rs.rmsynth_mlp_grad(None, z(8, NCHAN), z(8, NCHAN), 8, z(8), z(7), z(100))
    with pytest.raises(ValueError):
        rs.rmsynth_mlp_grad(None, z(8, NCHAN), z(8, NCHAN), 8, z(8), z(8), z(99))
    with pytest.raises(ValueError):
        rs.rmsynth_mlp_train_step(None, z(7, NCHAN), z(7, NCHAN), 8, z(8), z(8), 1e-3)
    with pytest.raises(ValueError):
        rs.rmsynth_gate_execute(None, None, z(5, NCHAN), z(5, NCHAN), 5, 0.5, z(5, dtype=torch.int32),
                                z(5), z(4), z(5, dtype=torch.int32), None, 0)
    with pytest.raises(ValueError):
        rs.rmsynth_synth_training(None, rs.TrainSpec(), 1, 0, 5, z(5, NCHAN), z(5, NCHAN),
                                  truth=z(5, 3))
