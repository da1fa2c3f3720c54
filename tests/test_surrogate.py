"""CPU checks of the learned-initial-state model (paper_2010_15069_amd.surrogate): its spectral layer
against the plain definition written out with NumPy's FFT, the loss's phase invariance, the
weights round trip and the input encoding."""
import numpy as np
import pytest
import torch

from paper_2010_15069_amd import surrogate
from workloads import Params, sweep_instances


def test_spectral_layer_matches_its_definition():
    torch.manual_seed(0)
    cin, cout, m, h, w = 3, 2, 3, 16, 12
    layer = surrogate.SpectralConv2d(cin, cout, m)
    u = torch.randn(2, cin, h, w)
    got = layer(u).detach().numpy()
    # definition: real FFT over (y, x); keep k_y in {0..m-1} and {h-m..h-1}, k_x in {0..m-1};
    # out_hat[o] = sum_i u_hat[i] W[k, i, o] there, zero elsewhere; inverse real FFT
    U = np.fft.rfft2(u.numpy().astype(np.float64))
    W = layer.weight.detach().numpy().astype(np.complex128)   # [2m, m, cin, cout]
    O = np.zeros((2, cout, h, w // 2 + 1), dtype=np.complex128)
    rows = list(range(m)) + list(range(h - m, h))
    for b in range(2):
        for r_i, ky in enumerate(rows):
            for kx in range(m):
                O[b, :, ky, kx] = U[b, :, ky, kx] @ W[r_i, kx]
    ref = np.fft.irfft2(O, s=(h, w))
    assert np.allclose(got, ref, atol=1e-5 * np.abs(ref).max())


def test_infidelity_is_zero_for_the_same_state_up_to_a_global_phase():
    torch.manual_seed(1)
    t = torch.randn(3, 4, 8, 8)
    phase = 0.7
    c, s = np.cos(phase), np.sin(phase)
    p = t.clone()
    p[:, 0::2] = c * t[:, 0::2] - s * t[:, 1::2]
    p[:, 1::2] = s * t[:, 0::2] + c * t[:, 1::2]
    assert float(surrogate.infidelity(2.5 * p, t)) < 1e-6
    q = torch.randn(3, 4, 8, 8)
    assert 0.5 < float(surrogate.infidelity(q, t)) <= 1.0


def test_weights_round_trip(tmp_path):
    torch.manual_seed(2)
    model = surrogate.FNO2d(width=8, modes=4, layers=2)
    x = torch.randn(1, surrogate.IN_CHANNELS, 16, 16)
    path = str(tmp_path / "w32.safetensors")
    surrogate.save(model, path, dtype=torch.float32)
    back = surrogate.load(path)
    assert torch.equal(model(x), back(x))
    assert back.config() == {"width": 8, "modes": 4, "layers": 2}
    path = str(tmp_path / "w16.safetensors")
    surrogate.save(model, path)          # default: fp16 storage
    back = surrogate.load(path)
    ref = model(x)
    assert torch.allclose(back(x), ref, atol=2e-3 * float(ref.abs().max()))


def test_encoding_and_prediction_shapes():
    ps = sweep_instances(seed=5, sizes=(32,), per_size=3)
    x = surrogate.encode(ps, "cpu")
    assert x.shape == (3, surrogate.IN_CHANNELS, 32, 32) and x.dtype == torch.float32
    assert torch.isfinite(x).all()
    model = surrogate.FNO2d(width=8, modes=4, layers=2)
    psi = surrogate.predict(model, ps, "cpu")
    for p, s in zip(ps, psi):
        dx = 2 * p.xmax / p.nx
        assert s.shape == (2, 32, 32)
        assert abs(dx * dx * np.sum(np.abs(s) ** 2) - p.norm0) < 1e-9


def test_bf16_spectral_mix_is_the_complex_product():
    # the GPU path's real-block bfloat16 form against the complex fp32 product
    import torch
    from paper_2010_15069_amd.surrogate import spectral_mix
    g = torch.Generator().manual_seed(0)
    a = torch.complex(torch.randn(12, 3, 32, generator=g), torch.randn(12, 3, 32, generator=g))
    w = torch.complex(torch.randn(12, 32, 32, generator=g), torch.randn(12, 32, 32, generator=g)) / 32
    ref = spectral_mix(a, w, bf16=False)
    got = spectral_mix(a, w, bf16=True)
    assert got.dtype == ref.dtype and got.shape == ref.shape
    rel = float((got - ref).abs().max() / ref.abs().max())
    assert rel < 3e-2, rel           # bfloat16 inputs: 8 significant bits
    # with inputs exact in bfloat16 what remains is the rounding of the result (bfloat16 on the
    # host; the GPU returns the fp32 accumulation)
    a16 = torch.complex(a.real.bfloat16().float(), a.imag.bfloat16().float())
    w16 = torch.complex(w.real.bfloat16().float(), w.imag.bfloat16().float())
    rel16 = float((spectral_mix(a16, w16, bf16=True) - spectral_mix(a16, w16, bf16=False)).abs().max()
                  / ref.abs().max())
    assert rel16 < 4e-3, rel16


def test_encoding_on_the_device_matches_the_host_encoding():
    # encode_on (torch, any device) and encode (numpy) give the same input maps; a set with a
    # non-positive coupling sum takes the host path
    from paper_2010_15069_amd import surrogate
    from workloads import Params, preset, sweep_instances
    ps = sweep_instances(seed=4, sizes=(256,), per_size=3) + [preset("ground_256")]
    a = surrogate.encode(ps, "cpu")
    b = surrogate.encode_on(ps, "cpu")
    assert a.dtype == b.dtype == torch.float32 and a.shape == b.shape
    assert float((a - b).abs().max()) <= 1e-6 * float(a.abs().max())
    odd = [Params(nx=64, ny=64, g_uu=-1.0, g_dd=1.0, g_ud=0.5)]
    assert torch.equal(surrogate.encode_on(odd, "cpu"), surrogate.encode(odd, "cpu"))
