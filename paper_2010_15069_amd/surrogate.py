"""Learned initial state for imaginary-time relaxation: a small Fourier neural operator (FNO).

It maps the problem's parameters on the grid to a two-component order parameter that starts the
plain split-step relaxation closer to the ground state.  The solver has the last word: a
predicted state is only a starting point, and the imaginary-time steps that follow are the
ordinary ones.

Model (one instance of the neural-operator family: lift, Fourier layers, project):
  * input channels on the n x n grid: V / max V, g / 100, Omega / 3, delta / 0.5, x / xmax,
    y / ymax, and the Thomas-Fermi amplitudes of both components (scaled to unit maximum);
  * lift: pointwise linear to `width` channels;
  * `layers` Fourier layers: u <- GELU(K u + W u), where K keeps the lowest `modes` x `modes`
    Fourier modes of u (both signs of k_y, k_x >= 0 of the real transform) and mixes channels per
    mode with a learned complex matrix, and W is pointwise linear;
  * project: pointwise linear (width -> 128 -> 4): re and im of the up and down components;
  * the output is normalised to the atom number.
On the GPU every channel mixing runs on the bfloat16 matrix cores with fp32 accumulation: the
pointwise layers under bfloat16 autocast, and the spectral mixing as one batched real product that
holds the complex one ([re a | im a] times the real 2x2-block form of the complex weight).  On the
host the spectral mixing stays a complex fp32 product.

Training minimises the phase-invariant infidelity 1 - |<p, t>|^2 / (<p, p> <t, t>) between the
predicted and the relaxed states (both components, one global phase), so the arbitrary global phase
of a ground state does not enter.
"""
from __future__ import annotations

import math
import time

import numpy as np
import torch

from workloads import Params, grid_axes, thomas_fermi_state

IN_CHANNELS = 8


def encode(params_list, device) -> torch.Tensor:
    """(B, IN_CHANNELS, ny, nx) float32 input maps for a list of same-grid parameter sets."""
    maps = []
    for p in params_list:
        x, y, _, _ = grid_axes(p)
        X, Y = np.meshgrid(x, y)
        V = 0.5 * (p.wx ** 2 * X ** 2 + p.wy ** 2 * Y ** 2)
        tf = thomas_fermi_state(p, seed=0, noise=0.0)
        amp = np.abs(tf)
        amp = amp / max(float(amp.max()), 1e-30)
        ones = np.ones_like(X)
        maps.append(np.stack([V / V.max(), ones * p.g_uu / 100.0, ones * p.omega / 3.0, ones * p.delta / 0.5,
                              X / p.xmax, Y / p.ymax, amp[0], amp[1]]).astype(np.float32))
    return torch.from_numpy(np.stack(maps)).to(device)


def encode_on(params_list, device) -> torch.Tensor:
    """`encode` computed with torch on `device` (fp64 there, one rounding to fp32 at the end), so a
    prediction on the GPU starts without a host round trip.  The Thomas-Fermi amplitudes scaled to
    unit maximum do not depend on the state's normalisation: sqrt((mu - V)_+ / g_s) over its maximum.
    Parameter sets with a non-positive coupling sum fall back to `encode`."""
    if any(p.g_uu + p.g_ud <= 0.0 or p.g_dd + p.g_ud <= 0.0 for p in params_list):
        return encode(params_list, device)
    maps = []
    for p in params_list:
        x, y, _, _ = grid_axes(p)
        X = torch.as_tensor(x, dtype=torch.float64, device=device).expand(p.ny, p.nx)
        Y = torch.as_tensor(y, dtype=torch.float64, device=device)[:, None].expand(p.ny, p.nx)
        V = 0.5 * (p.wx ** 2 * X * X + p.wy ** 2 * Y * Y)
        gu, gd = p.g_uu + p.g_ud, p.g_dd + p.g_ud
        mu = math.sqrt(p.norm0 * p.wx * p.wy * gu / (2.0 * math.pi))
        n = torch.clamp(mu - V, min=0.0)
        amp = torch.stack([torch.sqrt(n / gu), torch.sqrt(n / gd)])
        amp = amp / torch.clamp(amp.max(), min=1e-30)
        ones = torch.ones_like(X)
        maps.append(torch.stack([V / V.max(), ones * (p.g_uu / 100.0), ones * (p.omega / 3.0),
                                 ones * (p.delta / 0.5), X / p.xmax, Y / p.ymax, amp[0], amp[1]]))
    return torch.stack(maps).to(torch.float32)


def to_psi(out: torch.Tensor, params_list) -> list:
    """Network output (B, 4, ny, nx) -> list of (2, ny, nx) complex128 states normalised to norm0."""
    o = out.detach().to(torch.float64)
    psi = torch.complex(o[:, 0::2], o[:, 1::2])                       # (B, 2, ny, nx): up, down
    res = []
    for b, p in enumerate(params_list):
        _, _, dx, dy = grid_axes(p)
        nrm = dx * dy * float((psi[b].real ** 2 + psi[b].imag ** 2).sum())
        res.append((psi[b] * math.sqrt(p.norm0 / max(nrm, 1e-300))).cpu().numpy())
    return res


def to_channels(psi_list, device) -> torch.Tensor:
    """List of (2, ny, nx) complex states -> (B, 4, ny, nx) float32 targets."""
    a = np.stack([np.stack([s[0].real, s[0].imag, s[1].real, s[1].imag]) for s in psi_list]).astype(np.float32)
    return torch.from_numpy(a).to(device)


def spectral_mix(a: torch.Tensor, wmat: torch.Tensor, bf16: bool) -> torch.Tensor:
    """Batched complex product (M, b, cin) @ (M, cin, cout).  bf16: on the bfloat16 matrix cores
    with fp32 accumulation, as one real product [re a | im a] (b x 2 cin) @ [[re W, im W],
    [-im W, re W]] (2 cin x 2 cout); else a complex fp32 product."""
    cout = wmat.shape[-1]
    if not bf16:
        return torch.bmm(a.contiguous(), wmat.contiguous())
    ar = torch.cat([a.real, a.imag], dim=-1).to(torch.bfloat16).contiguous()
    wr = torch.cat([torch.cat([wmat.real, wmat.imag], dim=-1),
                    torch.cat([-wmat.imag, wmat.real], dim=-1)], dim=1).to(torch.bfloat16).contiguous()
    if ar.device.type == "cuda" and torch.is_grad_enabled() and (ar.requires_grad or wr.requires_grad):
        # training: the same bf16-rounded operands in an fp32 product, a differentiable stand-in for
        # the fp32-accumulating bf16 product (equal to it up to the order of summation)
        pr = torch.bmm(ar.float(), wr.float())
    elif ar.device.type == "cuda":
        pr = torch.bmm(ar, wr, out_dtype=torch.float32)   # fp32 result of the fp32 accumulation
    else:
        pr = torch.bmm(ar, wr).float()                    # the host's bf16 product rounds its result
    return torch.complex(pr[..., :cout], pr[..., cout:])


class SpectralConv2d(torch.nn.Module):
    """Channel mixing of the lowest modes x modes Fourier modes (k_y of both signs)."""

    def __init__(self, cin: int, cout: int, modes: int):
        super().__init__()
        self.cin, self.cout, self.modes = cin, cout, modes
        scale = 1.0 / (cin * cout)
        # [2 * modes (k_y: 0..m-1 and -m..-1), modes (k_x), cin, cout], complex
        self.weight = torch.nn.Parameter(scale * torch.randn(2 * modes, modes, cin, cout, dtype=torch.cfloat))

    def forward(self, u: torch.Tensor) -> torch.Tensor:
        b, c, h, w = u.shape
        m = self.modes
        uh = torch.fft.rfft2(u.float())                                   # (b, c, h, w//2+1)
        sel = torch.cat([uh[:, :, :m, :m], uh[:, :, h - m:, :m]], dim=2)  # (b, c, 2m, m)
        # per mode: (b, cin) @ (cin, cout) as one batched product over the 2m*m modes
        a = sel.permute(2, 3, 0, 1).reshape(2 * m * m, b, c)
        wmat = self.weight.reshape(2 * m * m, c, self.cout)
        prod = spectral_mix(a, wmat, bf16=(u.device.type == "cuda"))
        prod = prod.reshape(2 * m, m, b, self.cout).permute(2, 3, 0, 1)
        out = torch.zeros(b, self.cout, h, w // 2 + 1, dtype=torch.cfloat, device=u.device)
        out[:, :, :m, :m] = prod[:, :, :m]
        out[:, :, h - m:, :m] = prod[:, :, m:]
        return torch.fft.irfft2(out, s=(h, w))


class Pointwise(torch.nn.Module):
    """A 1x1 convolution (the same linear map at every grid point) computed as one channels-last
    matrix product (B H W, cin) @ (cin, cout) + bias: a GEMM on the matrix cores under bfloat16
    autocast, where the library's 1x1 convolution fell back to a slow direct kernel on this device
    (~1 s of a 256-set prediction).  Parameters as a Conv2d(cin, cout, 1) holds them, (cout, cin,
    1, 1) and (cout,), with its initialisation.  The output is an NCHW view of channels-last memory,
    so the next pointwise layer reads it without a copy."""

    def __init__(self, cin: int, cout: int):
        super().__init__()
        conv = torch.nn.Conv2d(cin, cout, 1)
        self.weight = conv.weight
        self.bias = conv.bias

    def forward(self, u: torch.Tensor) -> torch.Tensor:
        b, c, h, w = u.shape
        x = u.permute(0, 2, 3, 1).reshape(b * h * w, c)
        wt = self.weight.reshape(self.weight.shape[0], c).t().contiguous()
        y = torch.addmm(self.bias, x, wt)
        return y.reshape(b, h, w, -1).permute(0, 3, 1, 2)


class FNO2d(torch.nn.Module):
    def __init__(self, width: int = 32, modes: int = 16, layers: int = 4):
        super().__init__()
        self.width, self.modes, self.layers = width, modes, layers
        self.lift = Pointwise(IN_CHANNELS, width)
        self.spectral = torch.nn.ModuleList([SpectralConv2d(width, width, modes) for _ in range(layers)])
        self.pointwise = torch.nn.ModuleList([Pointwise(width, width) for _ in range(layers)])
        self.proj1 = Pointwise(width, 128)
        self.proj2 = Pointwise(128, 4)

    def forward(self, x: torch.Tensor) -> torch.Tensor:
        dev = x.device.type
        with torch.autocast(device_type=dev, dtype=torch.bfloat16, enabled=(dev == "cuda")):
            u = self.lift(x)
        for k in range(self.layers):
            s = self.spectral[k](u)
            with torch.autocast(device_type=dev, dtype=torch.bfloat16, enabled=(dev == "cuda")):
                u = torch.nn.functional.gelu(s + self.pointwise[k](u).float())
        with torch.autocast(device_type=dev, dtype=torch.bfloat16, enabled=(dev == "cuda")):
            u = self.proj2(torch.nn.functional.gelu(self.proj1(u)))
        return u.float()

    def config(self) -> dict:
        return {"width": self.width, "modes": self.modes, "layers": self.layers}


def infidelity(pred: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
    """Mean over the batch of 1 - |<p, t>|^2 / (<p, p> <t, t>) for (B, 4, ny, nx) real channels
    holding (re, im) of two components."""
    pr, pi = pred[:, 0::2], pred[:, 1::2]
    tr, ti = target[:, 0::2], target[:, 1::2]
    dims = (1, 2, 3)
    re = (pr * tr + pi * ti).sum(dims)
    im = (pr * ti - pi * tr).sum(dims)
    pp = (pr * pr + pi * pi).sum(dims)
    tt = (tr * tr + ti * ti).sum(dims)
    return (1.0 - (re * re + im * im) / (pp * tt)).mean()


def train(model: FNO2d, inputs: torch.Tensor, targets: torch.Tensor, epochs: int = 30, batch: int = 16,
          lr: float = 2e-3, log=print, seed: int = 0) -> list:
    """Adam with a cosine learning-rate schedule on the infidelity; returns the per-epoch mean loss."""
    g = torch.Generator(device="cpu").manual_seed(seed)
    opt = torch.optim.Adam(model.parameters(), lr=lr)
    n = inputs.shape[0]
    steps_total = epochs * ((n + batch - 1) // batch)
    sched = torch.optim.lr_scheduler.OneCycleLR(opt, max_lr=lr, total_steps=steps_total, pct_start=0.1)
    hist = []
    t0 = time.perf_counter()
    for ep in range(epochs):
        perm = torch.randperm(n, generator=g)
        tot = 0.0
        for i in range(0, n, batch):
            idx = perm[i:i + batch].to(inputs.device)
            loss = infidelity(model(inputs[idx]), targets[idx])
            opt.zero_grad(set_to_none=True)
            loss.backward()
            opt.step()
            sched.step()
            tot += float(loss.detach()) * len(idx)
        hist.append(tot / n)
        log(f"  epoch {ep + 1}/{epochs}: infidelity {hist[-1]:.3e} ({time.perf_counter() - t0:.0f} s)")
    return hist


def save(model: FNO2d, path: str, dtype=torch.float16) -> None:
    """Weights as safetensors in `dtype` (complex spectral weights stored as real/imag pairs);
    `load` widens them to fp32."""
    from safetensors.torch import save_file
    tensors = {}
    for k, v in model.state_dict().items():
        v = v.detach().cpu()
        if v.is_complex():
            tensors[k + ".re"] = v.real.to(dtype).contiguous()
            tensors[k + ".im"] = v.imag.to(dtype).contiguous()
        else:
            tensors[k] = v.to(dtype).contiguous()
    meta = {k: str(v) for k, v in model.config().items()}
    save_file(tensors, path, metadata=meta)


def load(path: str, device="cpu") -> FNO2d:
    from safetensors import safe_open
    with safe_open(path, framework="pt") as f:
        meta = f.metadata()
        tensors = {k: f.get_tensor(k) for k in f.keys()}
    model = FNO2d(width=int(meta["width"]), modes=int(meta["modes"]), layers=int(meta["layers"]))
    sd = {}
    for k in model.state_dict():
        if k + ".re" in tensors:
            sd[k] = torch.complex(tensors[k + ".re"].float(), tensors[k + ".im"].float())
        else:
            sd[k] = tensors[k].float()
    model.load_state_dict(sd)
    return model.to(device).eval()


def predict(model: FNO2d, params_list, device) -> list:
    """Initial states (complex128, normalised) for a list of same-grid parameter sets."""
    with torch.no_grad():
        return to_psi(model(encode_on(params_list, device)), params_list)


def predict_device(model: FNO2d, params_list, device) -> torch.Tensor:
    """Initial states for a list of same-grid parameter sets, left on the device in the solver's
    complex64 layout: (B, ny, nx, 4) float32 of (re_up, im_up, re_dn, im_dn), each set normalised to
    its norm0 (the sum in fp64).  For Solver.set_psi_device / Batch.set_psi_device."""
    with torch.no_grad():
        out = model(encode_on(params_list, device)).float()          # (B, 4, ny, nx)
        _, _, dx, dy = grid_axes(params_list[0])
        nrm = (out.double() ** 2).sum(dim=(1, 2, 3)) * (dx * dy)
        norm0 = torch.tensor([p.norm0 for p in params_list], dtype=torch.float64, device=out.device)
        scale = torch.sqrt(norm0 / nrm.clamp_min(1e-300)).float()
        return (out * scale[:, None, None, None]).permute(0, 2, 3, 1).contiguous()
