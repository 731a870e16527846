"""Optimiser state of a half-Gaussian scene on the GPU: raw parameters, Adam
moments, activated copies and densification statistics, driven through the
library's training entry points (Adam with the half-Gaussian schedule,
densification statistics, clone / split / prune, opacity reset).

Raw planes follow the hgs_params layout with log-scales and opacity logits.
The activated copies hold only the five planes whose activation is not the
identity (scales, opac1, opac2); the other planes of the rasterizer's
parameters point straight into the raw tensor.
"""
from __future__ import annotations

import torch

from . import binding as B
from .raster import Frame, _stream, sh_planes


def _planes(t: torch.Tensor, stride: int) -> B.hgs_param_grads:
    return B.grads_struct(t, stride)


class TrainState:
    """Raw SoA [planes, stride] float32 on the GPU plus Adam moments and the
    densification statistics of its n kernels."""

    def __init__(self, raw: torch.Tensor, n: int, sh_degree: int, extent: float, normal_lr: float = 0.003):
        if raw.dtype != torch.float32 or not raw.is_cuda or raw.dim() != 2:
            raise ValueError("raw must be a float32 [planes, stride] CUDA tensor")
        if raw.shape[0] != 15 + sh_planes(sh_degree) or raw.shape[1] < n:
            raise ValueError("raw has the wrong shape")
        self.raw = raw.contiguous()
        self.n, self.sh_degree, self.extent, self.normal_lr = n, sh_degree, float(extent), float(normal_lr)
        self.stride = self.raw.shape[1]
        self.m = torch.zeros_like(self.raw)
        self.v = torch.zeros_like(self.raw)
        self.act5 = torch.empty((5, self.stride), dtype=torch.float32, device=raw.device)
        self.step_count = 0
        self.clear_stats()
        B.hgs_activate(self.n, self.stride, sh_degree, self._raw(), self._act(), _stream())

    # -- pointer sets -----------------------------------------------------
    def _raw(self) -> B.hgs_param_grads:
        return _planes(self.raw, self.stride)

    def _act(self) -> B.hgs_param_grads:
        g = _planes(self.raw, self.stride)
        base, f = self.act5.data_ptr(), 4 * self.stride
        g.scales, g.opac1, g.opac2 = base, base + 3 * f, base + 4 * f
        return g

    def params(self) -> B.hgs_params:
        """The rasterizer's (activated) parameters."""
        a = self._act()
        p = B.hgs_params()
        p.means, p.scales, p.quats, p.normals = a.means, a.scales, a.quats, a.normals
        p.opac1, p.opac2, p.sh = a.opac1, a.opac2, a.sh
        p.n, p.stride, p.sh_degree = self.n, self.stride, self.sh_degree
        return p

    def activated_soa(self) -> torch.Tensor:
        """A dense activated SoA copy [planes, n] (for inspection)."""
        out = self.raw[:, :self.n].clone()
        out[3:6] = self.act5[0:3, :self.n]
        out[13:15] = self.act5[3:5, :self.n]
        return out

    # -- steps ------------------------------------------------------------
    def adam_step(self, grads: torch.Tensor):
        """One Adam step with the gradient SoA (activated space, as the
        backward pass writes it, same stride)."""
        self.step_count += 1
        cfg = B.hgs_adam_schedule(self.step_count, self.extent, self.normal_lr)
        B.hgs_adam_step(cfg, self.n, self.stride, self.sh_degree, self._raw(), _planes(grads, self.stride),
                        _planes(self.m, self.stride), _planes(self.v, self.stride), self._act(), _stream())

    def clear_stats(self):
        dev = self.raw.device
        self.grad_accum = torch.zeros(self.stride, dtype=torch.float32, device=dev)
        self.grad_count = torch.zeros(self.stride, dtype=torch.int32, device=dev)
        self.max_radii = torch.zeros(self.stride, dtype=torch.float32, device=dev)

    def stats(self):
        """(grad_accum, grad_count, max_radii) for backward_pass(stats=...)."""
        return self.grad_accum, self.grad_count, self.max_radii

    def add_stats(self, fr: Frame, record_grads: torch.Tensor):
        """Accumulate the densification statistics of one backward pass
        (record_grads as hgs_raster_bwd left it)."""
        B.hgs_densify_stats(fr.records, record_grads, fr.cams, fr.opts, self.n, self.grad_accum, self.grad_count,
                            self.max_radii, _stream())

    def densify(self, cfg: B.hgs_densify_config | None = None, generator: torch.Generator | None = None,
                samples: torch.Tensor | None = None) -> int:
        """Clone / split / prune; returns the new kernel count (reads it back:
        one synchronisation).  Statistics are cleared afterwards."""
        cfg = B.hgs_densify_default(self.extent) if cfg is None else cfg
        dev = self.raw.device
        if samples is None:
            samples = torch.randn((2, 3, max(self.n, 1)), generator=generator, device=dev, dtype=torch.float32)
        cap = max(2 * self.n, 1)
        stride_out = (cap + 3) // 4 * 4
        raw_o = torch.empty((self.raw.shape[0], stride_out), dtype=torch.float32, device=dev)
        m_o, v_o = torch.empty_like(raw_o), torch.empty_like(raw_o)
        n_out = torch.zeros(1, dtype=torch.int64, device=dev)
        overflow = torch.zeros(1, dtype=torch.int32, device=dev)
        ws = torch.empty(max(B.hgs_densify_workspace_bytes(self.n), 1), dtype=torch.uint8, device=dev)
        B.hgs_densify(cfg, self.n, self.stride, self.sh_degree, self._raw(), _planes(self.m, self.stride),
                      _planes(self.v, self.stride), self.grad_accum, self.grad_count, self.max_radii, samples, cap,
                      stride_out, _planes(raw_o, stride_out), _planes(m_o, stride_out), _planes(v_o, stride_out),
                      n_out, overflow, ws, _stream())
        n_new = int(n_out.item())
        if int(overflow.item()) != 0:
            raise RuntimeError("densify: output capacity exceeded")
        self.raw, self.m, self.v, self.n, self.stride = raw_o, m_o, v_o, n_new, stride_out
        self.act5 = torch.empty((5, self.stride), dtype=torch.float32, device=dev)
        B.hgs_activate(self.n, self.stride, self.sh_degree, self._raw(), self._act(), _stream())
        self.clear_stats()
        return n_new

    def reset_opacity(self, value: float = 0.02):
        B.hgs_reset_opacity(value, self.n, self._raw(), _planes(self.m, self.stride), _planes(self.v, self.stride),
                            self._act(), _stream())
