"""torch.autograd binding of the differentiable form.

`simulate_dense(sim, particles, event_offsets, seed, elayer, weights)` returns
the dense cell energies [n_events, n_cells] of a batch simulated with the
per-(particle, layer) energies `elayer` in place of the sampled Dirichlet
split.  Its backward is `fcs_backward`: hit counts and every hit's bin and
cell are held fixed (they are recomputed from their Philox counters), so

* dL/d elayer[t] = (1/n_t) * sum over the task's in-acceptance hits of g[cell];
* dL/d weights   = the likelihood-ratio gradient of the histogram weights
  with the samples drawn at the loaded weights.

`weights` must be the tensor whose values were loaded with
`load_parametrization` (f32 [n_histograms * 256]); it carries the gradient and
its values are not read by the forward pass.  Both passes run in the HIP
library; this module only marshals arguments.

With `async_launch=True` both passes return once their work is enqueued on
the library's stream (torch's current stream waits for their outputs), so
consecutive training steps need no host round trip; errors are then raised
by `sim.synchronize()`.
"""
from __future__ import annotations

import torch


class _SimulateDense(torch.autograd.Function):
    @staticmethod
    def forward(ctx, elayer, weights, sim, particles, event_offsets, seed, kw):
        out = sim.simulate_events(particles, event_offsets, seed, outputs=("dense",),
                                  elayer_override=elayer.detach(), **kw)
        ctx.sim, ctx.particles, ctx.event_offsets, ctx.seed, ctx.kw = (
            sim, particles, event_offsets, seed, kw)
        ctx.save_for_backward(elayer)
        return out["cells"]

    @staticmethod
    def backward(ctx, grad_cells):
        (elayer,) = ctx.saved_tensors
        need_e, need_w = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_e or need_w):
            return (None,) * 7
        bkw = {k: v for k, v in ctx.kw.items()
               if k in ("event_index_base", "hit_energy_scale", "nhit_cap", "min_layer_energy",
                        "async_launch", "chunk_hits", "big_task_hits", "tile_hits", "wg_per_cu",
                        "hit_energy_fluct")}
        # the forward's work queue is reused when no other call has rebuilt it
        # since (the library checks inputs, options and tuning)
        ge, gw = ctx.sim.backward(ctx.particles, ctx.event_offsets, ctx.seed,
                                  grad_cells.reshape(-1), elayer_override=elayer.detach(),
                                  need_elayer=need_e, need_weights=need_w,
                                  reuse_forward_queue=True, **bkw)
        return (ge, gw) + (None,) * 5


def sampled_elayer(sim, particles, event_offsets, seed, **kw):
    """The FP32 per-(particle, layer) energies of the Dirichlet split the
    forward simulation draws (device tensor [N * n_layers])."""
    return sim.simulate_events(particles, event_offsets, seed, outputs=("elayer",),
                               **kw)["elayer"]


def simulate_dense(sim, particles, event_offsets, seed, elayer, weights=None, **kw):
    """Dense cell energies [n_events, n_cells] (device f32) as a differentiable
    function of `elayer` (and of `weights`, when given).  `particles` and
    `event_offsets` must be device tensors; `kw` takes event_index_base,
    hit_energy_scale, nhit_cap, min_layer_energy, async_launch,
    hit_energy_fluct and the launch tuning."""
    if not (torch.is_tensor(elayer) and elayer.is_cuda and elayer.dtype == torch.float32):
        raise TypeError("elayer must be a float32 CUDA tensor")
    if weights is None:
        weights = torch.zeros(0, device=elayer.device)
    elif weights.numel() != sim.n_hist * 256:
        raise ValueError(f"weights must hold {sim.n_hist * 256} values")
    return _SimulateDense.apply(elayer, weights, sim, particles, event_offsets, seed, kw)
