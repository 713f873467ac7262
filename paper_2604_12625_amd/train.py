"""Training under BC simulation through the C ABI (ndgi_train_step), plus the
torch.autograd.Function wrapper whose backward recomputes the decoded features."""
from __future__ import annotations

import ctypes as C

import numpy as np

from . import ndgi as N


class Trainer:
    """Trainable state in device memory: flat float32 params / grads / Adam m, v with the
    layout [endpoints [H/4][W/4][8][2] | weights [H][W][8] | grid [T][Gh][Gw][8] | mlp]."""

    def __init__(self, ctx: N.Context, init: dict, lr_feat=1e-2, lr_mlp=1e-3, betas=(0.9, 0.999),
                 eps=1e-8, device="cuda"):
        import torch
        d = init["dims"]
        self.ctx = ctx
        self.W, self.H, self.Gw, self.Gh, self.T = d["W"], d["H"], d["Gw"], d["Gh"], d["T"]
        n = N.lib().ndgi_train_param_count(self.W, self.H, self.Gw, self.Gh, self.T)
        self.n_params = n
        if "flat" in init:     # device tensor already in the flat layout
            assert init["flat"].numel() == n and init["flat"].dtype == torch.float32
            self.params = init["flat"].to(device).contiguous()
        else:
            flat = np.concatenate([np.asarray(init[k], dtype=np.float32).ravel()
                                   for k in ("endpoints", "weights", "grid", "mlp")])
            assert flat.size == n, (flat.size, n)
            self.params = torch.from_numpy(flat).to(device)
        self.grads = torch.zeros(n, dtype=torch.float32, device=device)
        self.m = torch.zeros(n, dtype=torch.float32, device=device)
        self.v = torch.zeros(n, dtype=torch.float32, device=device)
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)
        self.state = N.NdgiTrainState(self.W, self.H, self.Gw, self.Gh, self.T, 0,
                                      self.params.data_ptr(), self.grads.data_ptr(),
                                      self.m.data_ptr(), self.v.data_ptr(), 0,
                                      float(lr_feat), float(lr_mlp), float(betas[0]),
                                      float(betas[1]), float(eps), 0.0)

    # segment views ------------------------------------------------------------------
    def split(self, flat):
        W, H, Gw, Gh, T = self.W, self.H, self.Gw, self.Gh, self.T
        n_e = (H // 4) * (W // 4) * 16
        n_w = H * W * 8
        n_g = T * Gh * Gw * 8
        return dict(endpoints=flat[:n_e].view(H // 4, W // 4, 8, 2),
                    weights=flat[n_e:n_e + n_w].view(H, W, 8),
                    grid=flat[n_e + n_w:n_e + n_w + n_g].view(T, Gh, Gw, 8),
                    mlp=flat[n_e + n_w + n_g:])

    @property
    def step_count(self) -> int:
        return int(self.state.step)

    # checkpoint -----------------------------------------------------------------------
    def save(self, path):
        """Checkpoint as an .npz file (arrays only): sizes, parameters, Adam moments, step
        count and optimiser settings.  Trainer.load resumes from it; the gradients are not
        part of the state (every step rebuilds them)."""
        st = self.state
        np.savez(path, **N.to_npz(dict(
            kind="ndgi_train", W=self.W, H=self.H, Gw=self.Gw, Gh=self.Gh, T=self.T,
            params=self.params.cpu().numpy(), m=self.m.cpu().numpy(), v=self.v.cpu().numpy(), step=int(st.step),
            lr_feat=st.lr_feat, lr_mlp=st.lr_mlp, beta1=st.beta1, beta2=st.beta2, eps=st.eps)))

    @classmethod
    def load(cls, ctx: N.Context, path, device="cuda") -> "Trainer":
        import torch
        z = N.from_npz(path)
        if z.get("kind") != "ndgi_train":
            raise ValueError(f"{path}: not a Trainer checkpoint")
        dims = {k: int(z[k]) for k in ("W", "H", "Gw", "Gh", "T")}
        tr = cls(ctx, dict(dims=dims, flat=torch.from_numpy(z["params"])), lr_feat=z["lr_feat"], lr_mlp=z["lr_mlp"],
                 betas=(z["beta1"], z["beta2"]), eps=z["eps"], device=device)
        tr.m.copy_(torch.from_numpy(z["m"]))
        tr.v.copy_(torch.from_numpy(z["v"]))
        tr.state.step = int(z["step"])
        return tr

    def _run(self, mode, samples=None, target=None, pred=None, grad_pred=None, stream=None):
        b = N.NdgiBatch(N._ptr(samples), 0 if samples is None else samples.shape[0],
                        N._ptr(target), N._ptr(pred), N._ptr(grad_pred))
        N.check(N.lib().ndgi_train_step(self.ctx.h, C.byref(self.state), C.byref(b), mode,
                                        self.loss.data_ptr(), N._stream(stream)), "ndgi_train_step")

    def forward(self, samples, pred=None):
        import torch
        if pred is None:
            pred = torch.empty((samples.shape[0], 3), dtype=torch.float32, device=samples.device)
        self._run(N.TRAIN_FORWARD, samples, pred=pred)
        return pred

    def backward(self, samples, grad_pred):
        self._run(N.TRAIN_BACKWARD, samples, grad_pred=grad_pred)

    def loss_grad(self, samples, target, pred=None):
        self._run(N.TRAIN_LOSS_GRAD, samples, target=target, pred=pred)
        return self.loss

    def step(self, samples, target):
        """Forward, FP64 L2 loss, backward and Adam in one stream order; returns the loss tensor."""
        self._run(N.TRAIN_FUSED, samples, target=target)
        return self.loss

    def adam(self):
        self._run(N.TRAIN_ADAM)

    def zero_grad(self):
        self._run(N.TRAIN_ZERO_GRAD)

    def export(self, grid_dtype=N.DTYPE_F16, mlp_dtype=N.DTYPE_F16) -> N.DeviceModel:
        import torch
        dev = self.params.device
        bc4 = torch.empty((self.H // 4, self.W // 4, 8, 8), dtype=torch.uint8, device=dev)
        tdt = {N.DTYPE_F16: torch.float16, N.DTYPE_F32: torch.float32}
        grid = torch.empty((self.T, self.Gh, self.Gw, 8), dtype=tdt[grid_dtype], device=dev)
        mlp = torch.empty(N.MLP_SIZE, dtype=tdt[mlp_dtype], device=dev)
        N.check(N.lib().ndgi_export(self.ctx.h, C.byref(self.state), bc4.data_ptr(), grid.data_ptr(),
                                    grid_dtype, mlp.data_ptr(), mlp_dtype, N._stream(None)), "ndgi_export")
        return N.DeviceModel(self.W, self.H, self.Gw, self.Gh, self.T, bc4, grid, mlp)


def _autograd_function():
    import torch

    class NdgiFunction(torch.autograd.Function):
        """pred = H_Theta(samples) under BC simulation.  Forward saves only the samples; the
        backward recomputes the decoded features inside the kernel and returns the gradient
        of the flat parameter tensor."""

        @staticmethod
        def forward(ctx, params, samples, trainer):
            assert params.data_ptr() == trainer.params.data_ptr()
            ctx.save_for_backward(samples)
            ctx.trainer = trainer
            return trainer.forward(samples)

        @staticmethod
        def backward(ctx, grad_pred):
            (samples,) = ctx.saved_tensors
            tr = ctx.trainer
            tr.zero_grad()
            tr.backward(samples, grad_pred.contiguous().float())
            return tr.grads.clone(), None, None

    return NdgiFunction


_FN = None


def ndgi_apply(trainer: Trainer, samples):
    """Differentiable prediction at packed samples (see NdgiFunction)."""
    global _FN
    if _FN is None:
        _FN = _autograd_function()
    return _FN.apply(trainer.params, samples, trainer)


HYB_KEYS = ("fuv_ep", "fuv_w", "fuvt_ep", "fuvt_w", "fut", "fvt", "mlp")


class HybridTrainer:
    """Trainable hybrid-layout state of one or more models of equal sizes in device memory
    (ndgi_hybrid_train_step): flat float32 params / grads / Adam m, v holding every model's
    feature block [F_uv endpoints | F_uv weights | F_uvt endpoints | F_uvt weights | F_ut |
    F_vt], model after model, then every model's decoder."""

    def __init__(self, ctx: N.Context, init, lr_feat=1e-3, lr_mlp=1e-3, betas=(0.9, 0.999), eps=1e-8,
                 seed=0, per_model=0, device="cuda"):
        import torch
        if isinstance(init, dict) and "flat" in init:   # a checkpoint's flat state of n_models models
            d, M = init["dims"], int(init["n_models"])
        else:
            inits = init if isinstance(init, (list, tuple)) else [init]
            d, M = inits[0]["dims"], len(inits)
        self.ctx, self.d, self.M = ctx, dict(d), M
        dims = [d[k] for k in ("W", "H", "Gu", "Gv", "S", "U", "V", "Tt", "hidden")]
        self.codec = int(d.get("codec", N.CODEC_BC4))
        n = int(N.lib().ndgi_hybrid_train_param_count(*dims, self.codec))
        self.n_params = n * self.M
        self.n_feat = n - N.hybrid_mlp_size(d["hidden"])
        if isinstance(init, dict) and "flat" in init:
            flat = np.asarray(init["flat"], dtype=np.float32)
        else:
            feats = [np.concatenate([np.asarray(m[k], dtype=np.float32).ravel() for k in HYB_KEYS[:-1]])
                     for m in inits]
            mlps = [np.asarray(m["mlp"], dtype=np.float32).ravel() for m in inits]
            assert feats[0].size == self.n_feat, (feats[0].size, self.n_feat)
            flat = np.concatenate(feats + mlps)
        assert flat.size == self.n_params, (flat.size, self.n_params)
        self.params = torch.from_numpy(flat).to(device)
        self.grads = torch.zeros_like(self.params)
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.loss = torch.zeros(1, dtype=torch.float64, device=device)
        keys = np.asarray(d.get("keys", []), dtype=np.float32)
        self.keys = torch.from_numpy(keys).to(device) if keys.size else None
        self.state = N.NdgiHybridTrainState(*dims, int(d["frames"]), self.M, int(per_model), self.codec, 0,
                                            N._ptr(self.keys),
                                            self.params.data_ptr(), self.grads.data_ptr(), self.m.data_ptr(),
                                            self.v.data_ptr(), 0, float(lr_feat), float(lr_mlp), float(betas[0]),
                                            float(betas[1]), float(eps), int(seed))

    def split(self, flat, model=0) -> dict:
        """Views of one model's arrays in a flat [params | grads | m | v]-shaped tensor."""
        d = self.d
        cw = () if self.codec == N.CODEC_BC7 else (4,)
        shapes = dict(fuv_ep=(d["H"] // 4, d["W"] // 4, 4, 2), fuv_w=(d["H"], d["W"]) + cw,
                      fuvt_ep=(d["S"], d["Gv"] // 4, d["Gu"] // 4, 4, 2), fuvt_w=(d["S"], d["Gv"], d["Gu"]) + cw,
                      fut=(d["Tt"], d["U"], 2), fvt=(d["Tt"], d["V"], 2))
        out, o = {}, model * self.n_feat
        for k in HYB_KEYS[:-1]:
            cnt = int(np.prod(shapes[k]))
            out[k] = flat[o:o + cnt].view(*shapes[k])
            o += cnt
        ms = N.hybrid_mlp_size(d["hidden"])
        o = self.M * self.n_feat + model * ms
        out["mlp"] = flat[o:o + ms]
        return out

    def _run(self, mode, flags, samples=None, target=None, pred=None, stream=None):
        b = N.NdgiHybridBatch(N._ptr(samples), 0 if samples is None else samples.shape[0], N._ptr(target),
                              N._ptr(pred))
        N.check(N.lib().ndgi_hybrid_train_step(self.ctx.h, C.byref(self.state), C.byref(b), mode, flags,
                                               self.loss.data_ptr(), N._stream(stream)), "ndgi_hybrid_train_step")

    def save(self, path):
        """Checkpoint as an .npz file (arrays only): sizes and key times, parameters, Adam
        moments, step count, optimiser settings and the noise seed (the noise stream is a
        function of seed and step, so a resumed run draws what the uninterrupted one would).
        HybridTrainer.load resumes from it."""
        st = self.state
        d = {k: v for k, v in self.d.items() if k != "keys"}
        keys = np.asarray(self.d.get("keys", []), dtype=np.float32)
        np.savez(path, **N.to_npz(dict(
            kind="ndgi_hybrid_train", n_models=self.M, per_model=int(st.per_model), seed=int(st.seed),
            keys=keys, params=self.params.cpu().numpy(), m=self.m.cpu().numpy(), v=self.v.cpu().numpy(),
            step=int(st.step), lr_feat=st.lr_feat, lr_mlp=st.lr_mlp, beta1=st.beta1, beta2=st.beta2, eps=st.eps,
            **{"dim_" + k: v for k, v in d.items()})))

    @classmethod
    def load(cls, ctx: N.Context, path, device="cuda") -> "HybridTrainer":
        import torch
        z = N.from_npz(path)
        if z.get("kind") != "ndgi_hybrid_train":
            raise ValueError(f"{path}: not a HybridTrainer checkpoint")
        dims = {k[4:]: int(v) for k, v in z.items() if k.startswith("dim_")}
        dims["keys"] = np.asarray(z["keys"], dtype=np.float32).reshape(-1)
        tr = cls(ctx, dict(dims=dims, n_models=z["n_models"], flat=z["params"]), lr_feat=z["lr_feat"],
                 lr_mlp=z["lr_mlp"], betas=(z["beta1"], z["beta2"]), eps=z["eps"], seed=z["seed"],
                 per_model=z["per_model"], device=device)
        tr.m.copy_(torch.from_numpy(z["m"]))
        tr.v.copy_(torch.from_numpy(z["v"]))
        tr.state.step = int(z["step"])
        return tr

    def set_lr(self, lr_feat=None, lr_mlp=None):
        if lr_feat is not None:
            self.state.lr_feat = float(lr_feat)
        if lr_mlp is not None:
            self.state.lr_mlp = float(lr_mlp)

    def forward(self, samples, flags, pred=None):
        import torch
        if pred is None:
            pred = torch.empty((samples.shape[0], 3), dtype=torch.float32, device=samples.device)
        self._run(N.TRAIN_FORWARD, flags, samples, pred=pred)
        return pred

    def loss_grad(self, samples, target, flags):
        self._run(N.TRAIN_LOSS_GRAD, flags, samples, target=target)
        return self.loss

    def step(self, samples, target, flags):
        self._run(N.TRAIN_FUSED, flags, samples, target=target)
        return self.loss

    def zero_grad(self):
        self._run(N.TRAIN_ZERO_GRAD, 0)

    def export(self, mlp_dtype=N.DTYPE_F16, model=0) -> N.HybridModel:
        import torch
        d, dev = self.d, self.params.device
        blk = (16,) if self.codec == N.CODEC_BC7 else (4, 8)
        fuv = torch.empty((d["H"] // 4, d["W"] // 4) + blk, dtype=torch.uint8, device=dev)
        fuvt = torch.empty((d["S"], d["Gv"] // 4, d["Gu"] // 4) + blk, dtype=torch.uint8, device=dev)
        fut = torch.empty((d["Tt"], d["U"], 2), dtype=torch.uint8, device=dev)
        fvt = torch.empty((d["Tt"], d["V"], 2), dtype=torch.uint8, device=dev)
        mlp = torch.empty(N.hybrid_mlp_size(d["hidden"]), dtype=torch.float16 if mlp_dtype == N.DTYPE_F16
                          else torch.float32, device=dev)
        N.check(N.lib().ndgi_hybrid_export(self.ctx.h, C.byref(self.state), model, fuv.data_ptr(), fuvt.data_ptr(),
                                           fut.data_ptr(), fvt.data_ptr(), mlp.data_ptr(), mlp_dtype,
                                           N._stream(None)), "ndgi_hybrid_export")
        keys = self.keys if self.keys is not None else torch.zeros(0, dtype=torch.float32, device=dev)
        return N.HybridModel(d["W"], d["H"], d["Gu"], d["Gv"], d["S"], d["U"], d["V"], d["Tt"], d["hidden"],
                             fuv, fuvt, fut, fvt, keys, mlp, self.codec)

    def encode(self, flags, codec, mlp_dtype=N.DTYPE_F16, model=0, maps=True) -> N.HybridModel:
        """The paper's export (ndgi_hybrid_encode): maps reconstructed as a step with `flags`
        reads them, quantised to 8 bits and block-encoded in `codec`; planes to 8 bits; the
        decoder in mlp_dtype.  maps=False skips the map encoding (the maps are then left
        uninitialised: for taking only a fine-tuned decoder and planes)."""
        import torch
        d, dev = self.d, self.params.device
        blk = (16,) if codec == N.CODEC_BC7 else (4, 8)
        fuv = torch.empty((d["H"] // 4, d["W"] // 4) + blk, dtype=torch.uint8, device=dev)
        fuvt = torch.empty((d["S"], d["Gv"] // 4, d["Gu"] // 4) + blk, dtype=torch.uint8, device=dev)
        fut = torch.empty((d["Tt"], d["U"], 2), dtype=torch.uint8, device=dev)
        fvt = torch.empty((d["Tt"], d["V"], 2), dtype=torch.uint8, device=dev)
        mlp = torch.empty(N.hybrid_mlp_size(d["hidden"]), dtype=torch.float16 if mlp_dtype == N.DTYPE_F16
                          else torch.float32, device=dev)
        N.check(N.lib().ndgi_hybrid_encode(self.ctx.h, C.byref(self.state), model, flags, codec,
                                           fuv.data_ptr() if maps else None, fuvt.data_ptr() if maps else None,
                                           fut.data_ptr(), fvt.data_ptr(), mlp.data_ptr(), mlp_dtype,
                                           N._stream(None)), "ndgi_hybrid_encode")
        keys = self.keys if self.keys is not None else torch.zeros(0, dtype=torch.float32, device=dev)
        return N.HybridModel(d["W"], d["H"], d["Gu"], d["Gv"], d["S"], d["U"], d["V"], d["Tt"], d["hidden"],
                             fuv, fuvt, fut, fvt, keys, mlp, codec)


def hybrid_import_models(ctx: N.Context, models, frames: int, lr_mlp=1e-3, seed=0, per_model=0, keys=None,
                         device="cuda") -> "HybridTrainer":
    """A directly parameterised state (BC4 layout, flag DIRECT) holding block-compressed
    models (ndgi_hybrid_import): for the final stage that fine-tunes the decoders on frozen
    features exactly as a decode of the models reads them (lr_feat = 0)."""
    m0 = models[0]
    d = m0.desc
    dims = dict(W=d.W, H=d.H, Gu=d.Gu, Gv=d.Gv, S=d.S, U=d.U, V=d.V, Tt=d.Tt, hidden=d.hidden, frames=int(frames),
                keys=np.zeros(0, np.float32) if keys is None else np.asarray(keys, np.float32), codec=N.CODEC_BC4)
    z = lambda *sh: np.zeros(sh, np.float32)
    init = dict(dims=dims, fuv_ep=z(d.H // 4, d.W // 4, 4, 2), fuv_w=z(d.H, d.W, 4),
                fuvt_ep=z(d.S, d.Gv // 4, d.Gu // 4, 4, 2), fuvt_w=z(d.S, d.Gv, d.Gu, 4), fut=z(d.Tt, d.U, 2),
                fvt=z(d.Tt, d.V, 2), mlp=z(N.hybrid_mlp_size(d.hidden)))
    tr = HybridTrainer(ctx, [init] * len(models), lr_feat=0.0, lr_mlp=lr_mlp, seed=seed, per_model=per_model,
                       device=device)
    for i, m in enumerate(models):
        N.check(N.lib().ndgi_hybrid_import(ctx.h, C.byref(m.desc), C.byref(tr.state), i, N._stream(None)),
                "ndgi_hybrid_import")
    return tr


def hybrid_normalize_target(ctx: N.Context, target_bits, gamma=2.2):
    """(normalised float target [n][H][W][3], means [n][3] float64) of an FP16 target."""
    import torch
    n, H, W = target_bits.shape[0], target_bits.shape[1], target_bits.shape[2]
    out = torch.empty((n, H, W, 3), dtype=torch.float32, device=target_bits.device)
    means = torch.empty((n, 3), dtype=torch.float64, device=target_bits.device)
    N.check(N.lib().ndgi_hybrid_normalize_target(ctx.h, target_bits.data_ptr(), n, W, H, float(gamma),
                                                 out.data_ptr(), means.data_ptr(), N._stream(None)),
            "ndgi_hybrid_normalize_target")
    return out, means


def hybrid_restore(ctx: N.Context, pred, mean3, gamma=2.2, out=None):
    import torch
    texels = pred.shape[0]
    if out is None:
        out = torch.empty((texels, 3), dtype=torch.float32, device=pred.device)
    pdt = N.DTYPE_F16 if pred.dtype == torch.float16 else N.DTYPE_F32
    N.check(N.lib().ndgi_hybrid_restore(ctx.h, pred.data_ptr(), pdt, texels, mean3.data_ptr(), float(gamma),
                                        out.data_ptr(), N._stream(None)), "ndgi_hybrid_restore")
    return out
