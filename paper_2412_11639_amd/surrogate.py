"""Learned surrogate: binding of the spk_sur_* entry points and its trainer.

A small CNN (four 3x3 convolutions, 33 -> 32 -> 32 -> 32 -> 1, ReLU between,
output added to the estimate) maps a 32-frame spike window plus the plain
short-window estimate to the intensity the plain method only reaches over a
long stable window.  Every
step (window extraction, the estimate, convolutions, gradients, loss, Adam,
fallback) runs in the library's kernels; this module marshals arguments,
owns the parameter and workspace tensors and drives the training loop.
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import _lib
from . import _stream_handle, _check_stream_tensor, reconstruct, FSR

NPARAMS = 28321
MAX_SAMPLES = 64
SHAPES = [("W1", (32, 9, 33)), ("b1", (32,)), ("W2", (32, 9, 32)), ("b2", (32,)),
          ("W3", (32, 9, 32)), ("b3", (32,)), ("W4", (1, 9, 32)), ("b4", (1,))]


class SurSample(ctypes.Structure):
    """Mirror of ``spk_sur_sample`` in include/spk.h."""
    _fields_ = [("stream", ctypes.c_void_p), ("H", ctypes.c_int32), ("W", ctypes.c_int32),
                ("T", ctypes.c_int32), ("oy", ctypes.c_int32), ("ox", ctypes.c_int32),
                ("t", ctypes.c_int32), ("target", ctypes.c_void_p)]


_P = ctypes.c_void_p
_i32 = ctypes.c_int32
_lib.EXTRA_DECLS.update({
    "spk_sur_input": [ctypes.POINTER(SurSample), _i32, _i32, _i32, ctypes.c_float, _P, _P, _P,
                      _P, _P],
    "spk_sur_stream_step": [_P, _i32, _i32, ctypes.c_float, _P, _P, _P, _P],
    "spk_sur_forward": [_P, _P, _P, _i32, _i32, _i32, _P, _P, _P],
    "spk_sur_infer": [_P, _P, _P, _i32, _i32, _i32, _P, _P, _P],
    "spk_sur_infer_prepacked": [_P, _P, _P, _i32, _i32, _i32, _P, _P, _P],
    "spk_sur_backward": [_P, _P, _P, _i32, _i32, _i32, _P, _P, _P, _P, _P, _P],
    "spk_sur_adam": [_P, _P, _P, _P, _i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                     ctypes.c_float, _P],
    "spk_sur_mux": [_P, _P, _P, ctypes.c_int64, _P, _P],
    "spk_sur_train_create": [ctypes.POINTER(_P), _P, _P, _P, ctypes.POINTER(SurSample), _P, _i32,
                             _i32, _i32, _i32, ctypes.c_float, ctypes.c_float, ctypes.c_float,
                             ctypes.c_float, _i32, _P],
    "spk_sur_train_run": [_P, _i32, _P],
    "spk_sur_train_destroy": [_P],
})


def _lib_sur():
    lib = _lib.load()
    if not getattr(lib, "_sur_declared", False):
        lib.spk_sur_workspace_bytes.restype = ctypes.c_size_t
        lib.spk_sur_workspace_bytes.argtypes = [_i32, _i32, _i32]
        lib.spk_sur_workspace_layout.restype = ctypes.c_int
        lib.spk_sur_workspace_layout.argtypes = [_i32, _i32, _i32,
                                                 ctypes.POINTER(ctypes.c_size_t)]
        for name, argtypes in _lib.EXTRA_DECLS.items():
            if name.startswith("spk_sur_"):
                f = getattr(lib, name)
                f.restype = ctypes.c_int
                f.argtypes = argtypes
        lib._sur_declared = True
    return lib


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal hidden weights, zero biases, zero output layer: the network
    starts as the identity on the plain estimate (y = est)."""
    rng = np.random.default_rng(seed)
    parts = []
    for name, shape in SHAPES:
        if name.startswith("W") and name != "W4":
            fan_in = shape[1] * shape[2]
            parts.append(rng.normal(0.0, math.sqrt(2.0 / fan_in), size=shape).reshape(-1))
        else:
            parts.append(np.zeros(int(np.prod(shape))))
    p = np.concatenate(parts)
    assert p.shape == (NPARAMS,)
    return p


class Surrogate:
    """Parameters (float32, device), Adam moments and per-shape workspaces."""

    def __init__(self, params=None, device="cuda", seed: int = 0):
        if params is None:
            params = init_params(seed)
        self.params = torch.as_tensor(np.asarray(params, dtype=np.float32)).to(device).contiguous()
        assert self.params.numel() == NPARAMS
        self.m = torch.zeros_like(self.params)
        self.v = torch.zeros_like(self.params)
        self.grad = torch.zeros_like(self.params)
        self.step_count = 0
        self.device = device
        self._ws = {}

    def workspace(self, B, Hc, Wc):
        key = (B, Hc, Wc)
        if key not in self._ws:
            n = int(_lib_sur().spk_sur_workspace_bytes(B, Hc, Wc))
            self._ws[key] = torch.empty(n, dtype=torch.uint8, device=self.device)
        return self._ws[key]

    def stored(self, B, Hc, Wc):
        """The values the last forward and backward of this batch shape left
        in its workspace (spk_sur_workspace_layout): dict of float32 device
        tensors a1, a2, a3, g1, g2 ([B, Hc, Wc, 32]) and dy ([B, Hc, Wc])."""
        offs = (ctypes.c_size_t * 7)()
        _lib.check("spk_sur_workspace_layout",
                   _lib_sur().spk_sur_workspace_layout(B, Hc, Wc, offs))
        ws = self.workspace(B, Hc, Wc)
        P = B * Hc * Wc
        out = {}
        for k, name in enumerate(("packed", "a1", "a2", "a3", "g1", "g2", "dy")):
            if name == "packed":
                continue
            if name == "dy":
                t = ws[offs[k]:offs[k] + 4 * P].view(torch.float32).reshape(B, Hc, Wc)
            else:
                t = ws[offs[k]:offs[k] + 2 * P * 32].view(torch.bfloat16).reshape(B, Hc, Wc, 32)
            out[name] = t.to(torch.float32)
        return out

    # -- inputs ---------------------------------------------------------------
    @staticmethod
    def input(samples, Hc, Wc, theta=1.0, with_target=False, stream=None):
        """samples: list of dicts (stream tensor, H, W, T, oy, ox, t[, target
        tensor]).  Returns (win uint32 as int32, est float32, stable uint8
        [, target float32]), each [B, Hc, Wc]."""
        B = len(samples)
        assert 0 < B <= MAX_SAMPLES
        dev = samples[0]["stream"].device
        arr = (SurSample * B)()
        for i, s in enumerate(samples):
            _check_stream_tensor(s["stream"], s["H"], s["W"], s["T"])
            tgt = s.get("target")
            arr[i] = SurSample(s["stream"].data_ptr(), s["H"], s["W"], s["T"], s["oy"], s["ox"],
                               s["t"], tgt.data_ptr() if tgt is not None else None)
        win = torch.empty((B, Hc, Wc), dtype=torch.int32, device=dev)
        est = torch.empty((B, Hc, Wc), dtype=torch.float32, device=dev)
        st = torch.empty((B, Hc, Wc), dtype=torch.uint8, device=dev)
        tg = torch.empty((B, Hc, Wc), dtype=torch.float32, device=dev) if with_target else None
        rc = _lib_sur().spk_sur_input(arr, B, Hc, Wc, float(theta), win.data_ptr(),
                                      est.data_ptr(), st.data_ptr(),
                                      tg.data_ptr() if tg is not None else None,
                                      _stream_handle(stream))
        _lib.check("spk_sur_input", rc)
        return (win, est, st, tg) if with_target else (win, est, st)

    @staticmethod
    def stream_step(frame, H, W, theta, win, est, stable, stream=None):
        """Advance full-frame windows by one packed frame (device uint8)."""
        rc = _lib_sur().spk_sur_stream_step(frame.data_ptr(), H, W, float(theta), win.data_ptr(),
                                            est.data_ptr(), stable.data_ptr(),
                                            _stream_handle(stream))
        _lib.check("spk_sur_stream_step", rc)

    # -- network --------------------------------------------------------------
    def forward(self, win, est, out=None, stream=None):
        B, Hc, Wc = win.shape
        y = out if out is not None else torch.empty((B, Hc, Wc), dtype=torch.float32,
                                                    device=win.device)
        rc = _lib_sur().spk_sur_forward(self.params.data_ptr(), win.data_ptr(), est.data_ptr(),
                                        B, Hc, Wc, y.data_ptr(),
                                        self.workspace(B, Hc, Wc).data_ptr(),
                                        _stream_handle(stream))
        _lib.check("spk_sur_forward", rc)
        return y

    def infer(self, win, est, out=None, stream=None, prepacked=False):
        """Forward for inference only (no activations kept for backward).
        prepacked: reuse the packed weights the last infer or forward of this
        batch shape left in its workspace (spk_sur_infer_prepacked); the
        parameters must not have changed since."""
        B, Hc, Wc = win.shape
        y = out if out is not None else torch.empty((B, Hc, Wc), dtype=torch.float32,
                                                    device=win.device)
        name = "spk_sur_infer_prepacked" if prepacked else "spk_sur_infer"
        rc = getattr(_lib_sur(), name)(self.params.data_ptr(), win.data_ptr(), est.data_ptr(),
                                       B, Hc, Wc, y.data_ptr(),
                                       self.workspace(B, Hc, Wc).data_ptr(),
                                       _stream_handle(stream))
        _lib.check(name, rc)
        return y

    def backward(self, win, est, y, target, stream=None):
        """Gradient of the MSE into self.grad; returns the loss partial sums
        tensor (sum / N is the loss)."""
        B, Hc, Wc = win.shape
        nblk = (B * Hc * Wc + 255) // 256
        lp = torch.empty(nblk, dtype=torch.float32, device=win.device)
        rc = _lib_sur().spk_sur_backward(self.params.data_ptr(), win.data_ptr(), est.data_ptr(),
                                         B, Hc, Wc, y.data_ptr(), target.data_ptr(),
                                         self.grad.data_ptr(), lp.data_ptr(),
                                         self.workspace(B, Hc, Wc).data_ptr(),
                                         _stream_handle(stream))
        _lib.check("spk_sur_backward", rc)
        return lp

    def adam(self, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self.step_count += 1
        rc = _lib_sur().spk_sur_adam(self.params.data_ptr(), self.m.data_ptr(), self.v.data_ptr(),
                                     self.grad.data_ptr(), self.step_count, lr, beta1, beta2, eps,
                                     _stream_handle(stream))
        _lib.check("spk_sur_adam", rc)

    @staticmethod
    def mux(y, est, stable, out=None, stream=None):
        out = out if out is not None else torch.empty_like(y)
        rc = _lib_sur().spk_sur_mux(y.data_ptr(), est.data_ptr(), stable.data_ptr(), y.numel(),
                                    out.data_ptr(), _stream_handle(stream))
        _lib.check("spk_sur_mux", rc)
        return out

    def train_step(self, win, est, target, lr=1e-3):
        y = self.forward(win, est)
        lp = self.backward(win, est, y, target)
        self.adam(lr=lr)
        return lp

    def state(self):
        return {"params": self.params.cpu().numpy().copy(), "m": self.m.cpu().numpy().copy(),
                "v": self.v.cpu().numpy().copy(), "step": self.step_count}

    # -- checkpoints ----------------------------------------------------------
    CKPT_VERSION = 1

    def save(self, path, extra: dict | None = None):
        """Write parameters, both Adam moments and the step count (float32
        values exactly as on the device) to a NumPy .npz file; ``extra``
        (JSON-serialisable, e.g. a sampler's random state) is stored beside
        them.  No pickled objects: load() reads it with allow_pickle=False."""
        import json
        st = self.state()
        blob = np.frombuffer(json.dumps(extra or {}).encode(), dtype=np.uint8)
        with open(path, "wb") as f:
            np.savez(f, version=np.int64(self.CKPT_VERSION), params=st["params"], m=st["m"],
                     v=st["v"], step=np.int64(st["step"]), extra=blob)

    @classmethod
    def load(cls, path, device="cuda"):
        """A Surrogate restored from save(): returns (model, extra)."""
        import json
        with np.load(path, allow_pickle=False) as z:
            if int(z["version"]) != cls.CKPT_VERSION:
                raise ValueError("checkpoint version %d" % int(z["version"]))
            model = cls(z["params"], device=device)
            model.m.copy_(torch.from_numpy(z["m"].astype(np.float32)))
            model.v.copy_(torch.from_numpy(z["v"].astype(np.float32)))
            model.step_count = int(z["step"])
            extra = json.loads(bytes(z["extra"]).decode() or "{}")
        return model, extra


# ---------------------------------------------------------------------------
# training data: seeded static block scenes, targets from the plain method

def scene_velocity(seed: int, vmax: float = 2.0):
    """The translation velocity (px/frame) of a moving block scene: speed
    uniform in (0, vmax], direction uniform, both from the scene's seed."""
    import spkgen
    speed = vmax * (1.0 - spkgen.rng_u64(seed, 7, 0) / 2.0 ** 64)
    ang = 2.0 * math.pi * (spkgen.rng_u64(seed, 7, 1) / 2.0 ** 64)
    return speed * math.cos(ang), speed * math.sin(ang)


class SceneSet:
    """Block scenes resident on the device with long-window plain targets at
    a few times per scene.  ``moving``: the blocks translate at
    scene_velocity(seed) instead of standing still.  ``target``: "whole"
    (FSR over the whole stream, valued at t) or "causal" (FSR over the
    frames up to t alone, valued at t: what a live system can know)."""

    def __init__(self, seeds, H=250, W=400, T=4096, target_times=(31, 1055, 2079, 3103, 4095),
                 theta=1.0, device="cuda", nthreads=None, moving=False, target="whole",
                 keep_host=True):
        import spkgen
        assert target in ("whole", "causal")
        self.H, self.W, self.T, self.theta = H, W, T, theta
        self.seeds = list(seeds)
        self.target_times = list(target_times)
        self.streams, self.targets, self.host = [], [], []
        for sd in self.seeds:
            vx, vy = scene_velocity(sd) if moving else (0.0, 0.0)
            s = spkgen.blocks(H, W, T, sd, vx=vx, vy=vy, nthreads=nthreads)
            ds = torch.from_numpy(s).to(device)
            self.streams.append(ds)
            if target == "whole":
                tg = reconstruct(ds, H, W, T, theta, self.target_times, order=FSR)
            else:
                tg = torch.empty((len(self.target_times), H, W), dtype=torch.float32,
                                 device=device)
                for k, t in enumerate(self.target_times):
                    reconstruct(ds[:t + 1], H, W, t + 1, theta, [t], order=FSR, out=tg[k])
            self.targets.append(tg)
            if keep_host:
                self.host.append(s)

    def extend(self, other: "SceneSet"):
        """Add another set's scenes (same shape and target times)."""
        assert (other.H, other.W, other.T) == (self.H, self.W, self.T)
        assert other.target_times == self.target_times
        self.seeds += other.seeds
        self.streams += other.streams
        self.targets += other.targets
        self.host += other.host
        return self

    def samples(self, rng, B, Hc, Wc):
        out = []
        for _ in range(B):
            i = int(rng.integers(len(self.seeds)))
            k = int(rng.integers(len(self.target_times)))
            out.append(dict(stream=self.streams[i], H=self.H, W=self.W, T=self.T,
                            oy=int(rng.integers(0, self.H - Hc + 1)),
                            ox=int(rng.integers(0, self.W - Wc + 1)),
                            t=self.target_times[k], target=self.targets[i][k]))
        return out


def train(model: Surrogate, scenes: SceneSet, steps: int, B: int = 16, Hc: int = 64,
          Wc: int = 64, lr: float = 2e-3, seed: int = 0, log_every: int = 0, rng=None,
          schedule_steps: int | None = None):
    """Adam on random crops; returns the per-step losses (host floats).
    ``rng`` (a numpy Generator) replaces the seed, e.g. to continue a run
    from a checkpoint; the cosine learning-rate schedule runs over
    ``schedule_steps`` (default ``steps``) and is indexed by the model's
    step count, so a resumed run continues it."""
    rng = np.random.default_rng(seed) if rng is None else rng
    total = max(1, schedule_steps if schedule_steps is not None else steps)
    first = model.step_count if schedule_steps is not None else 0
    losses = []
    n = B * Hc * Wc
    parts = []
    for step in range(steps):
        # cosine decay of the learning rate
        lr_t = lr * 0.5 * (1 + math.cos(math.pi * (first + step) / total))
        win, est, st, tgt = Surrogate.input(scenes.samples(rng, B, Hc, Wc), Hc, Wc,
                                            scenes.theta, with_target=True)
        parts.append(model.train_step(win, est, tgt, lr=lr_t))
        if log_every and (step + 1) % log_every == 0:
            l = float(torch.stack([p.sum() for p in parts]).cpu().sum()) / (n * len(parts))
            print("step %d loss %.6g" % (step + 1, l), flush=True)
            losses.append(l)
            parts = []
    if parts:
        losses.append(float(torch.stack([p.sum() for p in parts]).cpu().sum())
                      / (n * len(parts)))
    return losses


class TrainPlan:
    """``spk_sur_train_*``: the training loop of ``model`` over fixed crops
    (per step a list of B sample dicts, as for ``Surrogate.input``) and
    learning rates, replayed step by step from one captured HIP graph.
    ``run(n)`` enqueues n steps; ``losses()`` gives the mean squared error
    of every step run so far."""

    def __init__(self, model: "Surrogate", steps_samples, lrs, Hc, Wc, theta=1.0,
                 beta1=0.9, beta2=0.999, eps=1e-8):
        steps = len(steps_samples)
        B = len(steps_samples[0])
        assert steps > 0 and 0 < B <= MAX_SAMPLES and len(lrs) == steps
        self.model, self.steps, self.B, self.Hc, self.Wc = model, steps, B, Hc, Wc
        arr = (SurSample * (steps * B))()
        for k, samples in enumerate(steps_samples):
            assert len(samples) == B
            for i, smp in enumerate(samples):
                _check_stream_tensor(smp["stream"], smp["H"], smp["W"], smp["T"])
                arr[k * B + i] = SurSample(smp["stream"].data_ptr(), smp["H"], smp["W"],
                                           smp["T"], smp["oy"], smp["ox"], smp["t"],
                                           smp["target"].data_ptr())
        self._keep = [smp["stream"] for smps in steps_samples for smp in smps] + \
            [smp["target"] for smps in steps_samples for smp in smps]
        lr = np.ascontiguousarray(lrs, dtype=np.float32)
        self.nparts = (B * Hc * Wc + 255) // 256
        self.loss_partial = torch.empty((steps, self.nparts), dtype=torch.float32,
                                        device=model.params.device)
        h = _P()
        rc = _lib_sur().spk_sur_train_create(
            ctypes.byref(h), model.params.data_ptr(), model.m.data_ptr(), model.v.data_ptr(),
            arr, lr.ctypes.data, steps, B, Hc, Wc, float(theta), beta1, beta2, eps,
            model.step_count + 1, self.loss_partial.data_ptr())
        _lib.check("spk_sur_train_create", rc)
        self._h = h
        self.done = 0

    def run(self, n: int, stream=None):
        rc = _lib_sur().spk_sur_train_run(self._h, int(n), _stream_handle(stream))
        _lib.check("spk_sur_train_run", rc)
        self.done += int(n)
        self.model.step_count += int(n)

    def losses(self) -> np.ndarray:
        n = self.B * self.Hc * self.Wc
        return (self.loss_partial[:self.done].sum(dim=1) / n).cpu().numpy()

    def close(self):
        if self._h:
            _lib_sur().spk_sur_train_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def train_graph(model: Surrogate, scenes: SceneSet, steps: int, B: int = 16, Hc: int = 64,
                Wc: int = 64, lr: float = 2e-3, seed: int = 0, log_every: int = 0):
    """``train`` with the same crops and learning rates (same seed), run
    through a ``TrainPlan``: identical parameters, without per-step host
    work.  Returns the losses averaged as ``train`` does."""
    rng = np.random.default_rng(seed)
    samples = [scenes.samples(rng, B, Hc, Wc) for _ in range(steps)]
    lrs = [lr * 0.5 * (1 + math.cos(math.pi * k / max(1, steps))) for k in range(steps)]
    plan = TrainPlan(model, samples, lrs, Hc, Wc, scenes.theta)
    try:
        every = log_every if log_every else steps
        losses = []
        while plan.done < steps:
            n = min(every, steps - plan.done)
            plan.run(n)
            if log_every:
                l = float(plan.losses()[-n:].mean())
                print("step %d loss %.6g" % (plan.done, l), flush=True)
                losses.append(l)
        if not log_every:
            losses.append(float(plan.losses().mean()))
        return losses
    finally:
        plan.close()
