"""Learned warm start on the GPU: binding of include/rve_nn.h and the encoder-decoder built on it.

The solver of the paper starts MINRES from zero (Sec. 2, eq. galres).  Here a small 3-D
convolutional encoder-decoder, trained on fields the solver itself produces, predicts the strain
fluctuation from the voxel solid fraction; solve_rve projects that start onto compatible fields and
drops it when it does not lower the residual, so the converged answer is the solver's own.

Network (every step a kernel of librve.so; this module only sequences the calls):
  input [B, n, n, n, 16] BF16: channel 0 = phi, the rest zero
  levels l = 0..3 at n/2^l voxels per axis with (16, 32, 64, 128) channels:
    encoder  a_0 = input, a_l = pool2(e_{l-1});  h_l = relu(conv3(a_l)),  e_l = relu(conv3(h_l))
    decoder  d_3 = e_3;  c_l = [up2(d_{l+1}), e_l];  g_l = relu(conv3(c_l)),  d_l = relu(conv3(g_l))
  head: FP32 out = conv1(d_0), 48 channels; channel 6J + c = component c of the fluctuation for
  unit Mandel macro strain e_J, so any macro strain E gives sum_J E_J out[6J + c] (linearity of the
  cell problem in E).
The e_l live in the upper channel slice of the concatenation buffers c_l, so the skip connection
costs no copy.  Weights are BF16 with FP32 master copies updated by Adam; activations BF16;
accumulation FP32 on MFMA.

Inference runs at the training resolution: the fine phi is averaged over factor^3 blocks, the net
predicts the 36 unit-case fields there, and a periodic trilinear prolongation contracted with E
gives the fine starting field.
"""
from __future__ import annotations

import ctypes
import json

import numpy as np

from . import RVE_OK, RveError, _torch, load_library

CHANNELS = (16, 32, 64, 128)
IN_CH = 16   # phi and 15 zero channels
OUT_CH = 48
N_TARGET = 36
POOL2, POOL2_BWD_ACC, UP2, UP2_BWD = 0, 1, 2, 3

NN_ABI_SYMBOLS = ("rve_nn_conv3d", "rve_nn_wgrad_workspace_bytes", "rve_nn_conv3d_wgrad", "rve_nn_flip_weights",
                  "rve_nn_resample", "rve_nn_pack_input", "rve_nn_loss", "rve_nn_adam", "rve_nn_to_bf16",
                  "rve_nn_restrict", "rve_nn_prolong")

_bound = None


def nnlib():
    """librve.so with the rve_nn_* signatures declared."""
    global _bound
    lib = load_library()
    if _bound is lib:
        return lib
    vp, i32, i64, f32 = ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_float
    ip = ctypes.POINTER(ctypes.c_int32)
    sig = {
        "rve_nn_conv3d": [vp, i32, i32, i32, vp, vp, i32, vp, i32, i32, i32, i32, vp, i32, i32, ip, i32, vp],
        "rve_nn_conv3d_wgrad": [vp, i32, i32, i32, vp, i32, i32, i32, vp, vp, ip, i32, vp, ctypes.c_size_t, vp],
        "rve_nn_flip_weights": [vp, vp, i32, i32, i32, vp],
        "rve_nn_resample": [i32, vp, i32, i32, i32, vp, i32, i32, vp, i32, i32, ip, vp],
        "rve_nn_pack_input": [vp, vp, i32, vp, i32, i64, i32, vp],
        "rve_nn_loss": [vp, i32, vp, i32, vp, ctypes.POINTER(ctypes.c_float), i64, i32, f32, vp, i32, vp, i32, vp],
        "rve_nn_adam": [vp, vp, vp, vp, vp, i64, f32, f32, f32, f32, i32, f32, vp],
        "rve_nn_to_bf16": [vp, vp, i64, vp],
        "rve_nn_restrict": [vp, ip, i32, vp, vp],
        "rve_nn_prolong": [vp, i32, ip, i32, vp, vp, vp],
    }
    for name, args in sig.items():
        fn = getattr(lib, name)
        fn.argtypes = args
        fn.restype = ctypes.c_int
    lib.rve_nn_wgrad_workspace_bytes.argtypes = [i32, i32, ip, i32]
    lib.rve_nn_wgrad_workspace_bytes.restype = ctypes.c_size_t
    _bound = lib
    return lib


def _chk(st, where):
    if st != RVE_OK:
        raise RveError(st, where)


def _i32(*v):
    return (ctypes.c_int32 * len(v))(*[int(a) for a in v])


def _p(t):
    return ctypes.c_void_p(t.data_ptr()) if t is not None else None


class View:
    """A channel slice of a channels-last buffer: (tensor [V, stride], offset, channels)."""

    def __init__(self, t, off=0, ch=None):
        self.t = t
        self.stride = int(t.shape[-1])
        self.off = int(off)
        self.ch = int(ch if ch is not None else self.stride - off)


def layer_specs():
    """(name, cin, cout, ksize) in forward order."""
    c = CHANNELS
    out = []
    for l in range(4):
        out.append((f"enc{l}a", IN_CH if l == 0 else c[l - 1], c[l], 3))
        out.append((f"enc{l}b", c[l], c[l], 3))
    for l in (2, 1, 0):
        out.append((f"dec{l}a", c[l + 1] + c[l], c[l], 3))
        out.append((f"dec{l}b", c[l], c[l], 3))
    out.append(("head", c[0], OUT_CH, 1))
    return out


class WarmStartNet:
    """The encoder-decoder with FP32 master weights, BF16 working copies and Adam state on one device."""

    def __init__(self, device="cuda:0", seed: int = 0):
        torch = _torch()
        self.torch = torch
        self.device = torch.device(device)
        self.lib = nnlib()
        self.layers = {}
        off = 0
        for name, cin, cout, k in layer_specs():
            taps = 27 if k == 3 else 1
            nw = taps * cout * cin
            self.layers[name] = dict(cin=cin, cout=cout, k=k, w=off, b=off + nw, nw=nw)
            off += nw + cout
        self.n_params = off
        f32 = dict(dtype=torch.float32, device=self.device)
        self.p32 = torch.zeros(off, **f32)
        self.g32 = torch.zeros(off, **f32)
        self.m = torch.zeros(off, **f32)
        self.v = torch.zeros(off, **f32)
        self.pbf = torch.zeros(off, dtype=torch.bfloat16, device=self.device)
        self.pflip = torch.zeros(off, dtype=torch.bfloat16, device=self.device)
        self.step = 0
        self._bufs = {}
        self.meta = {}
        self.init_he(seed)

    # ------------------------------------------------------------------ parameters
    def init_he(self, seed: int):
        rng = np.random.default_rng(seed)
        host = np.zeros(self.n_params, dtype=np.float32)
        for name, L in self.layers.items():
            taps = 27 if L["k"] == 3 else 1
            std = np.sqrt(2.0 / (taps * L["cin"]))
            host[L["w"]:L["w"] + L["nw"]] = rng.standard_normal(L["nw"]) * std
        self.set_params(host)

    def set_params(self, host_f32: np.ndarray):
        torch = self.torch
        self.p32.copy_(torch.from_numpy(np.ascontiguousarray(host_f32, dtype=np.float32)))
        self._refresh()

    def params(self) -> dict:
        """name -> (w [taps, cout, cin], b [cout]) as float64 numpy copies of the BF16 working weights and
        the FP32 biases (what the kernels use)."""
        wb = self.pbf.float().cpu().numpy().astype(np.float64)
        b32 = self.p32.cpu().numpy().astype(np.float64)
        out = {}
        for name, L in self.layers.items():
            taps = 27 if L["k"] == 3 else 1
            out[name] = (wb[L["w"]:L["w"] + L["nw"]].reshape(taps, L["cout"], L["cin"]),
                         b32[L["b"]:L["b"] + L["cout"]].copy())
        return out

    def grads(self) -> dict:
        g = self.g32.cpu().numpy().astype(np.float64)
        out = {}
        for name, L in self.layers.items():
            taps = 27 if L["k"] == 3 else 1
            out[name] = (g[L["w"]:L["w"] + L["nw"]].reshape(taps, L["cout"], L["cin"]),
                         g[L["b"]:L["b"] + L["cout"]].copy())
        return out

    def _stream(self):
        return ctypes.c_void_p(self.torch.cuda.current_stream(self.device).cuda_stream)

    def _refresh(self):
        """BF16 working weights and the flipped weights of the data gradient from the FP32 masters."""
        s = self._stream()
        _chk(self.lib.rve_nn_to_bf16(_p(self.p32), _p(self.pbf), self.n_params, s), "rve_nn_to_bf16")
        self._flip()

    def _flip(self):
        s = self._stream()
        for name, L in self.layers.items():
            _chk(self.lib.rve_nn_flip_weights(ctypes.c_void_p(self.pbf.data_ptr() + 2 * L["w"]),
                                              ctypes.c_void_p(self.pflip.data_ptr() + 2 * L["w"]),
                                              L["cin"], L["cout"], L["k"], s), "rve_nn_flip_weights")

    def save(self, path: str, meta: dict | None = None):
        """BF16 weights (raw uint16) and FP32 biases in an .npz (no pickled objects)."""
        wbits = self.pbf.view(self.torch.int16).cpu().numpy().view(np.uint16)
        b32 = self.p32.cpu().numpy()
        arrays = {}
        for name, L in self.layers.items():
            arrays[name + "_w_bf16"] = wbits[L["w"]:L["w"] + L["nw"]].copy()
            arrays[name + "_b"] = b32[L["b"]:L["b"] + L["cout"]].copy()
        arrays["meta"] = np.frombuffer(json.dumps(meta or self.meta).encode(), dtype=np.uint8)
        np.savez(path, **arrays)

    def load(self, path: str):
        z = np.load(path, allow_pickle=False)
        host = np.zeros(self.n_params, dtype=np.float32)
        for name, L in self.layers.items():
            bits = z[name + "_w_bf16"].astype(np.uint32) << 16
            host[L["w"]:L["w"] + L["nw"]] = bits.view(np.float32)
            host[L["b"]:L["b"] + L["cout"]] = z[name + "_b"]
        self.meta = json.loads(bytes(z["meta"]).decode()) if "meta" in z else {}
        self.set_params(host)
        return self

    # ------------------------------------------------------------------ buffers
    def _buffers(self, B: int, n: int):
        key = (B, n)
        if key in self._bufs:
            return self._bufs[key]
        if n % 8:
            raise ValueError("the network grid must be a multiple of 8 per axis")
        torch = self.torch
        c = CHANNELS
        V = [B * (n >> l) ** 3 for l in range(4)]
        bf = dict(dtype=torch.bfloat16, device=self.device)
        a = {"in": torch.zeros(V[0], IN_CH, **bf), "out": torch.zeros(V[0], OUT_CH, dtype=torch.float32,
                                                                        device=self.device),
             "dout": torch.zeros(V[0], OUT_CH, **bf), "e3": torch.zeros(V[3], c[3], **bf),
             "de3": torch.zeros(V[3], c[3], **bf)}
        for l in range(4):
            a[f"h{l}"] = torch.zeros(V[l], c[l], **bf)
            a[f"dh{l}"] = torch.zeros(V[l], c[l], **bf)
            if l > 0:
                a[f"a{l}"] = torch.zeros(V[l], c[l - 1], **bf)
                a[f"da{l}"] = torch.zeros(V[l], c[l - 1], **bf)
            if l < 3:
                a[f"c{l}"] = torch.zeros(V[l], c[l + 1] + c[l], **bf)
                a[f"dc{l}"] = torch.zeros(V[l], c[l + 1] + c[l], **bf)
                for k in ("g", "d", "dg", "dd"):
                    a[f"{k}{l}"] = torch.zeros(V[l], c[l], **bf)
        ws = 0
        for name, L in self.layers.items():
            lvl = 0 if name == "head" else int(name[3])
            ws = max(ws, self.lib.rve_nn_wgrad_workspace_bytes(L["cin"], L["cout"], _i32(B, n >> lvl, n >> lvl,
                                                                                          n >> lvl), L["k"]))
        a["ws"] = torch.empty(max(ws, 256), dtype=torch.uint8, device=self.device)
        a["partials"] = torch.zeros(1024, dtype=torch.float64, device=self.device)
        a["dims"] = [_i32(B, n >> l, n >> l, n >> l) for l in range(4)]
        self._bufs = {key: a}  # keep one shape resident
        return a

    # ------------------------------------------------------------------ layers
    def _conv(self, name, x: View, y: View, dims, relu=True, y_f32=False):
        L = self.layers[name]
        assert x.ch == L["cin"] and y.ch == L["cout"]
        _chk(self.lib.rve_nn_conv3d(_p(x.t), x.ch, x.stride, x.off,
                                    ctypes.c_void_p(self.pbf.data_ptr() + 2 * L["w"]),
                                    ctypes.c_void_p(self.p32.data_ptr() + 4 * L["b"]), y.ch, _p(y.t), y.stride, y.off,
                                    1 if y_f32 else 0, 1 if relu else 0, None, 0, 0, dims, L["k"], self._stream()),
             f"rve_nn_conv3d({name})")

    def _dgrad(self, name, dy: View, dx: View, dims, mask: View | None):
        L = self.layers[name]
        assert dy.ch == L["cout"] and dx.ch == L["cin"]
        _chk(self.lib.rve_nn_conv3d(_p(dy.t), dy.ch, dy.stride, dy.off,
                                    ctypes.c_void_p(self.pflip.data_ptr() + 2 * L["w"]), None, dx.ch, _p(dx.t),
                                    dx.stride, dx.off, 0, 0, _p(mask.t) if mask else None,
                                    mask.stride if mask else 0, mask.off if mask else 0, dims, L["k"], self._stream()),
             f"rve_nn_conv3d dgrad({name})")

    def _wgrad(self, name, x: View, dy: View, dims, ws):
        L = self.layers[name]
        _chk(self.lib.rve_nn_conv3d_wgrad(_p(x.t), x.ch, x.stride, x.off, _p(dy.t), dy.ch, dy.stride, dy.off,
                                          ctypes.c_void_p(self.g32.data_ptr() + 4 * L["w"]),
                                          ctypes.c_void_p(self.g32.data_ptr() + 4 * L["b"]), dims, L["k"], _p(ws),
                                          ws.numel(), self._stream()), f"rve_nn_conv3d_wgrad({name})")

    def _resample(self, op, x: View, y: View, dims, mask: View | None = None):
        assert x.ch == y.ch
        _chk(self.lib.rve_nn_resample(op, _p(x.t), x.ch, x.stride, x.off, _p(y.t), y.stride, y.off,
                                      _p(mask.t) if mask else None, mask.stride if mask else 0,
                                      mask.off if mask else 0, dims, self._stream()), "rve_nn_resample")

    # ------------------------------------------------------------------ passes
    def forward(self, B: int, n: int):
        """Forward pass on the packed input buffer of shape (B, n); returns the FP32 output [B n^3, 48]."""
        a = self._buffers(B, n)
        c = CHANNELS
        dims = a["dims"]
        x = View(a["in"])
        for l in range(4):
            if l > 0:
                self._resample(POOL2, View(a[f"c{l - 1}"], c[l], c[l - 1]), View(a[f"a{l}"]), dims[l - 1])
                x = View(a[f"a{l}"])
            self._conv(f"enc{l}a", x, View(a[f"h{l}"]), dims[l])
            e = View(a["e3"]) if l == 3 else View(a[f"c{l}"], c[l + 1], c[l])
            self._conv(f"enc{l}b", View(a[f"h{l}"]), e, dims[l])
        d = View(a["e3"])
        for l in (2, 1, 0):
            self._resample(UP2, d, View(a[f"c{l}"], 0, c[l + 1]), dims[l + 1])
            self._conv(f"dec{l}a", View(a[f"c{l}"]), View(a[f"g{l}"]), dims[l])
            self._conv(f"dec{l}b", View(a[f"g{l}"]), View(a[f"d{l}"]), dims[l])
            d = View(a[f"d{l}"])
        self._conv("head", d, View(a["out"]), dims[0], relu=False, y_f32=True)
        return a["out"]

    def backward(self, B: int, n: int):
        """Gradients of every parameter (into g32) from dL/dout in the 'dout' buffer."""
        a = self._buffers(B, n)
        c = CHANNELS
        dims = a["dims"]
        ws = a["ws"]
        self._wgrad("head", View(a["d0"]), View(a["dout"]), dims[0], ws)
        self._dgrad("head", View(a["dout"]), View(a["dd0"]), dims[0], View(a["d0"]))
        for l in (0, 1, 2):
            self._wgrad(f"dec{l}b", View(a[f"g{l}"]), View(a[f"dd{l}"]), dims[l], ws)
            self._dgrad(f"dec{l}b", View(a[f"dd{l}"]), View(a[f"dg{l}"]), dims[l], View(a[f"g{l}"]))
            self._wgrad(f"dec{l}a", View(a[f"c{l}"]), View(a[f"dg{l}"]), dims[l], ws)
            self._dgrad(f"dec{l}a", View(a[f"dg{l}"]), View(a[f"dc{l}"]), dims[l], View(a[f"c{l}"]))
            nxt = View(a["de3"]) if l == 2 else View(a[f"dd{l + 1}"])
            self._resample(UP2_BWD, View(a[f"dc{l}"], 0, c[l + 1]), nxt, dims[l + 1])
        for l in (3, 2, 1, 0):
            if l == 3:
                de = View(a["de3"])
            else:
                de = View(a[f"dc{l}"], c[l + 1], c[l])
                self._resample(POOL2_BWD_ACC, View(a[f"da{l + 1}"]), de, dims[l], mask=View(a[f"c{l}"], c[l + 1],
                                                                                              c[l]))
            self._wgrad(f"enc{l}b", View(a[f"h{l}"]), de, dims[l], ws)
            self._dgrad(f"enc{l}b", de, View(a[f"dh{l}"]), dims[l], View(a[f"h{l}"]))
            x = View(a["in"]) if l == 0 else View(a[f"a{l}"])
            self._wgrad(f"enc{l}a", x, View(a[f"dh{l}"]), dims[l], ws)
            if l > 0:
                self._dgrad(f"enc{l}a", View(a[f"dh{l}"]), View(a[f"da{l}"]), dims[l], None)

    def pack(self, phi_batch, n: int):
        """Input buffer from phi (torch float32 [B, n, n, n]) on the device."""
        B = phi_batch.numel() // n ** 3
        a = self._buffers(B, n)
        phi = phi_batch.contiguous()
        _chk(self.lib.rve_nn_pack_input(_p(phi), None, 0, _p(a["in"]), IN_CH, n ** 3, B, self._stream()),
             "rve_nn_pack_input")
        return B

    def loss(self, B: int, n: int, target, phi, weight3, inv_norm: float):
        """Weighted squared error against target (float32 [B, 36, n^3]), voxel weight
        weight3[0] + weight3[1] phi + weight3[2] [0 < phi < 1]; writes dL/dout into 'dout' and returns the
        device tensor of loss partials (inv_norm * their sum = loss)."""
        a = self._buffers(B, n)
        w3 = (ctypes.c_float * 3)(*[float(v) for v in weight3])
        _chk(self.lib.rve_nn_loss(_p(a["out"]), OUT_CH, _p(target), N_TARGET, _p(phi), w3,
                                  n ** 3, B, ctypes.c_float(inv_norm), _p(a["dout"]), OUT_CH, _p(a["partials"]),
                                  a["partials"].numel(), self._stream()), "rve_nn_loss")
        return a["partials"]

    def adam(self, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, weight_decay=0.0):
        self.step += 1
        _chk(self.lib.rve_nn_adam(_p(self.p32), _p(self.g32), _p(self.m), _p(self.v), _p(self.pbf), self.n_params,
                                  ctypes.c_float(lr), ctypes.c_float(beta1), ctypes.c_float(beta2), ctypes.c_float(eps),
                                  self.step, ctypes.c_float(weight_decay), self._stream()), "rve_nn_adam")
        self._flip()

    def train_step(self, phi, target, inv_norm: float, lr: float, weight3=(0.1, 1.0, 0.0),
                   weight_decay: float = 0.0):
        """One Adam step on a batch: phi float32 [B, n, n, n], target float32 [B, 36, n^3] (device);
        inv_norm = 1 / (36 * sum over the batch of the voxel weights) makes the loss a weighted mean.
        Returns the device tensor of loss partials (inv_norm * their sum = loss)."""
        n = int(phi.shape[-1])
        B = self.pack(phi, n)
        self.forward(B, n)
        part = self.loss(B, n, target, phi, weight3, inv_norm)
        self.backward(B, n)
        self.adam(lr, weight_decay=weight_decay)
        return part

    # ------------------------------------------------------------------ inference
    def predict(self, phi, macro_strain, grid: int = 64):
        """Starting fields eps0 [n_cases, 6, N0, N1, N2] (float32, device) for phi [N0, N1, N2] (cubic,
        N a multiple of grid) and macro strains [n_cases, 6]: the network runs on the grid-sized cell
        (phi averaged over (N/grid)^3 blocks) and its 36 unit-case fields are prolonged and
        contracted with each macro strain."""
        torch = self.torch
        N = tuple(int(v) for v in phi.shape)
        if len(set(N)) != 1 or N[0] % grid:
            raise ValueError(f"phi must be cubic with a side that is a multiple of {grid}")
        f = N[0] // grid
        E = np.ascontiguousarray(np.asarray(macro_strain, dtype=np.float64).reshape(-1, 6))
        s = self._stream()
        if f > 1:
            coarse = torch.empty((grid, grid, grid), dtype=torch.float32, device=self.device)
            _chk(self.lib.rve_nn_restrict(_p(phi.contiguous()), _i32(*N), f, _p(coarse), s), "rve_nn_restrict")
        else:
            coarse = phi.contiguous()
        self.pack(coarse, grid)
        out = self.forward(1, grid)
        eps0 = torch.empty((E.shape[0], 6) + N, dtype=torch.float32, device=self.device)
        Ed = torch.from_numpy(E).to(self.device)
        for cs in range(E.shape[0]):
            _chk(self.lib.rve_nn_prolong(_p(out), OUT_CH, _i32(grid, grid, grid), f,
                                         ctypes.c_void_p(Ed.data_ptr() + 48 * cs), _p(eps0[cs]), s), "rve_nn_prolong")
        return eps0

