"""Learned surrogate of the SSLBM: a periodic 3x3-convolution U-Net on BF16
MFMA (FP32 accumulation) that advances the five SEIRD densities by a fixed
number of SSLBM steps in one evaluation, trained on the GPU on states the
SSLBM itself produces, with plain SSLBM as its fallback and error judge.

Every operation runs in the library's HIP kernels (include/surrogate.h);
this module allocates the buffers (torch, device memory only) and calls the
kernels in order: it is the network's layer plan and the training and
rollout loops.

Network (levels L, base width C, channels C_l = C 2^l):
  encoder level l: a_l = act(conv(in_l)), e_l = act(conv(a_l)),
                   in_0 = packed input (16 channels), in_l = pool(e_{l-1});
  decoder level l (L-2 .. 0): cat_l = [up(h_{l+1}), e_l],
                   b_l = act(conv(cat_l)), h_l = act(conv(b_l)), h_{L-1} = e_{L-1};
  output: conv(h_0) -> 16 FP32 channels, of which the first 5 are the
  increments of S, E, I, R, D in units of per-compartment scales.
The prediction is rho + scale_out * out (the network learns the increment).
e_l lives inside cat_l (channel offset C_{l+1}), so the skip connection
needs no copy.
"""
from __future__ import annotations

import ctypes
import math
import time
from dataclasses import dataclass

import numpy as np

from .binding import OK, SSLBMError, library

LEAKY, OUT_F32 = 1, 2
IN_CHANNELS = OUT_CHANNELS = 16


def _torch():
    import torch
    return torch


def _ptr(t, offset_elems: int = 0):
    return ctypes.c_void_p(t.data_ptr() + offset_elems * t.element_size())


def _check(st, what):
    if st != OK:
        raise SSLBMError(st, what)


def _floats(v):
    return (ctypes.c_float * len(v))(*[float(x) for x in v])


class _View:
    """A BF16 NHWC view: buffer, channel offset, channels (pitch = buffer's)."""

    def __init__(self, buf, offset: int, channels: int):
        self.buf, self.offset, self.c = buf, offset, channels

    @property
    def pitch(self):
        return self.buf.shape[-1]

    @property
    def ptr(self):
        return _ptr(self.buf, self.offset)


def _copy(v):
    """A copy of the channels a view (or a whole tensor) covers."""
    if isinstance(v, _View):
        return v.buf[..., v.offset:v.offset + v.c].clone()
    return v.clone()


def _up_cat_copy(low, skip):
    """The concatenation [up2(low), skip] that a decoder convolution reads
    without materialising it, as one tensor (for records)."""
    torch = _torch()
    up = _copy(low).repeat_interleave(2, dim=1).repeat_interleave(2, dim=2)
    return torch.cat([up, _copy(skip)], dim=3)


@dataclass
class _Conv:
    cin: int
    cout: int
    act: bool
    w_off: int = 0  # offset of W [cout][9][cin] in the flat parameter vector
    b_off: int = 0  # offset of b [cout]
    f_off: int = 0  # offset of the flipped W [cin][9][cout] in UNet.flipped


class UNet:
    """The surrogate network: parameters (FP32 master, BF16 copy), Adam
    state, and the forward and backward passes over a batch."""

    def __init__(self, levels: int = 4, base: int = 32, slope: float = 0.1, seed: int = 0,
                 overlap_sums: bool = True, fuse_up_bwd: bool = True):
        torch = _torch()
        self.lib = library()
        self.levels, self.base, self.slope = levels, base, slope
        # the weight gradients' split sums on a second stream (True), or on
        # the pass's own stream (False); the same bits either way
        self.overlap_sums = overlap_sums
        # a decoder's upsampling adjoint inside its first convolution's
        # backward-data pass (True), or as a pass of its own; the same bits
        self.fuse_up_bwd = fuse_up_bwd
        self.ch = [base * 2 ** l for l in range(levels)]
        convs = []
        c = IN_CHANNELS
        for l in range(levels):
            convs += [_Conv(c, self.ch[l], True), _Conv(self.ch[l], self.ch[l], True)]
            c = self.ch[l]
        for l in range(levels - 2, -1, -1):
            convs += [_Conv(self.ch[l + 1] + self.ch[l], self.ch[l], True),
                      _Conv(self.ch[l], self.ch[l], True)]
        convs.append(_Conv(self.ch[0], OUT_CHANNELS, False))
        off = 0
        for cv in convs:
            cv.w_off = off
            off += cv.cout * 9 * cv.cin
            off = (off + 7) // 8 * 8  # keep every weight block 16-byte aligned in BF16
            cv.b_off = off
            off += (cv.cout + 7) // 8 * 8
        self.convs, self.count = convs, off
        # the backward-data weights ([cin][9][cout], flipped in space), one
        # block per convolution, rebuilt from theta_bf16 by each backward pass
        foff = 0
        for cv in convs:
            cv.f_off = foff
            foff += (cv.cout * 9 * cv.cin + 7) // 8 * 8
        # He initialisation for the activated layers; a small last layer, so
        # the untrained network predicts increments near zero
        rng = np.random.default_rng(seed)
        theta = np.zeros(off, np.float32)
        for k, cv in enumerate(convs):
            std = math.sqrt(2.0 / (9 * cv.cin)) * (1.0 if cv.act else 0.1)
            theta[cv.w_off:cv.w_off + cv.cout * 9 * cv.cin] = rng.normal(
                0.0, std, cv.cout * 9 * cv.cin)
        self.theta = torch.tensor(theta, device="cuda")
        self.theta_bf16 = torch.empty(off, dtype=torch.bfloat16, device="cuda")
        self.flipped = torch.empty(foff, dtype=torch.bfloat16, device="cuda")
        self.grad = torch.zeros_like(self.theta)
        self.m = torch.zeros_like(self.theta)
        self.v = torch.zeros_like(self.theta)
        self.step_count = 0
        _check(self.lib.sur_to_bf16(_ptr(self.theta), _ptr(self.theta_bf16), off, None),
               "sur_to_bf16")
        self._shape = None
        self._sets = {}  # activation and gradient buffers per (batch, h, w)
        # When a list, every convolution of the forward and backward passes
        # appends copies of the exact tensors it read and wrote (dicts, see
        # _conv and _conv_backward), so that each layer can be checked on its
        # own inputs. It costs a device copy per tensor; None in normal use.
        self.record = None

    @property
    def parameters(self) -> int:
        return sum(cv.cout * 9 * cv.cin + cv.cout for cv in self.convs)

    def flops(self, batch: int, h: int, w: int) -> float:
        """Multiply-add flops (x2) of one forward pass."""
        total = 0.0
        for k, cv in enumerate(self._levels_of_convs()):
            hh, ww = h >> cv[1], w >> cv[1]
            total += 2.0 * batch * hh * ww * 9 * cv[0].cin * cv[0].cout
        return total

    def _levels_of_convs(self):
        L = self.levels
        lv = []
        for l in range(L):
            lv += [l, l]
        for l in range(L - 2, -1, -1):
            lv += [l, l]
        lv.append(0)
        return list(zip(self.convs, lv))

    # ------------------------------------------------------------ buffers --
    _BUFFER_NAMES = ("x0", "a", "pool", "cat", "e_dense", "e_last", "b", "hdec", "out", "g_cat",
                     "g_e_dense", "g_l",
                     "g_l2", "g_pool", "g_e_last", "dout", "wgrad_ws", "dims")
    # The backward pass runs the sums of each weight gradient's splits on a
    # second stream (default priority), overlapped with the rest of the
    # pass: every convolution has its own workspace and event for that.

    def _buffers(self, n, h, w):
        """Make the buffers of batch n at h x w current. Each shape's set is
        kept, so alternating between shapes (a rollout's whole grid and its
        judge tiles) allocates nothing after the first use of each."""
        if self._shape != (n, h, w):
            self._fused_up = None  # no forward pass on this shape yet
        if self._shape == (n, h, w):
            return
        if (n, h, w) in self._sets:
            for name, val in zip(self._BUFFER_NAMES, self._sets[(n, h, w)]):
                setattr(self, name, val)
            self._shape = (n, h, w)
            return
        torch = _torch()
        bf = torch.bfloat16
        L, ch = self.levels, self.ch
        if h % (1 << (L - 1)) or w % (8 << (L - 1)):
            raise ValueError(f"grid {h}x{w} must be divisible by {1 << (L - 1)} (rows) and "
                             f"{8 << (L - 1)} (columns)")
        dims = [(h >> l, w >> l) for l in range(L)]
        mk = lambda l, c: torch.empty((n, dims[l][0], dims[l][1], c), dtype=bf, device="cuda")
        self.x0 = torch.empty((n, h, w, IN_CHANNELS), dtype=bf, device="cuda")
        self.a = [mk(l, ch[l]) for l in range(L)]
        self.pool = [None] + [mk(l, ch[l - 1]) for l in range(1, L)]
        self.cat = [mk(l, ch[l + 1] + ch[l]) for l in range(L - 1)]
        # e_l on its own, for the levels whose decoder reads the upsampled
        # tensor directly: a channel slice of cat_l shares every pixel's
        # cache lines with the upsampled channels, which that decoder never
        # reads, so reading and writing the slice moves about twice its bytes
        self.e_dense = [mk(l, ch[l]) for l in range(L - 1)]
        self.e_last = mk(L - 1, ch[L - 1])
        self.b = [mk(l, ch[l]) for l in range(L - 1)]
        self.hdec = [mk(l, ch[l]) for l in range(L - 1)]
        self.out = torch.empty((n, h, w, OUT_CHANNELS), dtype=torch.float32, device="cuda")
        # gradients
        self.g_cat = [mk(l, ch[l + 1] + ch[l]) for l in range(L - 1)]
        # the gradient of e_l on its own where the upsampling adjoint runs
        # inside the backward-data pass (as e_dense, for the same reason)
        self.g_e_dense = [mk(l, ch[l]) for l in range(L - 1)]
        self.g_l = [mk(l, ch[l]) for l in range(L)]      # gradient of a level's C_l tensors
        self.g_l2 = [mk(l, ch[l]) for l in range(L)]
        self.g_pool = [None] + [mk(l, ch[l - 1]) for l in range(1, L)]
        self.g_e_last = mk(L - 1, ch[L - 1])
        self.dout = torch.empty((n, h, w, OUT_CHANNELS), dtype=bf, device="cuda")
        self.wgrad_ws = None  # per-convolution workspaces, made by the first backward pass
        self.dims = dims
        self._shape = (n, h, w)
        self._sets[(n, h, w)] = tuple(getattr(self, name) for name in self._BUFFER_NAMES)

    def e_view(self, l):
        """View of encoder output e_l: its own buffer at the bottleneck and
        where the decoder reads the upsampled tensor directly (this pass),
        else inside cat_l next to the upsampled copy."""
        if l == self.levels - 1:
            return _View(self.e_last, 0, self.ch[l])
        if self._fused_up is not None and self._fused_up[l]:
            return _View(self.e_dense[l], 0, self.ch[l])
        return _View(self.cat[l], self.ch[l + 1], self.ch[l])

    def _up_fits(self, l):
        """Decoder level l can read its upsampled input directly (the image
        holds halo tiles and the upsampled channels come in 32-channel
        chunks)."""
        hh, ww = self.dims[l]
        return hh >= 8 and ww >= 32 and self.ch[l + 1] % 32 == 0

    # ------------------------------------------------------------ forward --
    def _conv(self, k, src: _View, dst, l, f32=False, pooled=None):
        """Convolution k of level l from src into dst; with `pooled` (a BF16
        tensor of half the size) also the 2 x 2 means of dst, in one pass."""
        cv = self.convs[k]
        n = self._shape[0]
        hh, ww = self.dims[l]
        flags = (LEAKY if cv.act else 0) | (OUT_F32 if f32 else 0)
        dptr = dst.ptr if isinstance(dst, _View) else _ptr(dst)
        dpitch = dst.pitch if isinstance(dst, _View) else dst.shape[-1]
        args = (src.ptr, src.pitch, n, hh, ww, cv.cin, _ptr(self.theta_bf16, cv.w_off),
                _ptr(self.theta, cv.b_off), dptr, dpitch, cv.cout, flags, self.slope)
        if pooled is None:
            _check(self.lib.sur_conv3x3_forward(*args, None), "sur_conv3x3_forward")
        else:
            _check(self.lib.sur_conv3x3_forward_pool(*args, _ptr(pooled), pooled.shape[-1], None),
                   "sur_conv3x3_forward_pool")
        if self.record is not None:
            self.record.append({"pass": "forward", "k": k, "x": _copy(src), "y": _copy(dst),
                                "pooled": None if pooled is None else pooled.clone()})

    def _conv_up(self, k, low: _View, skip: _View, dst: _View, l):
        """Convolution k of decoder level l on [up2(low), skip] without the
        upsampled copy (sur_conv3x3_forward_up); False where the image is
        too small for it (the caller then upsamples explicitly)."""
        cv = self.convs[k]
        n = self._shape[0]
        hh, ww = self.dims[l]
        if not self._up_fits(l) or low.c != self.ch[l + 1]:
            return False
        flags = LEAKY if cv.act else 0
        _check(self.lib.sur_conv3x3_forward_up(
            low.ptr, low.pitch, low.c, skip.ptr, skip.pitch, n, hh, ww, cv.cin,
            _ptr(self.theta_bf16, cv.w_off), _ptr(self.theta, cv.b_off), dst.ptr, dst.pitch,
            cv.cout, flags, self.slope, None), "sur_conv3x3_forward_up")
        if self.record is not None:
            self.record.append({"pass": "forward", "k": k, "x": _up_cat_copy(low, skip),
                                "y": _copy(dst), "pooled": None})
        return True

    def _low_view(self, l):
        """The half-resolution input of decoder level l's upsampling: the
        decoder output of level l + 1, or the bottleneck's encoder output."""
        L = self.levels
        return self.e_view(L - 1) if l + 1 == L - 1 else _View(self.hdec[l + 1], 0, self.ch[l + 1])

    def forward_packed(self, fuse_up=True):
        """Network pass on self.x0 into self.out (FP32 NHWC, 16 channels).
        fuse_up: decoder convolutions read the upsampled half-resolution
        tensor directly, where the image allows (same bits as the explicit
        upsampled copy; the backward pass reads the same views)."""
        L, ch, lib = self.levels, self.ch, self.lib
        n = self._shape[0]
        # decided before the encoder runs: it writes e_l where the decoder
        # will read it
        self._fused_up = [fuse_up and self._up_fits(l) for l in range(max(L - 1, 0))]
        k = 0
        for l in range(L):
            src = _View(self.x0, 0, IN_CHANNELS) if l == 0 else _View(self.pool[l], 0, ch[l - 1])
            self._conv(k, src, _View(self.a[l], 0, ch[l]), l)
            # e_l, and (below the last level) its 2 x 2 means: the next input
            self._conv(k + 1, _View(self.a[l], 0, ch[l]), self.e_view(l), l,
                       pooled=self.pool[l + 1] if l + 1 < L else None)
            k += 2
        for l in range(L - 2, -1, -1):
            hh, ww = self.dims[l + 1]
            low = self._low_view(l)
            dst = _View(self.b[l], 0, ch[l])
            if self._fused_up[l]:
                if not self._conv_up(k, low, self.e_view(l), dst, l):
                    raise RuntimeError("decoder level cannot read its upsampled input directly")
            else:
                _check(lib.sur_up2(low.ptr, low.pitch, n, hh, ww, ch[l + 1],
                                   _ptr(self.cat[l]), self.cat[l].shape[-1], None), "sur_up2")
                self._conv(k, _View(self.cat[l], 0, ch[l + 1] + ch[l]), dst, l)
            self._conv(k + 1, _View(self.b[l], 0, ch[l]), _View(self.hdec[l], 0, ch[l]), l)
            k += 2
        h_view = _View(self.hdec[0], 0, ch[0]) if L > 1 else self.e_view(0)
        self._conv(k, h_view, self.out, 0, f32=True)
        return self.out

    # ----------------------------------------------------------- backward --
    def _flip_weights(self):
        """The backward-data weights of every convolution from theta_bf16,
        in one launch per 32 convolutions, on the side stream."""
        vp = ctypes.c_void_p
        for k0 in range(0, len(self.convs), 32):
            cvs = self.convs[k0:k0 + 32]
            m = len(cvs)
            w = (vp * m)(*[_ptr(self.theta_bf16, cv.w_off) for cv in cvs])
            f = (vp * m)(*[_ptr(self.flipped, cv.f_off) for cv in cvs])
            co = (ctypes.c_int * m)(*[cv.cout for cv in cvs])
            ci = (ctypes.c_int * m)(*[cv.cin for cv in cvs])
            _check(self.lib.sur_flip_weights(m, w, co, ci, f, vp(self._side.cuda_stream)),
                   "sur_flip_weights")

    def _backward_setup(self):
        """The per-convolution weight-gradient workspaces of the current
        shape, the side stream and the events (created on first use)."""
        torch = _torch()
        if getattr(self, "_side", None) is None:
            self._side = torch.cuda.Stream()
            self._events = [torch.cuda.Event() for _ in self.convs]
            self._flip_done = torch.cuda.Event()
            for ev in self._events + [self._flip_done]:
                ev.record(torch.cuda.default_stream())  # creates the event
        if self.wgrad_ws is None:
            n = self._shape[0]
            self.wgrad_ws = [
                torch.empty(self.lib.sur_conv3x3_backward_weight_workspace(
                    n, self.dims[l][0], self.dims[l][1], cv.cin, cv.cout),
                    dtype=torch.uint8, device="cuda")
                for cv, l in self._levels_of_convs()]
            self._sets[self._shape] = tuple(getattr(self, name) for name in self._BUFFER_NAMES)

    def _conv_backward(self, k, x, dz: _View, gx, act, l, up=None):
        """Gradients of conv k from dz (the gradient of its pre-activation
        output): weight and bias gradients into self.grad (their split sums
        on the side stream), and dX into view gx unless gx is None, through
        the adjoint of the activation whose output is `act` (the
        convolution's own input) when act is not None. x: the input view,
        or (low, skip) for a decoder convolution that read its upsampled
        input directly. up = (below, low): the upsampled channels' gradient
        goes, through the upsampling adjoint and the adjoint of the
        activation whose output is `low`, to the half-resolution view
        `below`, and gx is a view of the remaining (skip) channels only."""
        cv = self.convs[k]
        lib = self.lib
        n = self._shape[0]
        hh, ww = self.dims[l]
        ws = self.wgrad_ws[k]
        dw, db = _ptr(self.grad, cv.w_off), _ptr(self.grad, cv.b_off)
        low, skip = x if isinstance(x, tuple) else (None, x)
        vp = ctypes.c_void_p
        _check(lib.sur_conv3x3_backward_weight_overlap(
            None if low is None else low.ptr, 0 if low is None else low.pitch,
            0 if low is None else low.c, skip.ptr, skip.pitch, dz.ptr, dz.pitch, n, hh, ww,
            cv.cin, cv.cout, dw, db, _ptr(ws), ws.numel(), None,
            vp(self._side.cuda_stream) if self.overlap_sums else None,
            vp(self._events[k].cuda_event)), "sur_conv3x3_backward_weight_overlap")
        if gx is not None:
            if self._flip_pending:  # the flipped weights, from the side stream
                _torch().cuda.default_stream().wait_event(self._flip_done)
                self._flip_pending = False
            if up is not None:
                below, lo = up
                _check(lib.sur_conv3x3_backward_data_up(
                    dz.ptr, dz.pitch, n, hh, ww, cv.cout, _ptr(self.flipped, cv.f_off), cv.cin,
                    lo.c, gx.ptr, gx.pitch, below.ptr, below.pitch, lo.ptr, lo.pitch,
                    self.slope, None), "sur_conv3x3_backward_data_up")
            else:
                _check(lib.sur_conv3x3_backward_data_flipped(
                    dz.ptr, dz.pitch, n, hh, ww, cv.cout, _ptr(self.flipped, cv.f_off), cv.cin,
                    gx.ptr, gx.pitch, None if act is None else act.ptr,
                    0 if act is None else act.pitch, self.slope, None),
                    "sur_conv3x3_backward_data_flipped")
        if self.record is not None:
            _torch().cuda.default_stream().wait_stream(self._side)  # dW, db written
            self.record.append({
                "pass": "backward", "k": k,
                "x": _up_cat_copy(*x) if isinstance(x, tuple) else _copy(x),
                "dz": _copy(dz), "dx": None if gx is None else _copy(gx),
                "act": None if act is None else _copy(act),
                "dw": self.grad[cv.w_off:cv.w_off + cv.cout * 9 * cv.cin].clone(),
                "db": self.grad[cv.b_off:cv.b_off + cv.cout].clone()})

    def backward_packed(self):
        """Parameter gradients (into self.grad) from self.dout (BF16 NHWC,
        the loss gradient of self.out), after forward_packed(). Every
        gradient tensor a convolution reads is already its pre-activation
        gradient: the activation adjoints run inside the kernels that
        produce them (backward data, the upsampling and pooling adjoints)."""
        if getattr(self, "_fused_up", None) is None:
            raise RuntimeError("backward_packed needs a preceding forward_packed() on this shape")
        L, ch, lib = self.levels, self.ch, self.lib
        n = self._shape[0]
        torch = _torch()
        main = torch.cuda.default_stream()  # the stream of every library call here
        self._backward_setup()
        # the side stream starts after everything before (theta_bf16 from
        # the last Adam step); the flip there overlaps the first weight
        # gradient, and the first backward-data waits for it
        self._side.wait_stream(main)
        self._flip_weights()
        self._flip_done.record(self._side)
        self._flip_pending = True  # the first backward-data waits for it
        self._bwd_fused = [False] * max(L - 1, 0)
        k = len(self.convs) - 1
        # output layer (no activation: dZ = dout); its input is the last
        # activation's output
        h_in = _View(self.hdec[0], 0, ch[0]) if L > 1 else self.e_view(0)
        self._conv_backward(k, h_in, _View(self.dout, 0, OUT_CHANNELS),
                            _View(self.g_l[0], 0, ch[0]), h_in, 0)
        # decoder, from the top level down
        for l in range(0, L - 1):
            k_first = len(self.convs) - 1 - 2 * (l + 1)
            b = _View(self.b[l], 0, ch[l])
            g_b = _View(self.g_l2[l], 0, ch[l])
            self._conv_backward(k_first + 1, b, _View(self.g_l[l], 0, ch[l]), g_b, b, l)
            low = self._low_view(l)
            x = ((low, self.e_view(l)) if self._fused_up[l]
                 else _View(self.cat[l], 0, ch[l + 1] + ch[l]))
            # the upsampled part's gradient -> the pre-activation gradient of
            # the level below's output
            below = (_View(self.g_l[l + 1], 0, ch[l + 1]) if l + 1 < L - 1
                     else _View(self.g_e_last, 0, ch[L - 1]))
            g_cat = _View(self.g_cat[l], 0, ch[l + 1] + ch[l])
            # where the forward read the upsampled tensor directly, one pass
            # gives the skip gradient (on its own) and the half-resolution one
            # (a recording pass keeps the full-resolution gradient for its checks)
            self._bwd_fused[l] = self.fuse_up_bwd and self._fused_up[l] and self.record is None
            if self._bwd_fused[l]:
                self._conv_backward(k_first, x, g_b, _View(self.g_e_dense[l], 0, ch[l]), None, l,
                                    up=(below, low))
            else:
                self._conv_backward(k_first, x, g_b, g_cat, None, l)
                hh, ww = self.dims[l + 1]
                _check(lib.sur_up2_backward_act(
                    _ptr(self.g_cat[l]), self.g_cat[l].shape[-1], n, hh, ww, ch[l + 1],
                    below.ptr, below.pitch, low.ptr, low.pitch, self.slope, None),
                    "sur_up2_backward_act")
        # encoder, from the bottleneck up
        for l in range(L - 1, -1, -1):
            k1 = 2 * l
            e = self.e_view(l)
            if l == L - 1:
                g_e = _View(self.g_e_last, 0, ch[l])
            else:
                # the skip gradient is already there; the pooled path's
                # gradient adds to it, through the activation adjoint
                g_e = (_View(self.g_e_dense[l], 0, ch[l]) if self._bwd_fused[l]
                       else _View(self.g_cat[l], ch[l + 1], ch[l]))
                hh, ww = self.dims[l]
                _check(lib.sur_pool2_backward_act(_ptr(self.g_pool[l + 1]), ch[l], n, hh, ww,
                                                  ch[l], g_e.ptr, g_e.pitch, 1, e.ptr, e.pitch,
                                                  self.slope, None), "sur_pool2_backward_act")
            a = _View(self.a[l], 0, ch[l])
            g_a = _View(self.g_l2[l], 0, ch[l])
            self._conv_backward(k1 + 1, a, g_e, g_a, a, l)
            src = _View(self.x0, 0, IN_CHANNELS) if l == 0 else _View(self.pool[l], 0, ch[l - 1])
            g_src = None if l == 0 else _View(self.g_pool[l], 0, ch[l - 1])
            self._conv_backward(k1, src, g_a, g_src, None, l)
        main.wait_stream(self._side)  # self.grad complete; workspaces free

    def adam(self, lr: float, beta1=0.9, beta2=0.999, eps=1e-8):
        self.step_count += 1
        _check(self.lib.sur_adam(_ptr(self.theta), _ptr(self.theta_bf16), _ptr(self.grad),
                                 _ptr(self.m), _ptr(self.v), self.count, self.step_count,
                                 lr, beta1, beta2, eps, None), "sur_adam")

    def copy_from(self, other: "UNet"):
        self.theta.copy_(other.theta)
        _check(self.lib.sur_to_bf16(_ptr(self.theta), _ptr(self.theta_bf16), self.count, None),
               "sur_to_bf16")

    def weights_numpy(self):
        """(W [cout][9][cin], b) per conv as the BF16 values the kernels use,
        in FP64 (for checks against a reference implementation)."""
        wb = self.theta_bf16.float().cpu().numpy().astype(np.float64)
        th = self.theta.cpu().numpy().astype(np.float64)
        out = []
        for cv in self.convs:
            w = wb[cv.w_off:cv.w_off + cv.cout * 9 * cv.cin].reshape(cv.cout, 9, cv.cin)
            out.append((w, th[cv.b_off:cv.b_off + cv.cout]))
        return out

    def grads_numpy(self):
        g = self.grad.cpu().numpy().astype(np.float64)
        return [(g[cv.w_off:cv.w_off + cv.cout * 9 * cv.cin].reshape(cv.cout, 9, cv.cin),
                 g[cv.b_off:cv.b_off + cv.cout]) for cv in self.convs]


# ------------------------------------------------------------- the model --

def param_planes(params_list):
    """The 9 constant input planes of each instance: rates relative to the
    workloads' typical values and log10 lattice diffusivities (0 for a
    compartment at rest)."""
    rows = []
    for p in params_list:
        dl = [d * p.dt / (p.dx * p.dx) for d in p.d]
        rows.append([p.beta / 0.3 - 1.0, p.alpha / 0.2 - 1.0, p.gamma / 0.11 - 1.0,
                     p.phi / 0.09 - 1.0] + [(math.log10(v) + 3.0) if v > 0 else 0.0 for v in dl])
    return rows


class Surrogate:
    """A trained network plus its input/output scales: advances FP32 states
    [batch][5][h][w] by `jump` SSLBM steps per evaluation."""

    def __init__(self, net: UNet, jump: int, scale_in, scale_out):
        self.net, self.jump = net, int(jump)
        self.scale_in = [float(v) for v in scale_in]
        self.scale_out = [float(v) for v in scale_out]
        self.lib = library()

    def predict(self, rho, planes, out=None):
        torch = _torch()
        b, _, h, w = rho.shape
        self.net._buffers(b, h, w)
        pl = torch.tensor(planes, dtype=torch.float32, device="cuda").contiguous()
        _check(self.lib.sur_pack_input(_ptr(rho), b, h, w, _ptr(pl), _floats(self.scale_in),
                                       _ptr(self.net.x0), None), "sur_pack_input")
        self.net.forward_packed(fuse_up=True)
        if out is None:
            out = torch.empty_like(rho)
        _check(self.lib.sur_apply_output(_ptr(rho), _ptr(self.net.out), b, h, w,
                                         _floats(self.scale_out), _ptr(out), None),
               "sur_apply_output")
        return out


MAX_FOCI = 8


def _foci_states(flat, b, h, w, rng):
    """Fill the ensemble state `flat` (b equal grids) with 1-8 seeded
    Gaussian foci per grid: `inputs.gaussian_foci_state` fields, assembled
    on the device from their separable factors (one small upload instead of
    a full state per grid)."""
    torch = _torch()
    from .inputs import gaussian_foci_factors
    gy = np.zeros((b, MAX_FOCI, h))  # unused foci stay zero
    gx = np.zeros((b, MAX_FOCI, w))
    for k in range(b):
        foci = int(rng.integers(1, MAX_FOCI + 1))
        centres = list(zip(rng.integers(0, w, foci).tolist(), rng.integers(0, h, foci).tolist()))
        amp = float(rng.uniform(0.005, 0.05))
        gy[k, :foci], gx[k, :foci] = gaussian_foci_factors(w, h, centres, amp,
                                                           float(rng.uniform(3, 8)))
    gy_d = torch.tensor(gy.transpose(0, 2, 1).copy(), device="cuda")  # (b, h, foci)
    gx_d = torch.tensor(gx, device="cuda")                               # (b, foci, w)
    infected = torch.bmm(gy_d, gx_d).clamp_(max=1.0)
    x0 = flat.view(b, 5, h, w)  # instance blocks are contiguous (5 h w % 4 == 0)
    x0.zero_()
    x0[:, 0] = 1.0 - infected
    x0[:, 2] = infected


def _generator_launch(params_list, h, w, seed):
    """Pass shape of the data generator's ensemble (b equal grids), tuned
    once on a seeded batch (`Ensemble.tune`)."""
    from .binding import Ensemble
    b = len(params_list)
    ens = Ensemble([(w, h)] * b, params_list, dtype="f32")
    flat = ens.empty()
    _foci_states(flat, b, h, w, np.random.default_rng(seed))
    return ens.tune(flat, ens.empty())


def _ensemble_batch(params_list, h, w, seed, warm, jump, launch=None):
    """States (x_t, x_{t+jump}) of a batch of equal grids from 1-8 seeded
    Gaussian foci after `warm` SSLBM steps, advanced together by the
    library's ensemble kernel (FP32), with pass shape `launch` (a dict as
    from `_generator_launch`; None: the library's default)."""
    from .binding import Ensemble
    b = len(params_list)
    ens = Ensemble([(w, h)] * b, params_list, dtype="f32")
    if launch:
        ens.set_launch(**launch)
    flat = ens.empty()
    _foci_states(flat, b, h, w, np.random.default_rng(seed))
    scratch = ens.empty()
    if warm:
        ens.run(flat, warm, scratch)
    x_t = flat.view(b, 5, h, w).clone()
    ens.run(flat, jump, scratch)
    x_next = flat.view(b, 5, h, w).clone()
    return x_t, x_next


def sample_params(rng, count):
    """Rates and diffusivities of the training distribution: R0 uniform in
    [1.5, 5] through beta = R0 (gamma + mu), sigma = 0.2, gamma = 0.1,
    mu = 0.01, lattice diffusivities of S, E, I, R log-uniform in
    [1e-4, 1e-2], D at rest."""
    from .inputs import from_sigma_mu
    out = []
    for _ in range(count):
        r0 = rng.uniform(1.5, 5.0)
        dl = tuple(np.exp(rng.uniform(np.log(1e-4), np.log(1e-2), 4)).tolist()) + (0.0,)
        out.append(from_sigma_mu(r0 * 0.11, 0.2, 0.1, 0.01, dl))
    return out


@dataclass
class TrainReport:
    steps: int
    batch: int
    seconds: float
    first_loss: float
    last_loss: float
    samples: int
    conv_tflops: float


def train(net: UNet, *, steps=300, batch=16, size=256, jump=50, lr=1e-3, seed=0,
          max_warm=1500, log=None):
    """Train on freshly generated SSLBM pairs; returns (Surrogate, TrainReport)."""
    torch = _torch()
    lib = library()
    rng = np.random.default_rng(seed)
    # scales from probe batches spread over the warm-up range: RMS of each
    # density and of its increment over `jump` steps (with floors, so a
    # compartment that is still empty does not get a vanishing scale)
    sq_in, sq_out = np.zeros(5), np.zeros(5)
    probes = 4
    for j in range(probes):
        plist = sample_params(rng, batch)
        x_t, x_n = _ensemble_batch(plist, size, size, int(rng.integers(1 << 30)),
                                   (j * max_warm) // max(probes - 1, 1), jump)
        for c in range(5):
            sq_in[c] += float(torch.mean(x_t[:, c].double() ** 2)) / probes
            sq_out[c] += float(torch.mean((x_n[:, c] - x_t[:, c]).double() ** 2)) / probes
    scale_in = [max(math.sqrt(v), 1e-3) for v in sq_in]
    scale_out = [max(math.sqrt(v), 1e-5) for v in sq_out]
    sur = Surrogate(net, jump, scale_in, scale_out)
    # the pass shape of the data generator, tuned once for this batch of grids
    launch = _generator_launch(sample_params(rng, batch), size, size, int(rng.integers(1 << 30)))
    partials = torch.empty(1024, dtype=torch.float64, device="cuda")
    loss = torch.zeros(1, dtype=torch.float64, device="cuda")
    losses = []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for it in range(steps):
        plist = sample_params(rng, batch)
        x_t, x_n = _ensemble_batch(plist, size, size, int(rng.integers(1 << 30)),
                                   int(rng.integers(0, max_warm + 1)), jump, launch)
        net._buffers(batch, size, size)
        pl = torch.tensor(param_planes(plist), dtype=torch.float32, device="cuda")
        _check(lib.sur_pack_input(_ptr(x_t), batch, size, size, _ptr(pl), _floats(scale_in),
                                  _ptr(net.x0), None), "sur_pack_input")
        net.forward_packed()
        _check(lib.sur_mse_loss(_ptr(net.out), _ptr(x_t), _ptr(x_n), batch, size, size,
                                _floats(scale_out), _ptr(net.dout), _ptr(partials), _ptr(loss),
                                None), "sur_mse_loss")
        net.backward_packed()
        # cosine decay of the learning rate
        net.adam(lr * 0.5 * (1.0 + math.cos(math.pi * it / max(steps, 1))))
        if it == 0 or it == steps - 1 or (log and it % 50 == 0):
            losses.append((it, float(loss)))
            if log:
                log(f"train step {it}: loss {float(loss):.4e}")
    torch.cuda.synchronize()
    secs = time.perf_counter() - t0
    flops = 3.0 * net.flops(batch, size, size) * steps
    rep = TrainReport(steps, batch, secs, losses[0][1], losses[-1][1], steps * batch,
                      flops / secs / 1e12)
    return sur, rep


# --------------------------------------------------------------- rollout --

@dataclass
class RolloutReport:
    jumps: int
    accepted: int
    fallbacks: int
    seconds: float
    max_check_error: float
    min_check_error: float
    median_check_error: float
    threshold: float
    skipped: int = 0  # jumps taken by plain SSLBM without trying the surrogate
    prefiltered: int = 0  # fallbacks decided by the network on the judge tiles alone


def _rms(t):
    """Root mean square of each compartment of [.., 5, h, w] (FP64, 5 values)."""
    torch = _torch()
    dims = [d for d in range(t.dim()) if d != t.dim() - 3]
    return torch.sqrt(torch.mean(t.double() ** 2, dim=dims))


def relative_l2(a, b):
    """Largest per-compartment relative L2 difference ||a_c - b_c|| / ||b_c||
    of [.., 5, h, w] states (absolute where b_c is zero)."""
    torch = _torch()
    worst = 0.0
    for c in range(5):
        num = float(torch.linalg.vector_norm((a[..., c, :, :] - b[..., c, :, :]).double()))
        den = float(torch.linalg.vector_norm(b[..., c, :, :].double()))
        worst = max(worst, num / den if den > 0 else num)
    return worst


def receptive_radius(levels: int) -> int:
    """Pixels (Chebyshev distance) from an output of the U-Net to the
    farthest input it reads, over every alignment to the pooling grid: a 3x3
    convolution at level l reaches 2^l, a 2x2 pooling into level l 2^(l-1),
    and a nearest-neighbour upsampling nothing beyond the block its pooling
    formed; plus 1 for the last convolution."""
    convs = sum(2 * 2 ** l for l in range(levels)) + sum(2 * 2 ** l for l in range(levels - 1))
    pools = sum(2 ** (l - 1) for l in range(1, levels))
    return convs + pools + 1


class Rollout:
    """Advance one grid to step T in jumps of the surrogate, each judged by
    plain SSLBM recomputed on seeded sub-tiles: a tile of side `tile` is
    cropped with a halo of `jump` cells (the dependence cone of `jump`
    steps), advanced `jump` steps, and its centre compared with the
    surrogate's prediction. The error estimate of a compartment is the RMS
    difference over the tiles divided by the compartment's RMS over the
    whole grid (the larger of the state's and the recomputed tiles'), an
    estimate of the grid-wide relative L2 error of the jump that stays
    defined where a tile holds none of a compartment. A jump whose largest
    estimate exceeds the jump's share of the error budget is redone by plain
    SSLBM from the same state. The budget is `target`, the relative L2 error
    allowed at T; accepted errors can add up, so each of the T / jump jumps
    may spend target / (T / jump). A fixed `threshold` replaces that share
    (an infinite one runs the surrogate alone, unjudged).

    Prefilter: before the network runs on the whole grid, it runs on the
    judge tiles alone, each cropped with a halo that covers the network's
    receptive field and aligned to its pooling grid, so that a tile's centre
    sees the same inputs as in the whole-grid pass (up to the zero padding
    at the edges of a non-periodic whole grid). A jump whose tile-only
    error exceeds `prefilter_margin` times its share is redone by plain
    SSLBM without the whole-grid pass; otherwise the whole-grid prediction
    is judged as above. The prefilter only ever rejects, so it changes
    which jumps are tried, never what is accepted."""

    def __init__(self, sur: Surrogate, params, h: int, w: int, *, tiles=4, tile=64,
                 target=1e-3, threshold=None, seed=0, backoff=True, max_skip=32,
                 prefilter=True, prefilter_margin=4.0):
        from .binding import Ensemble, Solver
        torch = _torch()
        if tile % 16:
            raise ValueError("tile must be a multiple of 16")
        self.sur, self.params, self.h, self.w = sur, params, h, w
        self.tiles, self.tile = tiles, tile
        self.target, self.threshold = target, threshold
        self.backoff, self.max_skip = backoff, max_skip
        self.prefilter, self.prefilter_margin = prefilter, prefilter_margin
        self.rng = np.random.default_rng(seed)
        self.solver = Solver(w, h, params, dtype="f32")
        self.scratch = torch.empty((5, h, w), dtype=torch.float32, device="cuda")
        side = tile + 2 * sur.jump
        self.ens = Ensemble([(side, side)] * tiles, [params] * tiles, dtype="f32")
        self.crops = self.ens.empty()
        self.crop_scratch = self.ens.empty()
        self.pred_crops = torch.empty((tiles, 5, tile, tile), dtype=torch.float32, device="cuda")
        self.planes = param_planes([params])
        # prefilter tiles: side a multiple of 64 (the network's column
        # granule), halo >= the receptive field, (side - tile) / 2 a multiple
        # of 8 (tile corners are multiples of 8: the pooling grid of 4 levels)
        reach = max(receptive_radius(sur.net.levels), sur.jump)
        self.pre_side = -(-(tile + 2 * reach) // 64) * 64
        self.pre_pad = (self.pre_side - tile) // 2
        self.pre_in = torch.empty((tiles, 5, self.pre_side, self.pre_side), dtype=torch.float32,
                                  device="cuda")
        self.pre_out = torch.empty_like(self.pre_in)
        self.pre_planes = param_planes([params] * tiles)
        self.lib = library()

    def _reference(self, state):
        """Seeded tile corners (multiples of 8) and plain SSLBM advanced
        `jump` steps on each tile: (corners, [tiles, 5, tile, tile])."""
        jump, tile = self.sur.jump, self.tile
        side = tile + 2 * jump
        views = self.ens.views(self.crops)
        corners = [(int(self.rng.integers(0, self.h)) // 8 * 8,
                    int(self.rng.integers(0, self.w)) // 8 * 8) for _ in range(self.tiles)]
        for (y0, x0), v in zip(corners, views):
            _check(self.lib.sur_crop_periodic(_ptr(state), self.h, self.w, y0 - jump, x0 - jump,
                                              side, side, _ptr(v), None), "sur_crop_periodic")
        self.ens.run(self.crops, jump, self.crop_scratch)
        torch = _torch()
        ref = torch.stack([v[:, jump:jump + tile, jump:jump + tile] for v in views])
        return corners, ref

    def _error(self, state, pred_tiles, ref):
        torch = _torch()
        scale = torch.maximum(_rms(state), _rms(ref))
        err = _rms(pred_tiles - ref) / scale
        err = torch.where(scale > 0, err, _rms(pred_tiles - ref))
        return float(torch.max(err))

    def _tile_prediction(self, state, corners):
        """The network on the judge tiles alone: centres [tiles, 5, tile, tile]."""
        side, pad, tile = self.pre_side, self.pre_pad, self.tile
        for (y0, x0), v in zip(corners, self.pre_in):
            _check(self.lib.sur_crop_periodic(_ptr(state), self.h, self.w, y0 - pad, x0 - pad,
                                              side, side, _ptr(v), None), "sur_crop_periodic")
        self.sur.predict(self.pre_in, self.pre_planes, out=self.pre_out)
        return self.pre_out[:, :, pad:pad + tile, pad:pad + tile]

    def _judge(self, state, pred, corners, ref):
        tile = self.tile
        for (y0, x0), pc in zip(corners, self.pred_crops):
            _check(self.lib.sur_crop_periodic(_ptr(pred), self.h, self.w, y0, x0, tile, tile,
                                              _ptr(pc), None), "sur_crop_periodic")
        return self._error(state, self.pred_crops, ref)

    def run(self, rho0, T: int):
        """Returns (state at T, RolloutReport); T a multiple of the jump.

        With backoff (the default), a rejected jump makes the next attempt
        wait: after r rejections in a row the following min(2^r, max_skip)
        jumps are taken by plain SSLBM in one run, so a surrogate that keeps
        failing the judge costs a few network passes instead of one per jump."""
        torch = _torch()
        jump = self.sur.jump
        if T % jump:
            raise ValueError(f"T must be a multiple of {jump}")
        state = rho0.clone()
        pred = torch.empty_like(state)
        accepted = fallbacks = skipped = prefiltered = 0
        errs = []
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        share = self.threshold if self.threshold is not None else self.target / (T // jump)
        judged = math.isfinite(share)
        jumps, j, streak = T // jump, 0, 0
        while j < jumps:
            ok = True
            if judged:
                corners, ref = self._reference(state)
                if self.prefilter:
                    pre = self._error(state, self._tile_prediction(state, corners), ref)
                    if pre > self.prefilter_margin * share:
                        errs.append(pre)
                        prefiltered += 1
                        ok = False
            if ok:
                self.sur.predict(state[None], self.planes, out=pred[None])
                err = self._judge(state, pred, corners, ref) if judged else 0.0
                errs.append(err)
                if err <= share:
                    state, pred = pred, state
                    accepted += 1
                    streak = 0
                    j += 1
                    continue
            self.solver.run(state, jump, self.scratch)
            fallbacks += 1
            j += 1
            streak += 1
            if self.backoff:
                skip = min(2 ** streak, self.max_skip, jumps - j)
                if skip > 0:
                    self.solver.run(state, skip * jump, self.scratch)
                    skipped += skip
                    j += skip
        torch.cuda.synchronize()
        secs = time.perf_counter() - t0
        return state, RolloutReport(jumps, accepted, fallbacks, secs, max(errs), min(errs),
                                    float(np.median(errs)), share, skipped, prefiltered)




def _main(argv=None):
    """Time the network's passes (random weights and inputs): forward at
    one batch size, forward + backward at another, on square images.
    `python -m paper_2603_19789_amd.surrogate [--forward-batch 64]
    [--backward-batch 16] [--size 256] [--passes 3]`; prints one line per
    measurement (for kernel traces of the network's layers)."""
    import argparse
    torch = _torch()
    ap = argparse.ArgumentParser(description=_main.__doc__)
    ap.add_argument("--forward-batch", type=int, default=64)
    ap.add_argument("--backward-batch", type=int, default=16)
    ap.add_argument("--size", type=int, default=256)
    ap.add_argument("--passes", type=int, default=3)
    args = ap.parse_args(argv)
    net = UNet(levels=4, base=32, seed=0)
    for batch, backward in ((args.forward_batch, False), (args.backward_batch, True)):
        net._buffers(batch, args.size, args.size)
        net.x0.normal_()
        net.dout.normal_()
        # forward alone as inference runs it; with the backward as training does
        net.forward_packed()
        if backward:
            net.backward_packed()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.passes):
            net.forward_packed()
            if backward:
                net.backward_packed()
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t0) / args.passes * 1e3
        flops = net.flops(batch, args.size, args.size) * (3.0 if backward else 1.0)
        what = "forward + backward" if backward else "forward"
        print(f"{what}, batch {batch} at {args.size}^2: {ms:.3f} ms per pass, "
              f"{flops / ms / 1e9:.1f} TFLOP/s", flush=True)


if __name__ == "__main__":
    _main()
