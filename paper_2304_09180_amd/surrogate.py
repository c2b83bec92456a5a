"""Training of the learned reaction step on the GPU.

Pipeline (every numeric step runs in the library's HIP kernels; torch only holds
device buffers and the stream):
  1. run the plain solver on 2-D channel workloads and collect reaction-step states
     (14 species, ADP, eta, H_adh) of every cell at several times;
  2. sample training rows (half from cells with bound platelets, where reactions
     act, half uniformly), each with a log-uniform Dt in [5e-6, 1e-3] s (the larger
     steps are where a two-stage increment departs from RK4);
  3. label each row with the plain FP64 RK4 increment (clot_rxn_rk4_batch);
  4. choose the feature/target scales from the sums of squares (clot_surr_dataset),
     build bf16 features and f32 targets;
  5. train the BF16-MFMA MLP with the library's forward, MSE, backward and Adam
     kernels;
  6. return the float32 blob for clot_set_reaction_mode.
"""
from __future__ import annotations

import math

import numpy as np

from . import clot

ROW = 18
NSP = 14


def collect_states(descs_steps, precision=clot.FP32_MIXED, snapshots=5, log=print):
    """Reaction-step states of every cell of each workload at `snapshots` times."""
    import clot_inputs as ci
    rows = []
    for d, steps in descs_steps:
        s = clot.Solver([d], precision)
        xc, xf = ci.noise(d)
        s.init_state(0, xc, xf)
        hadh = s.get(0, "HADH")
        per = max(1, steps // snapshots)
        done = 0
        while done < steps:
            k = min(per, steps - done)
            s.step(k)
            done += k
            f = s.fields(0)
            sp = np.stack([f[n] for n in ("PMU", "PMA", "PBA", "PBSE", "S1", "S2", "E1", "E2",
                                           "S1B", "S2B", "E1B", "E2B", "C1", "C2")], axis=1)
            r = np.zeros((sp.shape[0], ROW))
            r[:, :NSP] = sp
            r[:, 14] = f["ADP"]
            r[:, 15] = f["ETA"]
            r[:, 16] = hadh
            r[:, 17] = d["dt"]
            rows.append(r)
        log(f"# collected {d['nx']}x{d['ny']}x{d['nz']} after {steps} steps")
        s.close()
    return np.concatenate(rows, axis=0)


def sample_rows(states, n, seed=7, dt_range=(5e-6, 1e-3)):
    rng = np.random.default_rng(seed)
    active = np.nonzero(states[:, 3] + states[:, 2] > 0)[0]
    n_act = min(n // 2, 10 * max(len(active), 1)) if len(active) else 0
    idx = np.concatenate([rng.choice(active, n_act) if n_act else np.zeros(0, int),
                          rng.integers(0, states.shape[0], n - n_act)])
    rows = states[idx].copy()
    rows[:, 17] = np.exp(rng.uniform(math.log(dt_range[0]), math.log(dt_range[1]), n))
    return rows


class Trainer:
    """Holds the device buffers of one training run."""

    def __init__(self, rows_np, params=None, seed=7, log=print):
        import torch
        self.torch = torch
        self.lib = clot.load()
        self.log = log
        self.p = params if params is not None else clot.default_params(clot.FP64)
        self.stream = torch.cuda.current_stream()
        sp = clot.ptr
        st = clot.C.c_void_p(self.stream.cuda_stream)
        self.st = st
        n = rows_np.shape[0]
        self.n = n
        dev = "cuda"
        self.rows = torch.from_numpy(np.ascontiguousarray(rows_np)).to(dev)
        self.inc = torch.empty((n, NSP), dtype=torch.float64, device=dev)
        clot.check(self.lib.clot_rxn_rk4_batch(clot.C.byref(self.p), sp(self.rows), n, sp(self.inc), st), "rk4 batch")
        nblk = (n + 255) // 256
        stats = torch.empty((nblk, 42), dtype=torch.float64, device=dev)
        clot.check(self.lib.clot_surr_dataset(clot.C.byref(self.p), sp(self.rows), sp(self.inc), n, None, None, None,
                                              sp(stats), st), "dataset stats")
        tot = stats.sum(0).cpu().numpy()
        sf = np.sqrt(tot[:NSP] / n)
        cnt = np.maximum(tot[2 * NSP:], 1.0)
        sc = np.sqrt(tot[NSP:2 * NSP] / cnt)
        self.scales = np.concatenate([np.where(sf > 1e-30, sf, 1.0), np.where(sc > 1e-30, sc, 1.0)]).astype(np.float32)
        self.sc_t = torch.from_numpy(self.scales).to(dev)
        self.x = torch.empty((n, 32), dtype=torch.int16, device=dev)
        self.t = torch.empty((n, 16), dtype=torch.float32, device=dev)
        clot.check(self.lib.clot_surr_dataset(clot.C.byref(self.p), sp(self.rows), sp(self.inc), n, sp(self.sc_t),
                                              sp(self.x), sp(self.t), None, st), "dataset")
        npar = int(self.lib.clot_mlp_nparam())
        self.npar = npar
        g = torch.Generator().manual_seed(seed)
        w = torch.zeros(npar, dtype=torch.float32)
        # Glorot-uniform weights, zero biases; the last layer starts at zero (explicit increment)
        offs = [(0, 64, 32), (64 * 32 + 64, 64, 64)]
        for off, fo, fi in offs:
            a = math.sqrt(6.0 / (fi + fo))
            w[off:off + fo * fi] = (torch.rand(fo * fi, generator=g) * 2 - 1) * a
        self.wf = w.to(dev)
        self.wb = torch.empty(npar, dtype=torch.int16, device=dev)
        self.m = torch.zeros(npar, dtype=torch.float32, device=dev)
        self.v = torch.zeros(npar, dtype=torch.float32, device=dev)
        self.grad = torch.empty(npar, dtype=torch.float32, device=dev)
        self._refresh_bf16()
        self.step_t = 0

    def _refresh_bf16(self):
        # the Adam kernel keeps the bf16 copy current; at start round the master once
        # (a zero-learning-rate Adam step with zero gradient does exactly that)
        z = self.torch.zeros_like(self.wf)
        m = self.torch.zeros_like(self.wf)
        v = self.torch.zeros_like(self.wf)
        clot.check(self.lib.clot_mlp_adam(clot.ptr(self.wf), clot.ptr(self.wb), clot.ptr(z), clot.ptr(m), clot.ptr(v), 1,
                                          0.0, 0.9, 0.999, 1e-8, self.st), "bf16 copy")

    def loss(self, idx=None, batch=65536):
        """Mean squared error of the scaled corrections over the set (or a slice)."""
        torch = self.torch
        sp = clot.ptr
        n = self.n if idx is None else len(idx)
        tot = 0.0
        for b0 in range(0, n, batch):
            sl = slice(b0, min(n, b0 + batch)) if idx is None else idx[b0:b0 + batch]
            x = self.x[sl].contiguous()
            t = self.t[sl].contiguous()
            nb = x.shape[0]
            y = torch.empty((nb, 16), dtype=torch.float32, device=x.device)
            dy = torch.empty_like(y)
            lp = torch.empty((nb + 255) // 256, dtype=torch.float64, device=x.device)
            clot.check(self.lib.clot_mlp_forward(sp(self.wf), sp(self.wb), sp(x), nb, sp(y), None, self.st), "fwd")
            clot.check(self.lib.clot_mlp_mse(sp(y), sp(t), nb, NSP, sp(dy), sp(lp), self.st), "mse")
            tot += float(lp.sum())
        return tot / (n * NSP)

    def train(self, epochs=20, batch=8192, lr=2e-3, seed=7):
        torch = self.torch
        sp = clot.ptr
        gen = torch.Generator(device="cuda").manual_seed(seed)
        n = self.n
        y = torch.empty((batch, 16), dtype=torch.float32, device="cuda")
        dy = torch.empty_like(y)
        cache = torch.empty((batch, 128), dtype=torch.int16, device="cuda")
        part = torch.empty(int(self.lib.clot_mlp_backward_workspace(batch)) // 4, dtype=torch.float32, device="cuda")
        lp = torch.empty((batch + 255) // 256, dtype=torch.float64, device="cuda")
        hist = []
        for ep in range(epochs):
            perm = torch.randperm(n, device="cuda", generator=gen)
            lr_ep = lr * 0.5 * (1 + math.cos(math.pi * ep / epochs))
            for b0 in range(0, n - batch + 1, batch):
                idx = perm[b0:b0 + batch]
                x = self.x[idx].contiguous()
                t = self.t[idx].contiguous()
                clot.check(self.lib.clot_mlp_forward(sp(self.wf), sp(self.wb), sp(x), batch, sp(y), sp(cache), self.st),
                           "fwd")
                clot.check(self.lib.clot_mlp_mse(sp(y), sp(t), batch, NSP, sp(dy), sp(lp), self.st), "mse")
                clot.check(self.lib.clot_mlp_backward(sp(self.wf), sp(self.wb), sp(x), sp(cache), sp(dy), batch, sp(part),
                                                      sp(self.grad), self.st), "bwd")
                self.step_t += 1
                clot.check(self.lib.clot_mlp_adam(sp(self.wf), sp(self.wb), sp(self.grad), sp(self.m), sp(self.v),
                                                  self.step_t, lr_ep, 0.9, 0.999, 1e-8, self.st), "adam")
            l = self.loss(idx=torch.arange(min(n, 65536), device="cuda"))
            hist.append(l)
            self.log(f"# epoch {ep + 1}/{epochs}: loss {l:.4e}")
        return hist

    def heldout_gain(self, rows_np):
        """Mean squared target over held-out rows with the trained network and with a
        zero network, in the units of this training set: the second is the midpoint
        increment's error vs RK4, the first what the network leaves of it."""
        other = Trainer.__new__(Trainer)
        other.__dict__.update(self.__dict__)
        torch = self.torch
        sp = clot.ptr
        n = rows_np.shape[0]
        rows = torch.from_numpy(np.ascontiguousarray(rows_np)).cuda()
        inc = torch.empty((n, NSP), dtype=torch.float64, device="cuda")
        clot.check(self.lib.clot_rxn_rk4_batch(clot.C.byref(self.p), sp(rows), n, sp(inc), self.st), "rk4 batch")
        other.x = torch.empty((n, 32), dtype=torch.int16, device="cuda")
        other.t = torch.empty((n, 16), dtype=torch.float32, device="cuda")
        other.n = n
        clot.check(self.lib.clot_surr_dataset(clot.C.byref(self.p), sp(rows), sp(inc), n, sp(self.sc_t), sp(other.x),
                                              sp(other.t), None, self.st), "dataset")
        trained = other.loss()
        zero = float((other.t[:, :NSP].double() ** 2).mean())
        return trained, zero

    def blob(self):
        return np.concatenate([self.wf.cpu().numpy().astype(np.float32), self.scales.astype(np.float32)])

    def zero_blob(self):
        """The same scales with a zero network: the explicit increment Dt R(y) alone."""
        return np.concatenate([np.zeros(self.npar, np.float32), self.scales.astype(np.float32)])


def default_training_states(log=print):
    """States from the two 2-D workloads over their whole horizons: the 64x16 channel
    (100 steps at 1e-4 s) and the 1024x256 channel (1000 steps at 1e-5 s)."""
    import clot_inputs as ci
    d1 = ci.workload("channel2d_64x16")
    d2 = ci.workload("channel2d_1024x256")
    return collect_states([(d1, d1["steps"]), (d2, d2["steps"])], log=log)


def train_default(n_samples=1_000_000, epochs=12, log=print):
    states = default_training_states(log=log)
    rows = sample_rows(states, n_samples)
    tr = Trainer(rows, log=log)
    l0 = tr.loss()
    hist = tr.train(epochs=epochs)
    log(f"# surrogate training: loss {l0:.4e} -> {hist[-1]:.4e} on {n_samples} samples")
    return tr
