"""Test-side helpers for driving the HIP library through its C ABI.

Format conversions only (spin packing, buffer allocation); no part of the
method is computed here.
"""
from __future__ import annotations

import sys

import numpy as np
import torch

import paper_2509_19006_amd as T


def say(msg: str):
    print(msg, flush=True)
    sys.stdout.flush()


def pack(spins_list):
    """List (per instance) of (n, L, L) arrays in {-1,+1} -> flat int64 words
    in the library's packed layout (instance, sample, row, word)."""
    out = []
    for s in spins_list:
        s = np.asarray(s)
        n, L, _ = s.shape
        W = (L + 63) // 64
        w = np.zeros((n, L, W), dtype=np.uint64)
        up = (s > 0).astype(np.uint64)
        for c in range(L):
            w[:, :, c // 64] |= up[:, :, c] << np.uint64(c % 64)
        out.append(w.ravel())
    return np.concatenate(out).view(np.int64)


def unpack(words, Ls, n):
    """Inverse of pack: flat words -> list of (n, L, L) int8 arrays."""
    w = np.asarray(words).view(np.uint64)
    out, off = [], 0
    for L in Ls:
        W = (L + 63) // 64
        cnt = n * L * W
        blk = w[off:off + cnt].reshape(n, L, W)
        off += cnt
        s = np.empty((n, L, L), dtype=np.int8)
        for c in range(L):
            s[:, :, c] = np.where((blk[:, :, c // 64] >> np.uint64(c % 64)) & np.uint64(1), 1, -1)
        out.append(s)
    return out


class Run:
    """A batch of instances built on the GPU at one precision."""

    def __init__(self, Js, chi, beta, precision, max_samples=256, flags=0):
        self.Ls = [int(jh.shape[0]) for jh, _ in Js]
        self.B = len(Js)
        self.jh = torch.as_tensor(np.concatenate([np.asarray(jh, np.float32).ravel() for jh, _ in Js])).cuda()
        self.jv = torch.as_tensor(np.concatenate([np.asarray(jv, np.float32).ravel() for _, jv in Js])).cuda()
        self.problem = T.Problem(self.jh, self.jv, self.Ls, chi, beta, flags=flags)
        self.precision = precision
        nbytes = T.tnmc_workspace_size(self.problem, precision, max_samples)
        self.ws = torch.zeros(nbytes, dtype=torch.uint8, device="cuda")
        self.logz_t = torch.zeros(self.B, dtype=torch.float64, device="cuda")
        self.env = T.tnmc_build_env(self.problem, precision, self.ws, self.logz_t)
        torch.cuda.synchronize()

    @property
    def logz(self):
        return self.logz_t.cpu().numpy()

    def words(self, n):
        return n * self.problem.spin_words_per_sample()

    def sample(self, n, seed=0, offset=0, forced=None, logits=False):
        """Returns (spins list, logq (B, n), logits list or None)."""
        spins = torch.zeros(self.words(n), dtype=torch.int64, device="cuda")
        logq = torch.zeros((self.B, n), dtype=torch.float64, device="cuda")
        lg = None
        if logits:
            lg = torch.zeros(n * sum(L * L for L in self.Ls), dtype=torch.float32, device="cuda")
        f = None if forced is None else torch.as_tensor(pack(forced)).cuda()
        T.tnmc_sample(self.env, n, seed, spins, logq, sample_offset=offset, forced_spins=f,
                      logits_out=lg)
        torch.cuda.synchronize()
        sp = unpack(spins.cpu().numpy(), self.Ls, n)
        lgs = None
        if logits:
            h = lg.cpu().numpy()
            lgs, off = [], 0
            for L in self.Ls:
                lgs.append(h[off:off + n * L * L].reshape(n, L, L))
                off += n * L * L
        return sp, logq.cpu().numpy(), lgs

    def energy(self, spins_list):
        n = spins_list[0].shape[0]
        w = torch.as_tensor(pack(spins_list)).cuda()
        E = torch.zeros((self.B, n), dtype=torch.float64, device="cuda")
        T.tnmc_energy(self.env, n, w, E)
        torch.cuda.synchronize()
        return E.cpu().numpy()

    def stats(self):
        return T.tnmc_env_stats(self.env)


def gpu_accept(logq, E, beta, seed, step_offset, chain=None):
    B, n = logq.shape
    lq = torch.as_tensor(np.ascontiguousarray(logq, np.float64)).cuda()
    e = torch.as_tensor(np.ascontiguousarray(E, np.float64)).cuda()
    b = torch.as_tensor(np.ascontiguousarray(np.broadcast_to(beta, (B,)), np.float64)).cuda()
    if chain is None:
        chain = torch.zeros(B * T.CHAIN_BYTES, dtype=torch.uint8, device="cuda")
    acc = torch.zeros((B, n), dtype=torch.uint8, device="cuda")
    st = torch.zeros((B, n), dtype=torch.int64, device="cuda")
    T.tnmc_accept(lq, e, b, chain, seed, step_offset, acc, st)
    torch.cuda.synchronize()
    return acc.cpu().numpy(), st.cpu().numpy(), chain
