"""Seeded synthetic workloads for the line-of-sight projection.

This module builds inputs only: the k and tau grids, their quadrature weights,
the primordial spectrum P(k) and synthetic source functions S_X(k, tau).  It
holds none of the projection arithmetic (no Bessel functions, no sums over
tau or k), so the GPU path and the CPU oracle can both be fed from it.

The paper's own workload (CAMB with Planck-2018 parameters, Sec. 3.1 and
Table 1) needs the full Boltzmann hierarchy to produce source functions; these
synthetic sources stand in for it with the same structure: a visibility-like
peak near recombination, a late broad ISW-like term, an E source carrying k^2,
and a broad lensing kernel.

Grids (both ends included):
* tau_n = n * tau0 / (ntau - 1), n = 0..ntau-1, tau0 = 14000 Mpc
* k_i log-spaced on [kmin, kmax]
* w_tau: trapezoid weights in tau; w_lnk: trapezoid weights in ln k
* P(k) = A_s (k / 0.05)^(n_s - 1)
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional, Tuple

import numpy as np

TAU0 = 14000.0
K_PIVOT = 0.05
PAIRS_TT = ((0, 0),)
PAIRS_4 = ((0, 0), (1, 1), (0, 1), (2, 2))  # TT, EE, TE, phi-phi
PAIR_NAMES_4 = ("TT", "EE", "TE", "PP")


@dataclasses.dataclass
class Workload:
    name: str
    lmin: int
    lmax: int
    k: np.ndarray          # [nk]
    tau: np.ndarray        # [ntau]
    tau0: float
    w_tau: np.ndarray      # [ntau]
    w_lnk: np.ndarray      # [nk]
    Pk: np.ndarray         # [nk]
    S: np.ndarray          # [nsrc, nk, ntau] float64
    pairs: Tuple[Tuple[int, int], ...]
    pair_names: Tuple[str, ...]
    params: Dict[str, float] = dataclasses.field(default_factory=dict)

    @property
    def nk(self) -> int:
        return int(self.k.size)

    @property
    def ntau(self) -> int:
        return int(self.tau.size)

    @property
    def nl(self) -> int:
        return self.lmax - self.lmin + 1

    @property
    def nsrc(self) -> int:
        return int(self.S.shape[0])


def tau_grid(ntau: int, tau0: float = TAU0) -> np.ndarray:
    """Uniform tau nodes on [0, tau0]; the last node is exactly tau0 (so chi = 0 there)."""
    return np.linspace(0.0, tau0, ntau)


def log_k_grid(nk: int, kmin: float, kmax: float) -> np.ndarray:
    return np.exp(np.linspace(np.log(kmin), np.log(kmax), nk))


def trapezoid_weights(nodes: np.ndarray) -> np.ndarray:
    """Trapezoid weights on (possibly non-uniform) nodes: w_0 = h_0/2, w_n = (h_{n-1}+h_n)/2."""
    h = np.diff(nodes)
    w = np.zeros_like(nodes)
    w[:-1] += 0.5 * h
    w[1:] += 0.5 * h
    return w


def primordial(k: np.ndarray, A_s: float, n_s: float) -> np.ndarray:
    return A_s * (k / K_PIVOT) ** (n_s - 1.0)


def gauss(tau: np.ndarray, mu: float, sig: float) -> np.ndarray:
    return np.exp(-((tau - mu) ** 2) / (2.0 * sig * sig))


def lensing_kernel(tau: np.ndarray) -> np.ndarray:
    """Broad kernel sin^2(pi (tau - 2000) / 11500) on [2000, 13500], zero elsewhere."""
    inside = (tau >= 2000.0) & (tau <= 13500.0)
    return np.where(inside, np.sin(np.pi * (tau - 2000.0) / 11500.0) ** 2, 0.0)


def sources(k: np.ndarray, tau: np.ndarray, nsrc: int, tau_star=280.0, width=20.0, a_isw=0.1):
    """Synthetic S[src, k, tau]: T, then E = 0.5 k^2 g(tau), then the lensing kernel."""
    if not 1 <= nsrc <= 3:
        raise ValueError("synthetic sources exist for nsrc = 1..3")
    g = gauss(tau, tau_star, width)[None, :]
    kk = k[:, None]
    S = np.empty((nsrc, k.size, tau.size), dtype=np.float64)
    S[0] = g * (1.0 + 0.3 * np.cos(150.0 * kk)) + a_isw * gauss(tau, 12000.0, 1500.0)[None, :]
    if nsrc > 1:
        S[1] = 0.5 * kk * kk * g
    if nsrc > 2:
        S[2] = np.broadcast_to(lensing_kernel(tau)[None, :], (k.size, tau.size))
    return S


def _make(name, lmax, nk, kmax, ntau, nsrc, kmin=1e-4, A_s=2.1e-9, n_s=0.965, **src_kw):
    k = log_k_grid(nk, kmin, kmax)
    tau = tau_grid(ntau)
    keep = [i for i, (a, b) in enumerate(PAIRS_4) if a < nsrc and b < nsrc]
    pairs = tuple(PAIRS_4[i] for i in keep)
    names = tuple(PAIR_NAMES_4[i] for i in keep)
    return Workload(name=name, lmin=2, lmax=lmax, k=k, tau=tau, tau0=TAU0,
                    w_tau=trapezoid_weights(tau), w_lnk=trapezoid_weights(np.log(k)),
                    Pk=primordial(k, A_s, n_s), S=sources(k, tau, nsrc, **src_kw),
                    pairs=pairs, pair_names=names, params=dict(A_s=A_s, n_s=n_s, **src_kw))


# The five benchmark configurations (the first three are single-model solves).
CONFIGS = {
    # plain FP64, one model, temperature only
    "C1": dict(lmax=300, nk=400, kmax=0.05, ntau=600, nsrc=1),
    # plain FP64 high accuracy, T/E/lensing
    "C2": dict(lmax=2500, nk=4000, kmax=0.5, ntau=3000, nsrc=3),
    # mixed-precision case
    "C3": dict(lmax=5000, nk=8000, kmax=1.0, ntau=4000, nsrc=3),
}

DESCRIPTIONS = {
    "C1": "TT, l=2..300, 400 log-k on [1e-4,0.05], 600 tau on [0,14000]",
    "C2": "TT/EE/TE/PP, l=2..2500, 4000 log-k on [1e-4,0.5], 3000 tau on [0,14000]",
    "C3": "TT/EE/TE/PP, l=2..5000, 8000 log-k on [1e-4,1.0], 4000 tau on [0,14000]",
    "C4": "256 drawn models, TT/EE/TE/PP, l_max in [1500,5000], 2000..8000 of the 8000 master "
          "log-k on [1e-4,1.0], 3000 tau on [0,14000]",
    "T2": "tensor modes TT/EE/BB/TE, l=2..1500, 2000 log-k on [1e-4,3000/14000], "
          "3000 tau on [0,14000]",
}


def config(name: str) -> Workload:
    c = CONFIGS[name]
    return _make(name, **c)


# Sources on a coarse wavenumber grid (the grid the perturbation equations are
# evolved on), to be interpolated in k onto the workload's own k grid: nkc
# log-spaced knots spanning the same [kmin, kmax].
COARSE_NK = {"C1": 100, "C2": 1000, "C3": 2000}


@dataclasses.dataclass
class CoarseSources:
    q: np.ndarray    # [nkc] knots, strictly increasing, q[0] = k[0], q[-1] = k[-1]
    Sc: np.ndarray   # [nsrc, nkc, ntau] float64, the synthetic sources at the knots


def coarse_sources(wl: Workload, nkc: int) -> CoarseSources:
    """The workload's synthetic sources evaluated on nkc log-spaced knots over its k range."""
    q = log_k_grid(nkc, float(wl.k[0]), float(wl.k[-1]))
    kw = {key: wl.params[key] for key in ("tau_star", "width", "a_isw") if key in wl.params}
    return CoarseSources(q=q, Sc=sources(q, wl.tau, wl.nsrc, **kw))


def l_samples(lmin: int, lmax: int, boost: float = 1.0) -> np.ndarray:
    """Multipoles computed explicitly at an output sampling density `boost`: from lmin,
    steps of round(0.1 l / boost) clipped to [1, max(1, round(50 / boost))], always
    ending at lmax.  boost = 50 (or any boost >= 50) samples every l."""
    if lmax < lmin:
        raise ValueError("lmax < lmin")
    cap = max(1, int(round(50.0 / boost)))
    out = [lmin]
    while out[-1] < lmax:
        step = min(max(1, int(round(0.1 * out[-1] / boost))), cap)
        out.append(min(out[-1] + step, lmax))
    return np.asarray(out, dtype=np.int32)


def small(lmax=40, nk=24, kmax=0.02, ntau=200, nsrc=3, kmin=1e-4, **kw) -> Workload:
    """A small workload of the same structure (for quick parity tests)."""
    return _make("small", lmax=lmax, nk=nk, kmax=kmax, ntau=ntau, nsrc=nsrc, kmin=kmin, **kw)


# --- tensor modes ---------------------------------------------------------------------------
#
# The tensor line-of-sight call projects a temperature source S_T and a
# polarisation source S_P (both from gravitational waves) on the tensor
# kernels; its spectra are TT, EE, BB and TE.  The paper's runs use
# l_max_tensor = 1500 and k eta_max = 3000 for tensors (Sec. 3.1), i.e. k up to
# 3000 / tau0.  Synthetic sources of the same structure: S_T an ISW-like term
# of a wave that decays after horizon entry (k tau > 1) plus a small
# recombination term, S_P a visibility peak times a wave amplitude that falls
# off for modes inside the horizon at recombination.
PAIRS_TENSOR = ((0, 0), (1, 1), (2, 2), (0, 1))  # TT, EE, BB, TE over (T, E, B)
PAIR_NAMES_TENSOR = ("TT", "EE", "BB", "TE")
TENSOR_R = 0.1


def tensor_sources(k: np.ndarray, tau: np.ndarray, tau_star=280.0, width=20.0) -> np.ndarray:
    """Synthetic tensor sources S[2, k, tau]: S_T, then S_P."""
    kk = k[:, None]
    kt = kk * tau[None, :]
    g = gauss(tau, tau_star, width)[None, :]
    S = np.empty((2, k.size, tau.size), dtype=np.float64)
    S[0] = kk * np.sin(kt) / (1.0 + kt * kt) + 0.05 * g * np.cos(150.0 * kk)
    S[1] = 0.5 * g * (1.0 + 0.3 * np.cos(150.0 * kk)) / (1.0 + (kk * tau_star) ** 2)
    return S


def tensor_workload(lmax=1500, nk=2000, kmax=3000.0 / TAU0, ntau=3000, kmin=1e-4,
                    A_s=2.1e-9, r=TENSOR_R, name="T2") -> Workload:
    """Tensor projection workload: l = 2..lmax, nk log-k on [kmin, kmax], ntau tau nodes;
    P_t(k) = r A_s (k / 0.05)^(-r/8) (the consistency-relation tilt)."""
    k = log_k_grid(nk, kmin, kmax)
    tau = tau_grid(ntau)
    return Workload(name=name, lmin=2, lmax=lmax, k=k, tau=tau, tau0=TAU0,
                    w_tau=trapezoid_weights(tau), w_lnk=trapezoid_weights(np.log(k)),
                    Pk=primordial(k, r * A_s, 1.0 - r / 8.0), S=tensor_sources(k, tau),
                    pairs=PAIRS_TENSOR, pair_names=PAIR_NAMES_TENSOR,
                    params=dict(A_s=A_s, r=r))


# --- batched configuration: per-model parameter draws -------------------------------------

BATCH_SEED = 20250925
MASTER_NK = 8000
MASTER_KMAX = 1.0


@dataclasses.dataclass
class ModelDraw:
    lmax: int
    nk: int
    tau_star: float
    width: float
    a_isw: float
    n_s: float
    ln1e10As: float

    @property
    def A_s(self) -> float:
        return float(np.exp(self.ln1e10As) * 1e-10)


def draw_models(n: int, seed: int = BATCH_SEED, lmax_range=(1500, 5000), nk_range=(2000, 8000)):
    """Per-model draws, in this order for each model: lmax, nk, tau*, width, ISW amp, n_s, ln(1e10 A_s)."""
    rng = np.random.default_rng(seed)
    out: List[ModelDraw] = []
    for _ in range(n):
        lmax = int(rng.integers(lmax_range[0], lmax_range[1] + 1))
        nk = int(rng.integers(nk_range[0], nk_range[1] + 1))
        out.append(ModelDraw(lmax=lmax, nk=nk, tau_star=float(rng.uniform(260.0, 300.0)),
                             width=float(rng.uniform(15.0, 25.0)), a_isw=float(rng.uniform(0.0, 0.2)),
                             n_s=float(rng.uniform(0.92, 1.0)),
                             ln1e10As=float(rng.uniform(2.9, 3.2))))
    return out


def master_indices(nk_model: int, master_nk: int = MASTER_NK) -> np.ndarray:
    """Model k-grid as a subset of the shared master grid: round(j (M-1)/(n-1))."""
    j = np.arange(nk_model, dtype=np.float64)
    return np.rint(j * (master_nk - 1) / (nk_model - 1)).astype(np.int64)


def model_workload(d: ModelDraw, ntau: int = 3000, master_nk: int = MASTER_NK,
                   master_kmax: float = MASTER_KMAX, kmin: float = 1e-4) -> Workload:
    """One drawn model as a stand-alone workload on its own subset of the master k grid."""
    kmaster = log_k_grid(master_nk, kmin, master_kmax)
    idx = master_indices(d.nk, master_nk)
    k = kmaster[idx]
    tau = tau_grid(ntau)
    return Workload(name="model", lmin=2, lmax=d.lmax, k=k, tau=tau, tau0=TAU0,
                    w_tau=trapezoid_weights(tau), w_lnk=trapezoid_weights(np.log(k)),
                    Pk=primordial(k, d.A_s, d.n_s),
                    S=sources(k, tau, 3, tau_star=d.tau_star, width=d.width, a_isw=d.a_isw),
                    pairs=PAIRS_4, pair_names=PAIR_NAMES_4,
                    params=dict(A_s=d.A_s, n_s=d.n_s, tau_star=d.tau_star, width=d.width,
                                a_isw=d.a_isw))


@dataclasses.dataclass
class BatchInputs:
    """A batch of drawn models on one shared master k grid (host arrays)."""
    draws: List[ModelDraw]
    k_master: np.ndarray   # [nk_master]
    tau: np.ndarray        # [ntau]
    tau0: float
    w_tau: np.ndarray      # [ntau]
    lmax: np.ndarray       # [nmodels] int32
    koff: np.ndarray       # [nmodels + 1] int64
    k_index: np.ndarray    # [koff[-1]] int64, master row of each (model, j)
    w_lnk: np.ndarray      # [koff[-1]] each model's own ln k trapezoid weights
    Pk: np.ndarray         # [koff[-1]] each model's A_s (k / k_pivot)^(n_s - 1)
    pairs: Tuple[Tuple[int, int], ...] = PAIRS_4

    @property
    def nmodels(self) -> int:
        return len(self.draws)

    @property
    def ntau(self) -> int:
        return int(self.tau.size)


def batch_inputs(draws: List[ModelDraw], ntau: int = 3000, master_nk: int = MASTER_NK,
                 master_kmax: float = MASTER_KMAX, kmin: float = 1e-4) -> BatchInputs:
    kmaster = log_k_grid(master_nk, kmin, master_kmax)
    tau = tau_grid(ntau)
    koff = [0]
    idx, wl, pk = [], [], []
    for d in draws:
        i = master_indices(d.nk, master_nk)
        k = kmaster[i]
        idx.append(i)
        wl.append(trapezoid_weights(np.log(k)))
        pk.append(primordial(k, d.A_s, d.n_s))
        koff.append(koff[-1] + i.size)
    return BatchInputs(draws=list(draws), k_master=kmaster, tau=tau, tau0=TAU0,
                       w_tau=trapezoid_weights(tau),
                       lmax=np.array([d.lmax for d in draws], dtype=np.int32),
                       koff=np.array(koff, dtype=np.int64), k_index=np.concatenate(idx),
                       w_lnk=np.concatenate(wl), Pk=np.concatenate(pk))


def batch_sources_host(b: BatchInputs, col: np.ndarray, ncols: int) -> np.ndarray:
    """S_packed[ncols, ntau] float32: row col[koff[m] + j] + s holds source s of model m at its
    j-th k (the layout a batch plan reports)."""
    S = np.zeros((ncols, b.ntau), dtype=np.float32)
    for m, d in enumerate(b.draws):
        lo, hi = b.koff[m], b.koff[m + 1]
        k = b.k_master[b.k_index[lo:hi]]
        Sm = sources(k, b.tau, 3, tau_star=d.tau_star, width=d.width, a_isw=d.a_isw)
        for s in range(3):
            S[col[lo:hi] + s] = Sm[s]
    return S


def batch_sources_device(b: BatchInputs, col: np.ndarray, S_packed, torch,
                         sources=(0, 1, 2)) -> None:
    """The same values as batch_sources_host, generated model by model on the device into the
    float32 tensor S_packed[ncols, ntau] (the full 256-model batch does not fit host memory
    comfortably).  Same formulas as `sources`, evaluated by torch in float64.  `sources` lists
    the source planes of the plan in order (0 T, 1 E, 2 lensing): (0,) fills a plan made for
    the temperature source alone (pairs [(0, 0)])."""
    dev = S_packed.device
    tau = torch.from_numpy(b.tau).to(dev)
    lens = torch.from_numpy(lensing_kernel(b.tau)).to(dev)
    late = torch.exp(-((tau - 12000.0) ** 2) / (2.0 * 1500.0 ** 2))
    for m, d in enumerate(b.draws):
        lo, hi = int(b.koff[m]), int(b.koff[m + 1])
        k = torch.from_numpy(b.k_master[b.k_index[lo:hi]]).to(dev)[:, None]
        g = torch.exp(-((tau - d.tau_star) ** 2) / (2.0 * d.width * d.width))[None, :]
        rows = torch.from_numpy(col[lo:hi]).to(dev)
        for plane, src in enumerate(sources):
            if src == 0:
                v = g * (1.0 + 0.3 * torch.cos(150.0 * k)) + d.a_isw * late[None, :]
            elif src == 1:
                v = 0.5 * k * k * g
            else:
                v = lens[None, :].expand(hi - lo, -1)
            S_packed[rows + plane] = v.float()


def model_sources_device(wl: Workload, torch, device="cuda"):
    """The sources S[3, nk, ntau] float64 of a drawn model's workload (model_workload(d,
    ...) built with S omitted is enough: k, tau and the draw's parameters), evaluated by torch
    on the device with the formulas of `sources` (host generation of a full-grid model is
    slow)."""
    p = wl.params
    tau = torch.from_numpy(wl.tau).to(device)
    k = torch.from_numpy(wl.k).to(device)[:, None]
    g = torch.exp(-((tau - p["tau_star"]) ** 2) / (2.0 * p["width"] * p["width"]))[None, :]
    late = torch.exp(-((tau - 12000.0) ** 2) / (2.0 * 1500.0 ** 2))[None, :]
    S = torch.empty((3, wl.k.size, wl.tau.size), dtype=torch.float64, device=device)
    S[0] = g * (1.0 + 0.3 * torch.cos(150.0 * k)) + p["a_isw"] * late
    S[1] = 0.5 * k * k * g
    S[2] = torch.from_numpy(lensing_kernel(wl.tau)).to(device)[None, :]
    return S


def model_grid(d: ModelDraw, ntau: int = 3000, master_nk: int = MASTER_NK,
               master_kmax: float = MASTER_KMAX, kmin: float = 1e-4) -> Workload:
    """model_workload without the host sources (S is None): grids, weights and P(k)."""
    kmaster = log_k_grid(master_nk, kmin, master_kmax)
    k = kmaster[master_indices(d.nk, master_nk)]
    tau = tau_grid(ntau)
    return Workload(name="model", lmin=2, lmax=d.lmax, k=k, tau=tau, tau0=TAU0,
                    w_tau=trapezoid_weights(tau), w_lnk=trapezoid_weights(np.log(k)),
                    Pk=primordial(k, d.A_s, d.n_s), S=None, pairs=PAIRS_4,
                    pair_names=PAIR_NAMES_4,
                    params=dict(A_s=d.A_s, n_s=d.n_s, tau_star=d.tau_star, width=d.width,
                                a_isw=d.a_isw))
