"""Seeded synthetic inputs shaped like the paper's workloads.

Holds no arithmetic of the method itself: only particle counts, energies,
directions, weights and cell parameters drawn from stated distributions.
Every generator takes a numpy ``Generator`` (PCG64) or a seed and returns a
``Workload`` of host numpy arrays; ``Workload.to_torch(device)`` moves it to
a device.  Both the oracle-side tests and the HIP path consume the same
arrays.

Units: momenta in m_e c, densities in m^-3, temperatures in eV, dt in s.
Weights are in density units (the density of a species in a cell is the sum
of its weights).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, Optional

import numpy as np

MEC2_MEV = 0.51099895000
PROC_BREMS, PROC_BH, PROC_TRIDENT = 1, 2, 4


@dataclasses.dataclass
class Workload:
    name: str
    Z: int
    dt: float
    processes: int
    steps: int
    cells: Dict[str, np.ndarray]        # Zstar, n_i, T_e
    electrons: Dict[str, np.ndarray]    # off, count(None), px, py, pz, w
    photons: Dict[str, np.ndarray]      # off (capacity), count, px, py, pz, w, parent
    ions: Dict[str, np.ndarray]         # off, count(None), w
    new_el: Dict[str, np.ndarray]       # off (capacity), count, px, py, pz, w, parent
    new_po: Dict[str, np.ndarray]
    seed: int = 1

    @property
    def n_cells(self) -> int:
        return len(self.cells["Zstar"])

    def copy(self) -> "Workload":
        def cp(d):
            return {k: (None if v is None else np.array(v, copy=True)) for k, v in d.items()}
        return dataclasses.replace(self, cells=cp(self.cells), electrons=cp(self.electrons),
                                   photons=cp(self.photons), ions=cp(self.ions),
                                   new_el=cp(self.new_el), new_po=cp(self.new_po))

    def to_torch(self, device):
        import torch

        def tt(d):
            return {k: (None if v is None else torch.from_numpy(np.ascontiguousarray(v)).to(device))
                    for k, v in d.items()}
        return dataclasses.replace(self, cells=tt(self.cells), electrons=tt(self.electrons),
                                   photons=tt(self.photons), ions=tt(self.ions),
                                   new_el=tt(self.new_el), new_po=tt(self.new_po))

    def host_subset(self, cells_idx) -> "Workload":
        """The given cells of a workload held in device tensors, copied to a
        host workload of numpy arrays (global ids in cells['cell_id']);
        only those cells' ranges are read from the device."""
        import torch
        idx = np.asarray(cells_idx, dtype=np.int64)

        def sub(d):
            off = d["off"].cpu().numpy()
            starts, ends = off[idx], off[idx + 1]
            new_off = np.zeros(len(idx) + 1, dtype=np.int64)
            np.cumsum(ends - starts, out=new_off[1:])
            take = np.concatenate([np.arange(a, b) for a, b in zip(starts, ends)]) if len(idx) else np.zeros(0, np.int64)
            out = {"off": new_off}
            for k, v in d.items():
                if k == "off":
                    continue
                if v is None:
                    out[k] = None
                elif k == "count":
                    out[k] = np.ascontiguousarray(v.cpu().numpy()[idx])
                else:
                    t = torch.from_numpy(take).to(v.device)
                    out[k] = np.ascontiguousarray(v.index_select(0, t).cpu().numpy())
            return out
        cells = {k: np.ascontiguousarray(v.cpu().numpy()[idx]) for k, v in self.cells.items() if k != "cell_id"}
        base_id = self.cells.get("cell_id")
        cells["cell_id"] = idx.copy() if base_id is None else np.ascontiguousarray(base_id.cpu().numpy()[idx])
        return dataclasses.replace(self, name=self.name + "-subset", cells=cells,
                                   electrons=sub(self.electrons), photons=sub(self.photons),
                                   ions=sub(self.ions), new_el=sub(self.new_el), new_po=sub(self.new_po))

    def subset(self, cells_idx) -> "Workload":
        """The given cells (global ids kept in cells['cell_id']) as a new workload."""
        idx = np.asarray(cells_idx, dtype=np.int64)

        def sub(d, live_key=None):
            off = d["off"]
            starts, ends = off[idx], off[idx + 1]
            lens = ends - starts
            new_off = np.zeros(len(idx) + 1, dtype=np.int64)
            np.cumsum(lens, out=new_off[1:])
            take = np.concatenate([np.arange(s, e) for s, e in zip(starts, ends)]) if len(idx) else np.zeros(0, np.int64)
            out = {"off": new_off}
            for k, v in d.items():
                if k == "off":
                    continue
                if v is None:
                    out[k] = None
                elif k == "count":
                    out[k] = np.ascontiguousarray(v[idx])
                else:
                    out[k] = np.ascontiguousarray(v[take])
            return out
        cells = {k: np.ascontiguousarray(v[idx]) for k, v in self.cells.items() if k != "cell_id"}
        base_id = self.cells.get("cell_id")
        cells["cell_id"] = idx.copy() if base_id is None else np.ascontiguousarray(base_id[idx])
        return dataclasses.replace(self, name=self.name + "-subset", cells=cells,
                                   electrons=sub(self.electrons), photons=sub(self.photons),
                                   ions=sub(self.ions), new_el=sub(self.new_el),
                                   new_po=sub(self.new_po))


# ------------------------------------------------------------------ helpers
def _offsets(counts):
    off = np.zeros(len(counts) + 1, dtype=np.int64)
    np.cumsum(np.asarray(counts, dtype=np.int64), out=off[1:])
    return off


def isotropic(rng, n):
    """Unit vectors, uniform on the sphere."""
    mu = rng.uniform(-1.0, 1.0, n)
    phi = rng.uniform(0.0, 2.0 * math.pi, n)
    s = np.sqrt(np.maximum(0.0, 1.0 - mu * mu))
    return np.stack([s * np.cos(phi), s * np.sin(phi), mu])


def momenta_from_gamma(rng, gamma):
    p = np.sqrt(np.maximum(gamma * gamma - 1.0, 0.0))
    u = isotropic(rng, len(gamma))
    return p * u[0], p * u[1], p * u[2]


def log_uniform(rng, lo, hi, n):
    return np.exp(rng.uniform(math.log(lo), math.log(hi), n))


def power_law_counts(rng, n, alpha, lo, hi):
    """floor of a power law x^-alpha on [lo, hi] (inverse CDF)."""
    u = rng.uniform(0.0, 1.0, n)
    a1 = 1.0 - alpha
    x = (lo ** a1 + u * (hi ** a1 - lo ** a1)) ** (1.0 / a1)
    return np.clip(np.floor(x).astype(np.int64), lo, hi)


def maxwell_juttner_table(theta, grid=200000):
    """Lorentz factors g and the cumulative distribution of
    f ~ gamma^2 beta exp(-gamma/theta) (isotropic relativistic Maxwellian)
    at them, on a fine grid (trapezoid rule): the inverse-CDF table of the
    samplers below."""
    g = 1.0 + np.linspace(0.0, 60.0 * theta + 40.0, grid) ** 1.0
    g = np.concatenate([1.0 + np.geomspace(1e-9, 1e-2, 2000), g[g > 1.0 + 1e-2]])
    pdf = g * np.sqrt(g * g - 1.0) * np.exp(-(g - 1.0) / theta)
    cdf = np.concatenate([[0.0], np.cumsum(0.5 * (pdf[1:] + pdf[:-1]) * np.diff(g))])
    cdf /= cdf[-1]
    return g, cdf


def maxwell_juttner_gamma(rng, n, theta, grid=200000):
    """Lorentz factors from f ~ gamma^2 beta exp(-gamma/theta) (isotropic
    relativistic Maxwellian) by inverse CDF on a fine grid."""
    g, cdf = maxwell_juttner_table(theta, grid)
    return np.interp(rng.uniform(0.0, 1.0, n), cdf, g)


def _slab(counts_cap, live=None, with_parent=True):
    off = _offsets(counts_cap)
    n = int(off[-1])
    d = {"off": off, "count": np.zeros(len(counts_cap), dtype=np.int32) if live is None
         else np.asarray(live, dtype=np.int32),
         "px": np.zeros(n), "py": np.zeros(n), "pz": np.zeros(n), "w": np.zeros(n),
         "parent": np.full(n, -1, dtype=np.int64) if with_parent else None}
    return d


def assemble(name, Z, dt, processes, steps, Zstar, n_i, T_e,
             e_gamma, e_w, ne_cnt, g_k, g_w, ng_cnt, i_w, ni_cnt, rng,
             photon_extra, pair_cap, seed=1) -> Workload:
    """Lay out per-cell SoA arrays.  Photons get capacity ng + photon_extra
    per cell (Bremsstrahlung photons are appended there); e-/e+ product slabs
    get pair_cap per cell."""
    n_cells = len(Zstar)
    ex, ey, ez = momenta_from_gamma(rng, e_gamma)
    electrons = {"off": _offsets(ne_cnt), "count": None, "px": ex, "py": ey, "pz": ez,
                 "w": np.asarray(e_w, dtype=np.float64), "parent": None}
    gcap = np.asarray(ng_cnt, dtype=np.int64) + np.asarray(photon_extra, dtype=np.int64)
    photons = _slab(gcap, live=ng_cnt)
    u = isotropic(rng, len(g_k))
    goff = photons["off"]
    src = _offsets(ng_cnt)
    pos = np.concatenate([np.arange(goff[c], goff[c] + ng_cnt[c]) for c in range(n_cells)]) \
        if len(g_k) else np.zeros(0, np.int64)
    photons["px"][pos] = g_k * u[0]
    photons["py"][pos] = g_k * u[1]
    photons["pz"][pos] = g_k * u[2]
    photons["w"][pos] = g_w
    del src
    ions = {"off": _offsets(ni_cnt), "count": None, "px": None, "py": None, "pz": None,
            "w": np.asarray(i_w, dtype=np.float64), "parent": None}
    cells = {"Zstar": np.asarray(Zstar, dtype=np.float64), "n_i": np.asarray(n_i, dtype=np.float64),
             "T_e": np.asarray(T_e, dtype=np.float64)}
    return Workload(name, Z, dt, processes, steps, cells, electrons, photons, ions,
                    _slab(pair_cap), _slab(pair_cap), seed)


def moving_ions(wl: Workload, rng, umax) -> Workload:
    """Gives the ions proper velocities u = gamma_i beta_i (stored in the
    ions' px, py, pz): isotropic directions, |u| uniform on [0, umax]."""
    n = len(wl.ions["w"])
    d = isotropic(rng, n)
    m = rng.uniform(0.0, umax, n)
    wl.ions["px"], wl.ions["py"], wl.ions["pz"] = d[0] * m, d[1] * m, d[2] * m
    wl.name += "-moving-ions"
    return wl


def _photon_energy(rng, n):
    """k = 1.022 MeV + Exp(mean 5 MeV), in m_e c^2."""
    return (1.022 + rng.exponential(5.0, n)) / MEC2_MEV


# ------------------------------------------------------------------ configs
def cfg1(rng: Optional[np.random.Generator] = None, n_cells=64, per_cell=256, dt=1e-16) -> Workload:
    """Plain FP64 Bremsstrahlung: Cu (Z=29), Z*=10, n_i=8.5e22 cm^-3, T=100 eV;
    electron kinetic energy log-uniform 1-100 MeV, isotropic, unit weights
    (W = n_i/256 so that the weights sum to the density); 10 steps, dt=0.1 fs."""
    rng = rng or np.random.default_rng(1001)
    n_i = 8.5e28
    N = n_cells * per_cell
    tk = log_uniform(rng, 1.0, 100.0, N) / MEC2_MEV
    W = n_i / per_cell
    cnt = np.full(n_cells, per_cell)
    return assemble("cfg1-brems-fp64", 29, dt, PROC_BREMS, 10,
                    np.full(n_cells, 10.0), np.full(n_cells, n_i), np.full(n_cells, 100.0),
                    1.0 + tk, np.full(N, W), cnt, np.zeros(0), np.zeros(0), np.zeros(n_cells, np.int64),
                    np.full(N, W), cnt, rng, photon_extra=2 * cnt, pair_cap=np.full(n_cells, 16))


def cfg2(rng: Optional[np.random.Generator] = None, n_cells=4096, per_cell=1024, dt=1e-16) -> Workload:
    """Bethe-Heitler: Au (Z=79), Z* ~ U[0,79] per cell, n_i=5.9e22 cm^-3,
    T log-uniform 10 eV-10 keV; photon energy 1.022 MeV + Exp(5 MeV);
    photon weights (n_i/1024) LogNormal(0,1); 100 steps, dt=0.1 fs."""
    rng = rng or np.random.default_rng(1002)
    n_i = 5.9e28
    N = n_cells * per_cell
    Zs = rng.uniform(0.0, 79.0, n_cells)
    T = log_uniform(rng, 10.0, 1e4, n_cells)
    k = _photon_energy(rng, N)
    Wi = n_i / per_cell
    gw = Wi * rng.lognormal(0.0, 1.0, N)
    cnt = np.full(n_cells, per_cell)
    return assemble("cfg2-bh-fp32", 79, dt, PROC_BH, 100, Zs, np.full(n_cells, n_i), T,
                    np.zeros(0), np.zeros(0), np.zeros(n_cells, np.int64), k, gw, cnt,
                    np.full(N, Wi), cnt, rng, photon_extra=np.zeros(n_cells, np.int64),
                    pair_cap=2 * cnt)


def cfg3(rng: Optional[np.random.Generator] = None, n_cells=16384, dt=1e-16, lo=16, hi=8192) -> Workload:
    """Batched uneven cells, all three processes: per-cell counts of
    electrons, photons and ions drawn independently from a power law
    (alpha=1.5) on [16, 8192]; electrons 1-500 MeV log-uniform, photons as
    cfg2, Au ions as cfg2; 200 steps."""
    rng = rng or np.random.default_rng(1003)
    n_i = 5.9e28
    ne_c = power_law_counts(rng, n_cells, 1.5, lo, hi)
    ng_c = power_law_counts(rng, n_cells, 1.5, lo, hi)
    ni_c = power_law_counts(rng, n_cells, 1.5, lo, hi)
    Zs = rng.uniform(0.0, 79.0, n_cells)
    T = log_uniform(rng, 10.0, 1e4, n_cells)
    Wi_c = n_i / ni_c
    e_g = 1.0 + log_uniform(rng, 1.0, 500.0, int(ne_c.sum())) / MEC2_MEV
    e_w = np.repeat(Wi_c, ne_c)
    k = _photon_energy(rng, int(ng_c.sum()))
    g_w = np.repeat(Wi_c, ng_c) * rng.lognormal(0.0, 1.0, int(ng_c.sum()))
    i_w = np.repeat(Wi_c, ni_c)
    return assemble("cfg3-batched", 79, dt, PROC_BREMS | PROC_BH | PROC_TRIDENT, 200,
                    Zs, np.full(n_cells, n_i), T, e_g, e_w, ne_c, k, g_w, ng_c, i_w, ni_c, rng,
                    photon_extra=np.maximum(64, ne_c // 8), pair_cap=np.maximum(64, (ne_c + ng_c) // 8))


def cfg4(rng: Optional[np.random.Generator] = None, n_cells=1024, per_cell=4096, dt=1e-16):
    """Differentiable expected yield: Cu, per-cell Z* ~ U[1,29],
    n_e log-uniform 1e21-1e24 cm^-3, T_e log-uniform 10 eV-10 keV;
    electrons gamma log-uniform 2-1000, isotropic, w = 1."""
    rng = rng or np.random.default_rng(1004)
    N = n_cells * per_cell
    Zs = rng.uniform(1.0, 29.0, n_cells)
    ne = log_uniform(rng, 1e27, 1e30, n_cells)
    T = log_uniform(rng, 10.0, 1e4, n_cells)
    g = log_uniform(rng, 2.0, 1000.0, N)
    px, py, pz = momenta_from_gamma(rng, g)
    return {"name": "cfg4-expected-yield", "Z": 29, "dt": dt, "Zstar": Zs, "n_e": ne, "T_e": T,
            "off": _offsets(np.full(n_cells, per_cell)), "px": px, "py": py, "pz": pz,
            "w": np.ones(N)}


MJ_THETA = 5.0 / MEC2_MEV      # T = 5 MeV
CFG5_W_E = 1.5e25              # fast-electron density of the 10 um foil, m^-3 (Sec. IV)


def cfg5(rng: Optional[np.random.Generator] = None, n_cells=131072, per_cell=4096, dt=5e-17,
         processes=PROC_BREMS | PROC_BH) -> Workload:
    """Foil-transport scale Bremsstrahlung -> Bethe-Heitler chain: Au ions,
    n_i=5.9e22 cm^-3, Z*=5, T=1 eV (the paper's foil values applied to Au);
    electrons Maxwell-Juttner with T=5 MeV, isotropic, W_e=1.5e19 cm^-3/4096;
    photon and pair buffers 2x the electron count per cell; dt=0.05 fs.
    Host arrays, for cells in numbers the host holds (cfg5_device builds the
    full size in device memory)."""
    rng = rng or np.random.default_rng(1005)
    n_i = 5.9e28
    N = n_cells * per_cell
    g = maxwell_juttner_gamma(rng, N, MJ_THETA)
    cnt = np.full(n_cells, per_cell)
    return assemble("cfg5-foil-chain", 79, dt, processes, 1000,
                    np.full(n_cells, 5.0), np.full(n_cells, n_i), np.full(n_cells, 1.0),
                    g, np.full(N, CFG5_W_E / per_cell), cnt, np.zeros(0), np.zeros(0),
                    np.zeros(n_cells, np.int64), np.full(N, n_i / per_cell), cnt, rng,
                    photon_extra=2 * cnt, pair_cap=2 * cnt)


def cfg5_device(device, n_cells=131072, per_cell=4096, dt=5e-17, seed=1005, chunk=1 << 25) -> Workload:
    """The foil-transport chain of cfg5 generated in device memory, for the
    full size (about 125 GB in HBM: electrons 17.2 GB, ion weights 4.3 GB,
    three product slabs of 34.4 GB, no parent arrays): the same recipe as
    cfg5, drawn from torch's device generator seeded `seed` (uniforms in
    FP64) instead of numpy's.  Electrons: Maxwell-Juttner with T = 5 MeV
    by inverse CDF on the table of maxwell_juttner_table (linear between
    its nodes), isotropic directions; W_e = 1.5e19 cm^-3/4096, ions
    W_i = n_i/4096; photon, e- and e+ slabs 2 x 4096 per cell, empty.
    Processes: the Bremsstrahlung -> Bethe-Heitler chain."""
    import torch
    dev = torch.device(device)
    f8, i8 = torch.float64, torch.int64
    gen = torch.Generator(device=dev)
    gen.manual_seed(seed)
    N = n_cells * per_cell
    n_i = 5.9e28
    g_tab, cdf = maxwell_juttner_table(MJ_THETA)
    gt = torch.from_numpy(g_tab).to(dev)
    ct = torch.from_numpy(cdf).to(dev)
    px = torch.empty(N, dtype=f8, device=dev)
    py = torch.empty(N, dtype=f8, device=dev)
    pz = torch.empty(N, dtype=f8, device=dev)
    for a in range(0, N, chunk):
        b = min(N, a + chunk)
        n = b - a
        u = torch.rand(n, generator=gen, dtype=f8, device=dev)
        hi = torch.searchsorted(ct, u).clamp_(1, len(cdf) - 1)
        lo = hi - 1
        c0, c1, g0, g1 = ct[lo], ct[hi], gt[lo], gt[hi]
        g = g0 + (u - c0) / (c1 - c0) * (g1 - g0)
        p = torch.sqrt(torch.clamp(g * g - 1.0, min=0.0))
        mu = torch.rand(n, generator=gen, dtype=f8, device=dev) * 2.0 - 1.0
        phi = torch.rand(n, generator=gen, dtype=f8, device=dev) * (2.0 * math.pi)
        st = torch.sqrt(torch.clamp(1.0 - mu * mu, min=0.0))
        px[a:b] = p * st * torch.cos(phi)
        py[a:b] = p * st * torch.sin(phi)
        pz[a:b] = p * mu
        del u, hi, lo, c0, c1, g0, g1, g, p, mu, phi, st
    off = torch.arange(n_cells + 1, dtype=i8, device=dev) * per_cell
    electrons = {"off": off, "count": None, "px": px, "py": py, "pz": pz,
                 "w": torch.full((N,), CFG5_W_E / per_cell, dtype=f8, device=dev), "parent": None}
    ions = {"off": off, "count": None, "px": None, "py": None, "pz": None,
            "w": torch.full((N,), n_i / per_cell, dtype=f8, device=dev), "parent": None}

    def slab():
        cap = 2 * per_cell
        return {"off": torch.arange(n_cells + 1, dtype=i8, device=dev) * cap,
                "count": torch.zeros(n_cells, dtype=torch.int32, device=dev),
                **{k: torch.empty(n_cells * cap, dtype=f8, device=dev) for k in ("px", "py", "pz", "w")},
                "parent": None}
    cells = {"Zstar": torch.full((n_cells,), 5.0, dtype=f8, device=dev),
             "n_i": torch.full((n_cells,), n_i, dtype=f8, device=dev),
             "T_e": torch.full((n_cells,), 1.0, dtype=f8, device=dev)}
    return Workload("cfg5-foil-chain", 79, dt, PROC_BREMS | PROC_BH, 1000, cells, electrons, slab(), ions,
                    slab(), slab(), 1)


CONFIGS = {"cfg1": cfg1, "cfg2": cfg2, "cfg3": cfg3, "cfg5": cfg5}
