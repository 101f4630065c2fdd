"""Error of the reduced screening potential against the two-exponential
Thomas-Fermi-Debye potential it replaces (Sec. II.B.2), over (Z*, T,
energy), as Figs. 5, 7 and 8 compare them: for each cell state and
incident energy, the spectrum k dsigma/dk of Bremsstrahlung (eq:csre up to
gamma_1 = 100, eq:csur above) or dsigma/dgamma_+ of Bethe-Heitler
(eq:dsdkbh) on a grid of x in (0, 1), in both forms, on the GPU
(cmc_cross_sections).  Reported per point: the mean and the largest
relative difference over x, and the relative difference of the spectrum's
integral over x (for Bremsstrahlung the radiated energy, i.e. the radiative
stopping power; for Bethe-Heitler the total cross section).

    python -m paper_1907_02814_amd.screening_map [--Z 29] [--ni 8.5e28]

prints the map as Markdown tables.  The paper takes Z*(T) from a fit that
it does not print: here Z* and T are independent axes."""
import argparse
import math

import numpy as np

MEC2_MEV = 0.51099895

ZSTARS = [0.0, 1.0, 5.0, 10.0, 20.0]
TEMPS = [1.0, 10.0, 100.0, 1e3, 1e4]
BREMS_MEV = [5.0, 100.0, 1000.0]      # electron kinetic energy
BH_MEV = [10.0, 100.0, 1e4]           # photon energy


def error_map(Z=29, n_i=8.5e28, zstars=ZSTARS, temps=TEMPS, brems_mev=BREMS_MEV, bh_mev=BH_MEV, nx=399):
    """{(process, E_MeV, Z*, T): (mean rel, max rel, integral rel)} from
    GPU evaluations of both forms; Z* above Z is skipped."""
    import torch
    import paper_1907_02814_amd as cmc
    tab = cmc.Tables(Z)
    x = (np.arange(nx) + 0.5) / nx
    rows, meta = [], []
    for proc, energies in ((cmc.BREMS, brems_mev), (cmc.BH, bh_mev)):
        for E in energies:
            e1 = 1.0 + E / MEC2_MEV if proc == cmc.BREMS else E / MEC2_MEV
            for zs in zstars:
                if zs > Z:
                    continue
                for T in temps:
                    meta.append((proc, E, zs, T))
                    rows.append((zs, T, e1))
    m = len(rows)
    rep = lambda v: np.repeat(np.asarray(v, dtype=np.float64), nx)
    Zs = rep([r[0] for r in rows])
    T = rep([r[1] for r in rows])
    e1 = rep([r[2] for r in rows])
    xx = np.tile(x, m)
    ni = np.full(m * nx, float(n_i))
    dev = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()
    procs = np.array([mm[0] for mm in meta])
    out = {}
    for proc in (cmc.BREMS, cmc.BH):
        sel = np.repeat(procs == proc, nx)
        if not sel.any():
            continue
        args = [dev(a[sel]) for a in (Zs, ni, T, e1, xx)]
        st = torch.zeros(1, dtype=torch.int32, device="cuda")
        r = cmc.cross_sections(tab, proc, *args, form=cmc.SCREEN_REDUCED, status=st).cpu().numpy()
        t = cmc.cross_sections(tab, proc, *args, form=cmc.SCREEN_TFD, status=st).cpu().numpy()
        if int(st.item()):
            raise RuntimeError(f"cmc_cross_sections: status {int(st.item())}")
        r, t = r.reshape(-1, nx), t.reshape(-1, nx)
        idx = [i for i, mm in enumerate(meta) if mm[0] == proc]
        for j, i in enumerate(idx):
            rel = np.abs(r[j] - t[j]) / t[j]
            out[meta[i]] = (float(rel.mean()), float(rel.max()), float(abs(r[j].sum() - t[j].sum()) / t[j].sum()))
    return out


def markdown(res, Z, n_i):
    lines = []
    for proc, name, unit in ((1, "Bremsstrahlung k dsigma/dk", "electron"), (2, "Bethe-Heitler dsigma/dgamma_+", "photon")):
        energies = sorted({k[1] for k in res if k[0] == proc})
        for E in energies:
            lines.append(f"\n{name}, {unit} {E:g} MeV, Z = {Z}, n_i = {n_i:g} m^-3: "
                         "mean / max relative difference over x, and of the integral (in %)\n")
            zs = sorted({k[2] for k in res if k[0] == proc and k[1] == E})
            ts = sorted({k[3] for k in res if k[0] == proc and k[1] == E})
            lines.append("| Z* \\ T (eV) | " + " | ".join(f"{t:g}" for t in ts) + " |")
            lines.append("|---|" + "---|" * len(ts))
            for z in zs:
                cells = []
                for t in ts:
                    a, b, c = res[(proc, E, z, t)]
                    cells.append(f"{100 * a:.2f} / {100 * b:.2f} / {100 * c:.2f}")
                lines.append(f"| {z:g} | " + " | ".join(cells) + " |")
    return "\n".join(lines)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--Z", type=int, default=29)
    ap.add_argument("--ni", type=float, default=8.5e28)
    a = ap.parse_args()
    res = error_map(a.Z, a.ni)
    print(markdown(res, a.Z, a.ni))


if __name__ == "__main__":
    main()
