"""Seeded synthetic inputs for the D2Q9 MRT lattice Boltzmann workloads.

This module is shared by the oracle-side tests and the GPU library's tests
and benchmark.  It holds input recipes only -- initial density and velocity
fields, relaxation parameter values and workload specifications -- and none
of the scheme's arithmetic (no moments, equilibria, collision or streaming).
Relaxation sets are returned as the raw numbers printed in the paper or drawn
by the recipe; converting a viscosity into a relaxation rate is left to each
consumer.

Recipes (with the paper passages they imitate):

* ``gaussian_pulse``: the Gaussian density pulse of Sec. 5.2,
  rho = rho0 + eps exp(-ln2 d^2 / b^2), u = (U0, 0), with b the half-width in
  cells and d the minimum-image distance on the periodic lattice.
* ``plane_waves``: a right-running plane acoustic wave along x superposed on
  a shear wave (u_y) on a uniform mean flow, the linear waves whose phase
  and decay the von Neumann analysis of Sec. 4 predicts.
* ``random_pulses``: sums of seeded Gaussian pulses for the precision study.
* ``batch_specs`` / ``serving_trace``: many independent lattices of uneven
  size with sampled relaxation parameters, and a Poisson stream of such jobs.
"""
import math
from dataclasses import dataclass, field
from typing import Callable, Dict, List, Optional

import numpy as np

CS = 1.0 / math.sqrt(3.0)   # D2Q9 sound speed printed in Sec. 5.1 (0.57735)

# Relaxation parameter sets printed in the paper.  Keys: s_e, s_eps, s_q and
# either s_nu or nu (lattice viscosity); each consumer converts nu -> s_nu.
PRESETS: Dict[str, Dict[str, float]] = {
    # Original MRT (Lallemand-Luo): only s_nu is free (Sec. 2.3).
    "LL": {"s_e": 1.64, "s_eps": 1.54, "s_q": 1.9},
    # Table 5, group A / B: optimised for a pulse with uniform flow (Sec. 5.2).
    "T5A": {"s_e": 1.99, "s_nu": 1.999960001, "s_eps": 1.962820428, "s_q": 1.992761413},
    "T5B": {"s_e": 1.99999, "s_nu": 1.999960001, "s_eps": 1.999875273, "s_q": 1.999969578},
    # Table 4, group A / B: point source, zero mean flow (Sec. 5.1); s_e = s_nu.
    "T4A": {"s_e": 1.99044751, "s_nu": 1.99044751, "s_eps": 2.0, "s_q": 0.00875438872,
            "nu_printed": 0.000799861},
    "T4B": {"s_e": 1.95321, "s_nu": 1.95321, "s_eps": 2.0, "s_q": 0.04126919093,
            "nu_printed": 0.00399257},
}

# Sigma-form tables (sigma = 1/s - 1/2), Sec. 4.2.
SIGMA_TABLES = {
    # Table 1 (zero mean flow, n = 5): sigma_e = sigma_nu, sigma_eps, sigma_q, F^o or curly-F
    "T1A": {"sigma_e": 0.0025, "sigma_nu": 0.0025, "sigma_eps": 0.0, "sigma_q": 105.468091254867,
            "Fo": 17.9024342612509066},
    "T1B": {"sigma_e": 0.0025, "sigma_nu": 0.0025, "sigma_eps": 0.0, "sigma_q": 105.465307838135,
            "F": 17.9030645832220686},
    "T1C": {"sigma_e": 0.1, "sigma_nu": 0.1, "sigma_eps": 0.0, "sigma_q": 26.3631592758091,
            "Fo": 17.9107477965877778},
    "T1D": {"sigma_e": 0.1, "sigma_nu": 0.1, "sigma_eps": 0.0, "sigma_q": 26.3520430827600,
            "F": 17.9208148202264042},
    # Table 2 (u_m = 0.1, n = 4)
    "T2A": {"sigma_e": 0.001, "sigma_nu": 0.001, "sigma_eps": 0.00751873323089156,
            "sigma_q": 0.00171909400064198},
    "T2B": {"sigma_e": 0.0025, "sigma_nu": 0.0025, "sigma_eps": 0.0187982349323006,
            "sigma_q": 0.00429903714246050},
    # Table 3 (bulk-viscosity separated, u_m = 0.1, n = 4)
    "T3A": {"sigma_e": 0.0025125628, "sigma_nu": 0.00001, "sigma_eps": 0.00947095595580122,
            "sigma_q": 0.00181622011980382},
    "T3B": {"sigma_e": 0.0000025, "sigma_nu": 0.00001, "sigma_eps": 0.0000311837523990053,
            "sigma_q": 0.00000760552251906507},
}


def _grid(nx: int, ny: int):
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    return x, y


def _min_image(d, n):
    return d - n * np.round(d / n)


def gaussian_pulse(nx: int, ny: int, amplitude: float, half_width: float,
                   center: Optional[tuple] = None, rho0: float = 1.0,
                   u0: tuple = (0.0, 0.0)):
    """(rho, ux, uy) float64 [ny, nx] for one Gaussian density pulse.

    Default centre: cell (nx // 2, ny // 2), 0-based."""
    if center is None:
        center = (nx // 2, ny // 2)
    x, y = _grid(nx, ny)
    dx = _min_image(x - center[0], nx)
    dy = _min_image(y - center[1], ny)
    rho = rho0 + amplitude * np.exp(-math.log(2.0) * (dx * dx + dy * dy) / (half_width ** 2))
    ux = np.full((ny, nx), float(u0[0]))
    uy = np.full((ny, nx), float(u0[1]))
    return np.ascontiguousarray(rho), ux, uy


def plane_waves(nx: int, ny: int, mode: int, amplitude: float, shear_amplitude: float,
                u0x: float, rho0: float = 1.0):
    """Plane acoustic wave along x (rho' = A cos kx, u_x' = A c_s cos kx) plus a
    shear wave u_y = A_s cos kx on a mean flow u0x, k = 2 pi mode / nx.
    Every row is identical (the fields do not depend on y)."""
    k = 2.0 * math.pi * mode / nx
    x = np.arange(nx, dtype=np.float64)
    c = np.cos(k * x)
    rho = np.broadcast_to(rho0 + amplitude * c, (ny, nx)).copy()
    ux = np.broadcast_to(u0x + amplitude * CS * c, (ny, nx)).copy()
    uy = np.broadcast_to(shear_amplitude * c, (ny, nx)).copy()
    return rho, ux, uy


@dataclass
class PulseSpec:
    amplitude: float
    half_width: float
    cx: float
    cy: float


def random_pulse_specs(nx: int, ny: int, seed: int, count: int = 16,
                       amp_range=(1e-5, 1e-3), width_range=(3.0, 12.0)) -> List[PulseSpec]:
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(count):
        a = math.exp(rng.uniform(math.log(amp_range[0]), math.log(amp_range[1])))
        b = rng.uniform(*width_range)
        out.append(PulseSpec(a, b, rng.uniform(0, nx), rng.uniform(0, ny)))
    return out


def pulses_field(nx: int, ny: int, specs: List[PulseSpec], rho0: float = 1.0,
                 rows: Optional[slice] = None):
    """rho = rho0 + sum of the pulses (minimum-image distance); u = 0.

    ``rows`` restricts the output to a band of rows (for sampled checks on
    large lattices)."""
    ys = np.arange(ny, dtype=np.float64)
    if rows is not None:
        ys = ys[rows]
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = ys[:, None]
    rho = np.full((len(ys), nx), rho0)
    for p in specs:
        dx = _min_image(x - p.cx, nx)
        dy = _min_image(y - p.cy, ny)
        rho += p.amplitude * np.exp(-math.log(2.0) * (dx * dx + dy * dy) / (p.half_width ** 2))
    z = np.zeros_like(rho)
    return rho, z, z.copy()


def pulses_field_torch(nx: int, ny: int, specs: List[PulseSpec], device, rho0: float = 1.0):
    """``pulses_field`` generated on a torch device (float64)."""
    import torch
    x = torch.arange(nx, dtype=torch.float64, device=device)[None, :]
    y = torch.arange(ny, dtype=torch.float64, device=device)[:, None]
    rho = torch.full((ny, nx), rho0, dtype=torch.float64, device=device)
    for p in specs:
        dx = x - p.cx
        dx = dx - nx * torch.round(dx / nx)
        dy = y - p.cy
        dy = dy - ny * torch.round(dy / ny)
        rho += p.amplitude * torch.exp(-math.log(2.0) * (dx * dx + dy * dy) / (p.half_width ** 2))
    z = torch.zeros_like(rho)
    return rho, z, z.clone()


def pulses_window(nx: int, ny: int, specs: List[PulseSpec], x0: int, y0: int, w: int, rho0: float = 1.0):
    """The fields of ``pulses_field`` on a w x w window of the periodic
    nx x ny lattice whose corner is cell (x0, y0): entry [i, j] is cell
    ((x0 + j) mod nx, (y0 + i) mod ny)."""
    x = ((x0 + np.arange(w)) % nx).astype(np.float64)[None, :]
    y = ((y0 + np.arange(w)) % ny).astype(np.float64)[:, None]
    rho = np.full((w, w), rho0)
    for p in specs:
        dx = _min_image(x - p.cx, nx)
        dy = _min_image(y - p.cy, ny)
        rho += p.amplitude * np.exp(-math.log(2.0) * (dx * dx + dy * dy) / (p.half_width ** 2))
    z = np.zeros_like(rho)
    return rho, z, z.copy()


def random_pulses(nx: int, ny: int, seed: int, count: int = 16,
                  amp_range=(1e-5, 1e-3), width_range=(3.0, 12.0)):
    """Sum of ``count`` seeded Gaussian pulses on rho0 = 1, u = 0."""
    return pulses_field(nx, ny, random_pulse_specs(nx, ny, seed, count, amp_range, width_range))


def draw_relaxation(rng) -> Dict[str, float]:
    """One candidate relaxation set: s_e, s_eps ~ U[1, 1.9], s_q ~ U[1, 1.99],
    nu ~ U[1e-4, 1e-2] (lattice units)."""
    return {"s_e": float(rng.uniform(1.0, 1.9)), "s_eps": float(rng.uniform(1.0, 1.9)),
            "s_q": float(rng.uniform(1.0, 1.99)), "nu": float(rng.uniform(1e-4, 1e-2))}


@dataclass
class LatticeSpec:
    nx: int
    ny: int
    relax: Dict[str, float]
    pulse: PulseSpec
    steps: int = 500
    storage: str = "f32"
    init: str = "pulse"          # "pulse" or "wave"
    wave_mode: int = 0
    wave_amplitude: float = 0.0
    arrival: float = 0.0
    tag: int = 0

    def fields(self):
        if self.init == "wave":
            return plane_waves(self.nx, self.ny, self.wave_mode, self.wave_amplitude, 0.0, 0.0)
        return pulses_field(self.nx, self.ny, [self.pulse])

    def fields_torch(self, device):
        """The same fields generated on a torch device (float64)."""
        import torch
        x = torch.arange(self.nx, dtype=torch.float64, device=device)[None, :]
        y = torch.arange(self.ny, dtype=torch.float64, device=device)[:, None]
        if self.init == "wave":
            k = 2.0 * math.pi * self.wave_mode / self.nx
            c = torch.cos(k * x).expand(self.ny, self.nx)
            rho = 1.0 + self.wave_amplitude * c
            ux = self.wave_amplitude * CS * c
            uy = torch.zeros_like(rho)
            return rho.contiguous(), ux.contiguous(), uy
        p = self.pulse
        dx = x - p.cx
        dx = dx - self.nx * torch.round(dx / self.nx)
        dy = y - p.cy
        dy = dy - self.ny * torch.round(dy / self.ny)
        rho = 1.0 + p.amplitude * torch.exp(-math.log(2.0) * (dx * dx + dy * dy) / (p.half_width ** 2))
        z = torch.zeros_like(rho)
        return rho.contiguous(), z, z.clone()


def _log_uniform_int(rng, lo, hi):
    return int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))


def batch_specs(seed: int, count: int = 256, side_range=(64, 1024), steps: int = 500,
                accept: Optional[Callable[[Dict[str, float]], bool]] = None) -> List[LatticeSpec]:
    """Independent lattices with log-uniform side lengths (nx, ny drawn
    separately), sampled relaxation sets (redrawn until ``accept`` returns
    True), and one pulse each (A = 1e-3, b ~ U[3, 12] capped at min(nx,ny)/8,
    centre uniform)."""
    rng = np.random.default_rng(seed)
    out = []
    for t in range(count):
        nx = _log_uniform_int(rng, *side_range)
        ny = _log_uniform_int(rng, *side_range)
        while True:
            relax = draw_relaxation(rng)
            if accept is None or accept(relax):
                break
        b = min(rng.uniform(3.0, 12.0), min(nx, ny) / 8.0)
        pulse = PulseSpec(1e-3, b, rng.uniform(0, nx), rng.uniform(0, ny))
        out.append(LatticeSpec(nx, ny, relax, pulse, steps=steps, tag=t))
    return out


def serving_trace(seed: int, rate: float, njobs: int, side_range=(128, 4096),
                  steps_range=(200, 5000),
                  accept: Optional[Callable[[Dict[str, float]], bool]] = None,
                  storages=("f32", "f16")) -> List[LatticeSpec]:
    """A Poisson stream of simulation jobs (exponential inter-arrival times at
    ``rate`` jobs/s): square side log-uniform, steps uniform, storage drawn
    uniformly from ``storages`` (default f32 or f16 50/50), sampled relaxation
    set, pulse (A = 1e-3) or x-plane wave (A = 1e-4, mode 1..8) 50/50."""
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for j in range(njobs):
        t += rng.exponential(1.0 / rate)
        side = _log_uniform_int(rng, *side_range)
        steps = int(rng.integers(steps_range[0], steps_range[1] + 1))
        storage = storages[min(int(rng.uniform() * len(storages)), len(storages) - 1)]
        while True:
            relax = draw_relaxation(rng)
            if accept is None or accept(relax):
                break
        if rng.uniform() < 0.5:
            b = min(rng.uniform(3.0, 12.0), side / 8.0)
            spec = LatticeSpec(side, side, relax, PulseSpec(1e-3, b, rng.uniform(0, side),
                                                              rng.uniform(0, side)),
                               steps=steps, storage=storage, arrival=t, tag=j)
        else:
            spec = LatticeSpec(side, side, relax, PulseSpec(0.0, 1.0, 0.0, 0.0), steps=steps,
                               storage=storage, init="wave", wave_mode=int(rng.integers(1, 9)),
                               wave_amplitude=1e-4, arrival=t, tag=j)
        out.append(spec)
    return out


# The named workloads of the benchmark and the tests.
WORKLOADS = {
    "pulse64": dict(nx=64, ny=64, storage="f64", relax="LL", nu=1e-3, steps=500,
                    amplitude=1e-3, half_width=4.0),
    "waves4096": dict(nx=4096, ny=4096, storage="f32", relax="T5A", steps=2000, mode=8,
                      amplitude=1e-4, shear_amplitude=1e-4, u0x=0.1 * CS),
    "pulses8192": dict(nx=8192, ny=8192, relax="LL", nu=1e-3, steps=1000, count=16, seed=1234),
    "batch256": dict(count=256, steps=500, seed=2024),
}
