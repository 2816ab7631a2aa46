"""JSON-lines log of a lattice or ensemble run.

Each call of ``RunLog.record`` appends one line: the step, the wall time since
the log was opened, the lattice-update rate since the previous record, and per
replica the mass, momentum, density range and count of non-finite or
non-positive densities (the library's FP64 reductions, ``fsc_stats``), plus,
if asked for, the S(k) bins accumulated so far (``fsc_read_sk``).  The log only
serialises what the library returns.

    with fsc.Lattice(p) as lat, RunLog("run.jsonl", lat, sk_kind=fsc.FSC_SK_AXIS) as log:
        lat.init_uniform()
        for _ in range(10):
            lat.run(1000, sk_every=100)
            log.record()
"""
from __future__ import annotations

import json
import time


class RunLog:
    def __init__(self, path: str, sim, replicas=None, sk_kind=None, mode: str = "w"):
        """sim: a Lattice or an Ensemble; replicas: the ensemble replicas to
        log (default all); sk_kind: FSC_SK_AXIS or FSC_SK_RADIAL to add the
        bins, None to leave them out."""
        self.sim = sim
        self.ensemble = hasattr(sim, "plist")
        if self.ensemble:
            self.replicas = list(range(sim.n)) if replicas is None else list(replicas)
        else:
            self.replicas = [None]
        self.sk_kind = sk_kind
        self._fh = open(path, mode)
        self._t0 = time.perf_counter()
        self._last = (self._t0, int(sim.t))

    def _stats(self, r):
        if self.ensemble:
            return self.sim.stats(r, allow_diverged=True)
        return self.sim.stats(allow_diverged=True)

    def _sk(self, r):
        if self.ensemble:
            return self.sim.read_sk(r, self.sk_kind)
        return self.sim.read_sk(self.sk_kind)

    def record(self, **extra) -> dict:
        """Appends one record (extra keyword values are stored as given) and
        returns it."""
        step = int(self.sim.t)
        reps, nodes = [], 0
        for r in self.replicas:
            st = self._stats(r)
            nodes += int(st["nodes"])
            rec = {"replica": r, "mass": float(st["mass"]),
                   "mom": [float(v) for v in st["mom"]],
                   "rho_min": float(st["rho_min"]), "rho_max": float(st["rho_max"]),
                   "bad": int(st["bad"])}
            if self.sk_kind is not None:
                s, s2, cnt = self._sk(r)
                rec["sk_sum"] = s.tolist()
                rec["sk_sumsq"] = s2.tolist()
                rec["sk_count"] = cnt.tolist()
            reps.append(rec)
        now = time.perf_counter()
        dt, dsteps = now - self._last[0], step - self._last[1]
        line = {"step": step, "wall_s": now - self._t0,
                "mlups": nodes * dsteps / dt / 1e6 if dt > 0 and dsteps > 0 else None,
                "replicas": reps}
        line.update(extra)
        self._fh.write(json.dumps(line) + "\n")
        self._fh.flush()
        self._last = (now, step)
        return line

    def close(self):
        if not self._fh.closed:
            self._fh.close()

    def __enter__(self):
        return self

    def __exit__(self, *a):
        self.close()


def read(path: str) -> list:
    """The records of a run log, in order."""
    with open(path) as fh:
        return [json.loads(line) for line in fh if line.strip()]
