"""Max-pressure signal control through the runtime control API.

The paper evaluates signal control on the simulator, with max pressure
(Varaiya, 2013) among the baselines; here it is the closed-loop use of
``moss_set_signal_phase`` and ``moss_read_road_stats``.  Every ``period``
steps each signalised node shows the phase with the largest pressure:

    pressure(p) = sum over incoming roads r of group p of (n_r - mean_out),

where n_r is the number of vehicles on road r and mean_out the mean number on
the node's outgoing roads (turning shares are not known, so every movement of
the node is taken to discharge into the same average downstream road).  Ties
keep the phase shown.  The decision is made on the host from the road
measures; the simulation itself stays on the GPU.
"""
from __future__ import annotations

from typing import Tuple

import numpy as np


class MaxPressure:
    def __init__(self, sc, period: int = 10):
        self.period = int(period)
        groups = np.asarray(sc.road_group, np.int64)
        to = np.asarray(sc.road_to, np.int64)
        frm = np.asarray(sc.road_from, np.int64)
        sig = np.asarray(sc.node_cycle) > 0
        self.nodes = np.flatnonzero(sig).astype(np.int32)
        n_groups = int(groups.max()) + 1 if groups.size and groups.max() >= 0 else 0
        self.n_groups = max(n_groups, 1)
        # incoming roads with a group at signalised nodes, outgoing roads of every node
        self.in_roads = [np.flatnonzero((to == j) & (groups >= 0)) for j in self.nodes]
        self.in_groups = [groups[r] for r in self.in_roads]
        self.out_roads = [np.flatnonzero(frm == j) for j in self.nodes]
        self.phase = np.zeros(self.nodes.shape[0], np.int32)

    def decide(self, count: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
        """Phases for every signalised node from the vehicles per road."""
        count = np.asarray(count, np.float64)
        for q in range(self.nodes.shape[0]):
            out = self.out_roads[q]
            mean_out = count[out].mean() if out.size else 0.0
            press = np.zeros(self.n_groups)
            np.add.at(press, self.in_groups[q], count[self.in_roads[q]] - mean_out)
            best = int(np.argmax(press))
            if press[best] > press[self.phase[q]]:
                self.phase[q] = best
        return self.nodes, self.phase.copy()

    def run(self, sim, steps: int, also=None):
        """Steps the simulator under control; `also` (another simulator, e.g.
        the oracle) receives the same decisions."""
        done = 0
        while done < steps:
            count, _ = sim.road_stats()
            nodes, phases = self.decide(count)
            sim.set_signal_phase(nodes, phases)
            if also is not None:
                also.set_signal_phase(nodes, phases)
            k = min(self.period, steps - done)
            sim.step(k)
            if also is not None:
                also.step(k)
            done += k
