"""Device-side request buffers for the serving loop (marshalling only).

A ray pool (world-space rays) and its broad-phase pairs, sorted by ray, live on
the device once.  A request is a window [start, start + n) of the pool: its rays
and output are views of pool-sized buffers, its pairs are the pool pairs whose ray
falls in the window, re-indexed to the window.
"""

import numpy as np


class RequestSet:
    def __init__(self, L, rays, pair_ray, pair_inst, instances, windows, device="cuda"):
        import torch
        self.L = L
        order = np.lexsort((pair_inst, pair_ray))           # by ray, then instance
        pr, pi = pair_ray[order].astype(np.int64), pair_inst[order]
        self.rays = torch.from_numpy(np.ascontiguousarray(rays)).to(device)
        self.inst = torch.from_numpy(L.instances_array(instances)).to(device)
        self.windows = windows
        self.outs, self.pr, self.pi = [], [], []
        for (s, n, _) in windows:
            a, b = np.searchsorted(pr, s), np.searchsorted(pr, s + n)
            self.pr.append(torch.from_numpy((pr[a:b] - s).astype(np.int32)).to(device))
            self.pi.append(torch.from_numpy(pi[a:b].astype(np.int32)).to(device))
            self.outs.append(torch.empty((n, 6), dtype=torch.float32, device=device))

    def request(self, j, timeout_ns=0):
        s, n, _ = self.windows[j]
        return self.L.make_request(rays=self.rays[s:s + n], out=self.outs[j], pair_ray=self.pr[j],
                                   pair_inst=self.pi[j], inst=self.inst, timeout_ns=timeout_ns)

    def rays_of(self, j):
        s, n, _ = self.windows[j]
        return self.rays[s:s + n]

    def total_rays(self):
        return sum(n for (_, n, _) in self.windows)
