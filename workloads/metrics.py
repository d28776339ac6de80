"""Search quality: exact FP64 cosine ground truth and k@n recall.

The ground truth ranks database vectors by the float64 scalar product of the
float32 vectors (they are l2-normalised, so this is cosine similarity;
Sec. 1.1 explains why cosine and Euclidean rank alike), nearest first, ties
to the lower id.  Recall "k@n" is the fraction of the k true nearest
neighbours found among the first n results of the proxy search (Sec. 5.3).
"""
from __future__ import annotations

import numpy as np
import torch


class ExactTopK:
    """Running exact top-k of fp64 dot products, fed one database chunk at a time."""

    def __init__(self, queries: torch.Tensor, k: int):
        self.q = queries.to(torch.float64)
        self.k = int(k)
        nq = self.q.shape[0]
        dev = self.q.device
        self.scores = torch.full((nq, 0), -np.inf, dtype=torch.float64, device=dev)
        self.ids = torch.zeros((nq, 0), dtype=torch.int64, device=dev)

    def add(self, rows: torch.Tensor, first_id: int) -> None:
        s = self.q @ rows.to(device=self.q.device, dtype=torch.float64).T
        ids = torch.arange(first_id, first_id + rows.shape[0], device=self.q.device).expand(s.shape[0], -1)
        # ids ascending before a stable sort by descending score = ties to lower id
        cs = torch.cat([self.scores, s], 1)
        ci = torch.cat([self.ids, ids], 1)
        order = torch.sort(ci, dim=1, stable=True).indices
        cs, ci = torch.gather(cs, 1, order), torch.gather(ci, 1, order)
        order = torch.sort(cs, dim=1, descending=True, stable=True).indices[:, : self.k]
        self.scores, self.ids = torch.gather(cs, 1, order), torch.gather(ci, 1, order)

    def result(self):
        return self.ids.cpu().numpy(), self.scores.cpu().numpy()


def recall_at(true_ids: np.ndarray, found_ids: np.ndarray, k: int, n: int) -> float:
    """Mean over queries of |first k true ids & first n found ids| / k."""
    t = np.asarray(true_ids)[:, :k]
    f = np.asarray(found_ids)[:, :n]
    hits = [len(set(a.tolist()) & set(b.tolist())) for a, b in zip(t, f)]
    return float(np.mean(hits)) / k
