"""Seeded graph generators (edge lists over vertices 0..n-1, i < j)."""
from __future__ import annotations

from typing import List, Tuple

import numpy as np

Edge = Tuple[int, int]


def erdos_renyi(n: int, p: float, rng: np.random.Generator) -> List[Edge]:
    """G(n, p): pairs visited in lexicographic order (i < j), each kept with
    probability p by one uniform draw (App. F, max-cut and Lovasz classes)."""
    edges = []
    for i in range(n):
        for j in range(i + 1, n):
            if rng.random() < p:
                edges.append((i, j))
    return edges


def circulant(n: int, conn: List[int]) -> List[Edge]:
    """Circulant graph: vertex j adjacent to j +/- d (mod n) for d in conn."""
    es = set()
    for d in conn:
        for j in range(n):
            a, b = j, (j + d) % n
            if a != b:
                es.add((min(a, b), max(a, b)))
    return sorted(es)


def random_circulant(n: int, rng: np.random.Generator, prob: float = 0.3) -> Tuple[List[int], List[Edge]]:
    """Random connection set S in {1..floor(n/2)}, each d kept with prob `prob`,
    redrawn while S is empty or full; returns (S, edges)."""
    half = n // 2
    while True:
        S = [d for d in range(1, half + 1) if rng.random() < prob]
        if 0 < len(S) < half:
            return S, circulant(n, S)


def complete_graph(n: int) -> List[Edge]:
    return [(i, j) for i in range(n) for j in range(i + 1, n)]


def cycle_graph(n: int) -> List[Edge]:
    return circulant(n, [1])


def petersen_graph() -> List[Edge]:
    outer = [(i, (i + 1) % 5) for i in range(5)]
    spokes = [(i, i + 5) for i in range(5)]
    inner = [(5 + i, 5 + (i + 2) % 5) for i in range(5)]
    return sorted((min(a, b), max(a, b)) for a, b in outer + spokes + inner)
