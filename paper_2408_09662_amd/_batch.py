"""Persistent multi-program batches and HIP-graph replay (binding)."""

from __future__ import annotations


class Batch:
    def __init__(self, programs, **options):
        raise NotImplementedError("batch launch is not available yet")


class Graph:
    def __init__(self, *a, **k):
        raise NotImplementedError("graph capture is not available yet")
