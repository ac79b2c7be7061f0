"""CPU ORACLE (brute force) -- TEST INFRASTRUCTURE ONLY.

The definition written out in plain Python, for tiny inputs: every group
keeps its full history; after each batch the window of a touched group is
the last W values of that history and its sum is recomputed from scratch
(the experimental setting of Section 5.1 rescans the whole window after
every insertion; only the end-of-batch value is emitted here).  Python
integers are exact and ``int / int`` is the correctly rounded IEEE double
quotient.
"""
from __future__ import annotations

from collections import defaultdict


class BruteForce:
    def __init__(self, groups: int, window: int):
        self.groups = groups
        self.window = window
        self.history = defaultdict(list)

    def push(self, keys, values):
        keys = [int(k) for k in keys]
        values = [int(v) for v in values]
        if any(k < 0 or k >= self.groups for k in keys):
            raise ValueError("key out of range")
        for k, v in zip(keys, values):
            self.history[k].append(v)
        out = []
        for g in sorted(set(keys)):
            win = self.history[g][-self.window:]
            s = sum(win)
            c = len(win)
            out.append((g, s, c, s / c))
        return out

    def push_tuples(self, keys, values):
        """Per tuple: its group's last W values right after it arrived,
        summed afresh (Section 5.1 rescans the window after every insert)."""
        keys = [int(k) for k in keys]
        values = [int(v) for v in values]
        if any(k < 0 or k >= self.groups for k in keys):
            raise ValueError("key out of range")
        out = []
        for k, v in zip(keys, values):
            self.history[k].append(v)
            win = self.history[k][-self.window:]
            s = sum(win)
            out.append((s, len(win), s / len(win)))
        return out
