"""Independent brute-force model of JaTAM assembly, used to pin the oracle.

Written separately from the C oracle and sharing nothing with it: its own
genome decoding, its own bond rule (stated as the paper's prose rule,
"labels bind in pairs 1-2, 3-4, ...; 0 is inert", §1.2, rather than the
matrix form of App. B.2), its own rotation of tiles, and, unlike the
oracle's incremental update, every frontier site's options are recomputed
from scratch from all occupied neighbours in every state (the "isotropic"
check of every frontier position, §3.2).

Two uses:
  explore()  every growth order, memoised on the configuration: the set of
             reachable events and terminal shapes (true class of a genotype);
  replay()   one run re-derived state by state, choosing the frontier site
             with rank floor(u*|F|/2^32) in row-major order, u taken from a
             caller-supplied word generator (the Philox stream).
"""
from __future__ import annotations

from dataclasses import dataclass, field

N, E, S, W = 0, 1, 2, 3
STEP = {N: (0, -1), E: (1, 0), S: (0, 1), W: (-1, 0)}


def decode(genome: int, t: int, c: int) -> list[tuple[int, int, int, int]]:
    """Tiles in genome order (seed first), each (N, E, S, W)."""
    bits = c.bit_length() - 1
    digits = []
    for k in range(4 * t):
        digits.append((genome >> (bits * (4 * t - 1 - k))) & (c - 1))
    return [tuple(digits[4 * i:4 * i + 4]) for i in range(t)]


def bonds(a: int, b: int, c: int) -> bool:
    """Labels bind in adjacent pairs (1,2), (3,4), ...; 0 binds nothing and a
    label whose partner would be >= c binds nothing."""
    lo, hi = min(a, b), max(a, b)
    return lo >= 1 and lo % 2 == 1 and hi == lo + 1 and hi < c


def rotate(tile, r: int):
    """Tile turned clockwise by r quarter turns (no flips)."""
    return tuple(tile[(d - r) % 4] for d in range(4))


def oriented_tiles(tiles) -> list[tuple[int, int, int, int]]:
    out = []
    for tile in tiles:
        for r in range(4):
            rt = rotate(tile, r)
            if rt not in out:
                out.append(rt)
    return out


def facing(d: int) -> int:
    return (d + 2) % 4


class Model:
    def __init__(self, genome: int, t: int, c: int, grid: int):
        self.tiles = decode(genome, t, c)
        self.c = c
        self.G = grid
        self.orients = oriented_tiles(self.tiles)
        self.seed_tile = self.tiles[0]
        self.centre = (grid // 2, grid // 2)

    def on_ring(self, x: int, y: int) -> bool:
        return x == 0 or y == 0 or x == self.G or y == self.G

    def site_options(self, placed: dict, x: int, y: int) -> set:
        """Distinct oriented tiles that bond to at least one occupied
        neighbour of the empty site (x, y)."""
        opts = set()
        for d, (dx, dy) in STEP.items():
            nb = placed.get((x + dx, y + dy))
            if nb is None:
                continue
            shown = nb[facing(d)]
            for o in self.orients:
                if bonds(o[d], shown, self.c):
                    opts.add(o)
        return opts

    def analyse(self, placed: dict):
        """From scratch: (event, frontier) where event is None, 'UNBOUND' or
        'AMBIG' and frontier maps each site with one option to that tile."""
        empty = set()
        for (x, y) in placed:
            for dx, dy in STEP.values():
                q = (x + dx, y + dy)
                if q not in placed:
                    empty.add(q)
        unbound = ambiguous = False
        frontier = {}
        for q in empty:
            opts = self.site_options(placed, *q)
            if not opts:
                continue
            if self.on_ring(*q):
                unbound = True
            elif len(opts) >= 2:
                ambiguous = True
            else:
                frontier[q] = next(iter(opts))
        event = "UNBOUND" if unbound else "AMBIG" if ambiguous else None
        return event, frontier


@dataclass
class Exploration:
    events: set = field(default_factory=set)
    terminals: set = field(default_factory=set)   # frozensets of occupied cells
    states: int = 0
    capped: bool = False
    choice_free: bool = True                      # no state had >= 2 frontier sites
    path_steps: int = -1                          # placements on the path if choice_free

    @property
    def truly_det(self) -> bool:
        return not self.capped and not self.events and len(self.terminals) == 1


def explore(genome: int, t: int, c: int = 8, grid: int = 16, cap: int = 200_000,
            stop_at: set | None = None) -> Exploration:
    """Every growth order from the seed, memoised on the configuration.
    Depth first; stops early once an event in stop_at has been reached."""
    m = Model(genome, t, c, grid)
    res = Exploration()
    start = {m.centre: m.seed_tile}
    seen = set()
    stack = [start]
    while stack:
        placed = stack.pop()
        key = frozenset(placed.items())
        if key in seen:
            continue
        seen.add(key)
        res.states += 1
        if res.states > cap:
            res.capped = True
            break
        event, frontier = m.analyse(placed)
        if event is not None:
            res.events.add(event)
            if stop_at and event in stop_at:
                break
            continue
        if not frontier:
            res.terminals.add(frozenset(placed))
            if res.choice_free:
                res.path_steps = len(placed) - 1
            continue
        if len(frontier) >= 2:
            res.choice_free = False
        for q, tile in frontier.items():
            nxt = dict(placed)
            nxt[q] = tile
            stack.append(nxt)
    if not res.choice_free:
        res.path_steps = -1
    return res


def replay(genome: int, t: int, c: int, grid: int, word):
    """One run re-derived from scratch.  word(s) returns the 32-bit random
    word of step s.  Returns (placements in order as (x, y), event or None,
    choice flag, final configuration)."""
    m = Model(genome, t, c, grid)
    placed = {m.centre: m.seed_tile}
    order = [m.centre]
    choice = False
    s = 0
    while True:
        event, frontier = m.analyse(placed)
        if event is not None or not frontier:
            return order, event, choice, placed
        if len(frontier) >= 2:
            choice = True
        sites = sorted(frontier, key=lambda q: (q[1], q[0]))
        j = (word(s) * len(sites)) >> 32
        q = sites[j]
        placed[q] = frontier[q]
        order.append(q)
        s += 1
