"""PROSITE-like protein patterns -> minimal DFAs (seeded synthetic workloads).

The paper builds its benchmark DFAs from PROSITE protein patterns and PCRE
expressions with an external toolset (Section 6, first paragraph; Section 6
"DFA construction" remark). Neither the pattern sets nor the toolset are
available, so this module writes its own construction from the textbook
definitions:

* a random pattern in the PROSITE element grammar (residue ``A``, allowed set
  ``[ST]``, excluded set ``{P}``, wildcard ``x``, repetition ``e(k)`` and
  ``e(k,l)``), drawn from a seed;
* Thompson's construction of an epsilon-NFA;
* the subset construction;
* Hopcroft's partition-refinement minimisation;
* states renumbered in breadth-first order from the start state (start = 0).

The default language is "the input contains the pattern", i.e. Sigma* P Sigma*
(the paper matches protein sequences against patterns, Section 6); an
anchored mode (exactly P, with a non-accepting error sink) is also offered.

Everything here produces *inputs* (DFAs and their patterns); none of it is the
membership test itself.  ``nfa_accepts`` simulates the Thompson NFA directly
(sets of NFA states, no subset construction, no minimisation) and
``to_python_regex`` renders the pattern for Python's ``re``; tests use both to
check the generated DFAs.
"""
from __future__ import annotations

import functools
import re
from dataclasses import dataclass
from typing import Dict, FrozenSet, List, Optional, Sequence, Tuple

import numpy as np

# The 20 standard one-letter amino-acid codes; symbol index = position here.
AMINO = "ACDEFGHIKLMNPQRSTVWY"
N_AMINO = len(AMINO)


@dataclass(frozen=True)
class Element:
    """One pattern element: a set of allowed residues repeated lo..hi times."""
    kind: str                 # 'res', 'set', 'excl', 'any'
    residues: Tuple[int, ...]  # residues named in the element (allowed or excluded)
    lo: int
    hi: int

    def allowed(self) -> Tuple[int, ...]:
        if self.kind in ("res", "set"):
            return tuple(sorted(self.residues))
        if self.kind == "excl":
            return tuple(a for a in range(N_AMINO) if a not in self.residues)
        return tuple(range(N_AMINO))

    def text(self) -> str:
        if self.kind == "res":
            core = AMINO[self.residues[0]]
        elif self.kind == "set":
            core = "[" + "".join(AMINO[a] for a in sorted(self.residues)) + "]"
        elif self.kind == "excl":
            core = "{" + "".join(AMINO[a] for a in sorted(self.residues)) + "}"
        else:
            core = "x"
        if self.lo == self.hi == 1:
            return core
        if self.lo == self.hi:
            return f"{core}({self.lo})"
        return f"{core}({self.lo},{self.hi})"


@dataclass(frozen=True)
class Pattern:
    elements: Tuple[Element, ...]

    def text(self) -> str:
        return "-".join(e.text() for e in self.elements)


def random_pattern(seed: int, n_elements: Optional[Tuple[int, int]] = None) -> Pattern:
    """Draw a PROSITE-like pattern from ``seed`` (numpy PCG64)."""
    rng = np.random.default_rng(seed)
    lo_n, hi_n = n_elements if n_elements is not None else (4, 12)
    n = int(rng.integers(lo_n, hi_n + 1))
    elems: List[Element] = []
    for idx in range(n):
        u = rng.random()
        if u < 0.40:
            kind, res = "res", (int(rng.integers(0, N_AMINO)),)
        elif u < 0.65:
            k = int(rng.integers(2, 5))
            kind, res = "set", tuple(int(a) for a in rng.choice(N_AMINO, k, replace=False))
        elif u < 0.75:
            k = int(rng.integers(1, 3))
            kind, res = "excl", tuple(int(a) for a in rng.choice(N_AMINO, k, replace=False))
        else:
            kind, res = "any", ()
        # first and last elements are never bare wildcards (as in PROSITE usage)
        if kind == "any" and idx in (0, n - 1):
            kind, res = "res", (int(rng.integers(0, N_AMINO)),)
        v = rng.random()
        if v < 0.65:
            lo = hi = 1
        elif v < 0.82:
            lo = hi = int(rng.integers(2, 5))
        else:
            lo = int(rng.integers(1, 4))
            hi = lo + int(rng.integers(1, 4))
        elems.append(Element(kind, res, lo, hi))
    return Pattern(tuple(elems))


def to_python_regex(p: Pattern, contains: bool = True) -> str:
    """Render the pattern for Python ``re`` over the amino-acid letters."""
    parts = []
    for e in p.elements:
        core = "[" + "".join(AMINO[a] for a in e.allowed()) + "]"
        parts.append(f"{core}{{{e.lo},{e.hi}}}")
    body = "".join(parts)
    if contains:
        return f"[{AMINO}]*{body}[{AMINO}]*"
    return body


# --------------------------------------------------------------------------
# Thompson epsilon-NFA
# --------------------------------------------------------------------------
class NFA:
    """epsilon-NFA: ``eps[s]`` = list of targets; ``edges[s]`` = (symbol set, target)."""

    def __init__(self) -> None:
        self.eps: List[List[int]] = []
        self.edges: List[List[Tuple[FrozenSet[int], int]]] = []
        self.start = 0
        self.final = 0

    def new(self) -> int:
        self.eps.append([])
        self.edges.append([])
        return len(self.eps) - 1


def _frag_symbols(nfa: NFA, syms: FrozenSet[int]) -> Tuple[int, int]:
    a, b = nfa.new(), nfa.new()
    nfa.edges[a].append((syms, b))
    return a, b


def _frag_concat(nfa: NFA, f: Tuple[int, int], g: Tuple[int, int]) -> Tuple[int, int]:
    nfa.eps[f[1]].append(g[0])
    return f[0], g[1]


def _frag_optional(nfa: NFA, f: Tuple[int, int]) -> Tuple[int, int]:
    a, b = nfa.new(), nfa.new()
    nfa.eps[a] += [f[0], b]
    nfa.eps[f[1]].append(b)
    return a, b


def _frag_star(nfa: NFA, f: Tuple[int, int]) -> Tuple[int, int]:
    a, b = nfa.new(), nfa.new()
    nfa.eps[a] += [f[0], b]
    nfa.eps[f[1]] += [f[0], b]
    return a, b


def _frag_empty(nfa: NFA) -> Tuple[int, int]:
    a, b = nfa.new(), nfa.new()
    nfa.eps[a].append(b)
    return a, b


def thompson(p: Pattern, contains: bool = True) -> NFA:
    """Thompson construction for P (anchored) or Sigma* P Sigma* (contains)."""
    nfa = NFA()
    any_sym = frozenset(range(N_AMINO))
    frag = _frag_empty(nfa)
    if contains:
        frag = _frag_concat(nfa, frag, _frag_star(nfa, _frag_symbols(nfa, any_sym)))
    for e in p.elements:
        syms = frozenset(e.allowed())
        for _ in range(e.lo):
            frag = _frag_concat(nfa, frag, _frag_symbols(nfa, syms))
        for _ in range(e.hi - e.lo):
            frag = _frag_concat(nfa, frag, _frag_optional(nfa, _frag_symbols(nfa, syms)))
    if contains:
        frag = _frag_concat(nfa, frag, _frag_star(nfa, _frag_symbols(nfa, any_sym)))
    nfa.start, nfa.final = frag
    return nfa


def _closure(nfa: NFA, states) -> FrozenSet[int]:
    stack = list(states)
    seen = set(stack)
    while stack:
        s = stack.pop()
        for t in nfa.eps[s]:
            if t not in seen:
                seen.add(t)
                stack.append(t)
    return frozenset(seen)


def _move(nfa: NFA, states: FrozenSet[int], a: int) -> FrozenSet[int]:
    out = set()
    for s in states:
        for syms, t in nfa.edges[s]:
            if a in syms:
                out.add(t)
    return frozenset(out)


def nfa_accepts(nfa: NFA, word: Sequence[int]) -> bool:
    """Direct set simulation of the epsilon-NFA (no determinisation)."""
    cur = _closure(nfa, [nfa.start])
    for a in word:
        cur = _closure(nfa, _move(nfa, cur, a))
        if not cur:
            return False
    return nfa.final in cur


# --------------------------------------------------------------------------
# Subset construction + Hopcroft minimisation
# --------------------------------------------------------------------------
class TooLarge(Exception):
    pass


def subset_construction(nfa: NFA, n_sym: int, contains: bool, max_states: int
                        ) -> Tuple[np.ndarray, np.ndarray]:
    """Return (delta[Q][n_sym] int64, accepting bool[Q]); start = state 0.

    In "contains" mode every subset that holds the NFA final state accepts
    every continuation, so such subsets are merged into one accepting sink
    while they are built (the language is unchanged; minimisation would merge
    them anyway).
    """
    start = _closure(nfa, [nfa.start])
    ids: Dict[FrozenSet[int], int] = {start: 0}
    order = [start]
    rows: List[List[int]] = []
    SINK = frozenset([-1])  # marker for the merged accepting sink
    i = 0
    while i < len(order):
        S = order[i]
        row = []
        for a in range(n_sym):
            if S == SINK:
                T = SINK
            else:
                T = _closure(nfa, _move(nfa, S, a))
                if contains and nfa.final in T:
                    T = SINK
            if T not in ids:
                if len(order) >= max_states:
                    raise TooLarge
                ids[T] = len(order)
                order.append(T)
            row.append(ids[T])
        rows.append(row)
        i += 1
    delta = np.asarray(rows, dtype=np.int64)
    acc = np.array([(S == SINK) or (nfa.final in S) for S in order], dtype=bool)
    return delta, acc


def hopcroft_minimise(delta: np.ndarray, acc: np.ndarray) -> Tuple[np.ndarray, np.ndarray]:
    """Hopcroft's algorithm; returns the quotient DFA in BFS order from state 0."""
    nq, ns = delta.shape
    # inverse transitions: inv[a][t] = list of s with delta[s][a] == t
    inv = [[[] for _ in range(nq)] for _ in range(ns)]
    for s in range(nq):
        for a in range(ns):
            inv[a][int(delta[s, a])].append(s)
    F = frozenset(np.nonzero(acc)[0].tolist())
    NF = frozenset(range(nq)) - F
    partition = [blk for blk in (F, NF) if blk]
    block_of = np.zeros(nq, dtype=np.int64)
    for bi, blk in enumerate(partition):
        for s in blk:
            block_of[s] = bi
    work = set()
    if len(partition) == 2:
        work.add(min(range(2), key=lambda b: len(partition[b])))
    elif partition:
        work.add(0)
    while work:
        A = partition[work.pop()]
        for a in range(ns):
            X = set()
            for t in A:
                X.update(inv[a][t])
            if not X:
                continue
            touched: Dict[int, List[int]] = {}
            for s in X:
                touched.setdefault(int(block_of[s]), []).append(s)
            for bi, members in touched.items():
                Y = partition[bi]
                if len(members) == len(Y):
                    continue
                inter = frozenset(members)
                diff = Y - inter
                partition[bi] = inter
                nb = len(partition)
                partition.append(diff)
                for s in diff:
                    block_of[s] = nb
                if bi in work:
                    work.add(nb)
                else:
                    work.add(bi if len(inter) <= len(diff) else nb)
    # quotient + BFS renumbering from the block of state 0
    nb = len(partition)
    qdelta = np.zeros((nb, ns), dtype=np.int64)
    qacc = np.zeros(nb, dtype=bool)
    for bi, blk in enumerate(partition):
        rep = next(iter(blk))
        qdelta[bi] = block_of[delta[rep]]
        qacc[bi] = acc[rep]
    start = int(block_of[0])
    order = [start]
    newid = {start: 0}
    i = 0
    while i < len(order):
        b = order[i]
        for a in range(ns):
            t = int(qdelta[b, a])
            if t not in newid:
                newid[t] = len(order)
                order.append(t)
        i += 1
    out = np.zeros((len(order), ns), dtype=np.int64)
    oacc = np.zeros(len(order), dtype=bool)
    for b in order:
        out[newid[b]] = [newid[int(t)] for t in qdelta[b]]
        oacc[newid[b]] = qacc[b]
    return out, oacc


@dataclass
class PatternDFA:
    pattern: Pattern
    seed: int
    contains: bool
    delta: np.ndarray        # uint32 [Q][20]
    accepting: np.ndarray    # uint32 state ids
    q0: int
    byte_to_symbol: np.ndarray  # uint8 [256], 0xFF = not an amino-acid letter

    @property
    def num_states(self) -> int:
        return int(self.delta.shape[0])


def amino_byte_map() -> np.ndarray:
    lut = np.full(256, 0xFF, dtype=np.uint8)
    for i, ch in enumerate(AMINO):
        lut[ord(ch)] = i
    return lut


def pattern_dfa(seed: int, contains: bool = True, max_states: int = 20000,
                n_elements: Optional[Tuple[int, int]] = None) -> PatternDFA:
    p = random_pattern(seed, n_elements)
    nfa = thompson(p, contains)
    delta, acc = subset_construction(nfa, N_AMINO, contains, max_states)
    mdelta, macc = hopcroft_minimise(delta, acc)
    return PatternDFA(p, seed, contains, mdelta.astype(np.uint32),
                      np.nonzero(macc)[0].astype(np.uint32), 0, amino_byte_map())


def occurrence_bound(p: Pattern, weights: Sequence[float]) -> float:
    """Union bound on the probability that an occurrence of P starts at a given
    position of an i.i.d. residue stream with letter weights ``weights``:
    prod over elements of sum_{k=lo..hi} q_e^k, q_e = probability of one of the
    element's allowed residues (every combination of repeat counts is counted
    once)."""
    w = np.asarray(weights, dtype=float)
    q = w / w.sum()
    u = 1.0
    for e in p.elements:
        qe = float(q[list(e.allowed())].sum())
        u *= sum(qe ** k for k in range(e.lo, e.hi + 1))
    return u


@functools.lru_cache(maxsize=None)
def search_pattern_dfa(first_seed: int, lo: int, hi: int, contains: bool = True,
                       n_elements: Optional[Tuple[int, int]] = None,
                       max_tries: int = 20000, rare_in: Optional[int] = None,
                       weights: Optional[Tuple[float, ...]] = None,
                       expected_max: float = 0.05) -> PatternDFA:
    """First seed s = first_seed, first_seed+1, ... whose minimal DFA has lo <= #Q <= hi.

    With ``rare_in = n`` only patterns whose expected number of occurrences in
    n residues drawn i.i.d. from ``weights`` is at most ``expected_max`` (by
    ``occurrence_bound``) qualify, so that a walk over such an input almost
    surely never reaches the accepting sink of Sigma* P Sigma*; the cheap test
    runs before the DFA is built."""
    for s in range(first_seed, first_seed + max_tries):
        if rare_in is not None:
            if rare_in * occurrence_bound(random_pattern(s, n_elements), weights) > expected_max:
                continue
        try:
            d = pattern_dfa(s, contains, max_states=max(4 * hi, 64), n_elements=n_elements)
        except TooLarge:
            continue
        if lo <= d.num_states <= hi:
            return d
    raise RuntimeError(f"no pattern DFA with {lo}..{hi} states from seed {first_seed}")


def python_regex_accepts(p: Pattern, word: bytes, contains: bool = True) -> bool:
    return re.fullmatch(to_python_regex(p, contains), word.decode("ascii")) is not None
