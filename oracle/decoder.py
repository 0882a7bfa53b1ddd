"""Detection events and minimum-weight perfect-matching decoding of the logical
readout of the memory experiment, Z basis (logical |0>) or X basis (logical
|+>) (test infrastructure).

Follows the decoding procedure of Sec. III.B: syndromes of adjacent rounds
are XORed to locate flips, the flips are paired by minimum-weight perfect
matching (networkx, as in the paper), the recovery is applied, and the logical
Z is read from the final Z measurement of the data qubits.

Conventions (the readings used throughout the tests):
  * records are raw ancilla bits; the trivial bit of a check is r0 (w/2 mod 2
    for the cross-resonance circuit, 0 for the textbook circuit), so the
    syndrome is record XOR r0;
  * the logical operator is Z on the top row of data qubits (labels 1..d) --
    the printed Z1 Z7 Z13 Z19 Z25 anticommutes with X checks of Table I;
  * decoding graph: one node per (Z check, layer), layers 0..R-1 for the
    rounds plus layer R for the Z checks recomputed from the final data bits;
    a data qubit in two Z checks joins them within a layer, a data qubit in one
    Z check joins it to the boundary; consecutive layers of a check are joined
    (measurement errors); unit weights;
  * the checks of a round are measured one after another with the single
    ancilla (Sec. II.B), so an X error on a data qubit shared by Z checks A
    (measured first) and B that occurs between their measurements in round r
    flips B in layer r and A in layer r + 1: such a data qubit also joins
    (B, r) and (A, r + 1).
"""
import itertools

import networkx as nx
import numpy as np

from . import layout as _layout


class MemoryDecoder:
    """basis "Z": Z-check events, Z_L on the top row (logical |0> memory);
    basis "X": X-check events, X_L on the first column (logical |+> memory,
    final bits are X-basis outcomes).  The attribute names say z for the
    checks of the decoded type."""

    def __init__(self, d, rounds, gateset, basis="Z"):
        self.d, self.R = d, rounds
        stabs = _layout(d)
        self.zidx = [i for i, (t, _) in enumerate(stabs) if t == basis]
        self.zsup = [[q for q in stabs[i][1] if q] for i in self.zidx]
        self.r0 = np.array([(len(s) // 2) % 2 if gateset == 0 else 0 for s in self.zsup], dtype=np.uint8)
        self.zl = set(range(1, d + 1)) if basis == "Z" else set(1 + d * r for r in range(d))
        nz = len(self.zidx)
        B = "B"
        g = nx.Graph()
        owners = {}
        for k, sup in enumerate(self.zsup):
            for q in sup:
                owners.setdefault(q, []).append(k)
        for r in range(rounds + 1):
            for q, ks in owners.items():
                flip = 1 if q in self.zl else 0
                if len(ks) == 2:
                    g.add_edge((ks[0], r), (ks[1], r), flip=flip)
                    if r < rounds:  # ks[0] is measured before ks[1]
                        g.add_edge((ks[0], r + 1), (ks[1], r), flip=flip)
                else:
                    g.add_edge((ks[0], r), B, flip=flip)
            if r < rounds:
                for k in range(nz):
                    g.add_edge((k, r), (k, r + 1), flip=0)
        # shortest-path length and logical-flip parity between every pair
        self.dist, self.par = {}, {}
        for src in g.nodes:
            paths = nx.single_source_shortest_path(g, src)
            for dst, path in paths.items():
                p = 0
                for a, b in zip(path, path[1:]):
                    p ^= g.edges[a, b]["flip"]
                self.dist[src, dst] = len(path) - 1
                self.par[src, dst] = p

    def detectors(self, records, final_bits):
        """Detection events [n_z, R+1] from raw records [R, n_stab] and final bits [d*d]."""
        s = records[:, self.zidx] ^ self.r0
        fin = np.array([sum(int(final_bits[q - 1]) for q in sup) % 2 for sup in self.zsup], dtype=np.uint8)
        layers = np.vstack([s, fin[None, :]])
        prev = np.vstack([np.zeros_like(layers[:1]), layers[:-1]])
        return (layers ^ prev).T

    def logical_raw(self, final_bits):
        return sum(int(final_bits[q - 1]) for q in self.zl) % 2

    def correction(self, det):
        """Parity of the matched recovery on the logical Z support."""
        return self.matching(det)[0]

    def matching(self, det):
        """(parity of the matched recovery on Z_L, total path length of the
        matching)."""
        ev = [(k, r) for k, r in zip(*np.nonzero(det))]
        if not ev:
            return 0, 0
        g = nx.Graph()
        big = 10 * (len(ev) + 1) * (self.d + self.R + 2)
        for a, b in itertools.combinations(range(len(ev)), 2):
            g.add_edge(("e", a), ("e", b), weight=big - self.dist[ev[a], ev[b]])
        for a in range(len(ev)):
            g.add_edge(("e", a), ("b", a), weight=big - self.dist[ev[a], "B"])
        for a, b in itertools.combinations(range(len(ev)), 2):
            g.add_edge(("b", a), ("b", b), weight=big)
        m = nx.max_weight_matching(g, maxcardinality=True)
        p, w = 0, 0
        for u, v in m:
            if u[0] == "b" and v[0] == "b":
                continue
            if u[0] == "b":
                u, v = v, u
            if v[0] == "b":
                p ^= self.par[ev[u[1]], "B"]
                w += self.dist[ev[u[1]], "B"]
            else:
                p ^= self.par[ev[u[1]], ev[v[1]]]
                w += self.dist[ev[u[1]], ev[v[1]]]
        return p, w

    def failed(self, records, final_bits):
        """1 if the corrected logical reads -1."""
        det = self.detectors(records, final_bits)
        return self.logical_raw(final_bits) ^ self.correction(det)


ZDecoder = MemoryDecoder


def logical_error_rate(d, gateset, records, final_bits, basis="Z"):
    """Fraction of trajectories whose corrected logical (Z_L, or X_L for the
    X-basis memory) is -1."""
    R = records.shape[1]
    dec = MemoryDecoder(d, R, gateset, basis)
    fails = [dec.failed(records[i], final_bits[i]) for i in range(records.shape[0])]
    return float(np.mean(fails)), int(np.sum(fails))
