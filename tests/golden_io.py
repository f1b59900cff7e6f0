"""Reader for the worked-example fixtures under tests/golden/."""
import glob
import os

import numpy as np

import qcw_inputs as qi

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")

NAMED = {"H": qi.H, "X": qi.X, "Y": qi.Y, "Z": qi.Z, "CNOT": qi.CNOT, "CZ": qi.CZ,
         "SWAP": qi.SWAP, "TOFFOLI": qi.TOFFOLI}


class Golden:
    def __init__(self, path):
        self.name = os.path.basename(path)
        self.nq = None
        self.init = None
        self.circ = None
        self.expect = {}
        self.zero_elsewhere = False
        self.exact_zeros = False
        with open(path) as f:
            for line in f:
                line = line.split("#", 1)[0].strip()
                if not line:
                    continue
                w = line.split()
                if w[0] == "nq":
                    self.nq = int(w[1])
                    self.circ = qi.Circuit(self.nq)
                elif w[0] == "init":
                    assert w[1] == "basis"
                    self.init = qi.basis_state(self.nq, int(w[2]))
                elif w[0] == "gate":
                    self.circ.add(NAMED[w[1]], *[int(x) for x in w[2:]])
                elif w[0] == "expect":
                    self.expect[int(w[1])] = complex(float(w[2]), float(w[3]))
                elif w[0] == "zero_elsewhere":
                    self.zero_elsewhere = True
                elif w[0] == "exact_zeros":
                    self.zero_elsewhere = self.exact_zeros = True
                else:
                    raise ValueError(f"{path}: bad directive {w[0]}")

    def check(self, psi, tol=4 * 2.0 ** -53):
        """Assert psi matches; tol is absolute (a few ulp of unit-size values)."""
        psi = np.asarray(psi)
        for n, v in self.expect.items():
            assert abs(psi[n] - v) <= tol, (self.name, n, psi[n], v)
        if self.zero_elsewhere:
            mask = np.ones(psi.size, bool)
            mask[list(self.expect)] = False
            if self.exact_zeros:
                assert np.all(psi[mask] == 0), (self.name, np.nonzero(psi[mask]))
            else:
                assert np.all(np.abs(psi[mask]) <= tol), (self.name, np.abs(psi[mask]).max())


def all_golden():
    return [Golden(p) for p in sorted(glob.glob(os.path.join(GOLDEN, "*.txt")))
            if not p.endswith("README.txt")]
