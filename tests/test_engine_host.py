"""Host logic of the GPU drivers without a GPU: the library's device calls are
replaced by stand-ins that keep a fake state's slot bookkeeping, so the
drivers' control flow (slot ownership on errors, per-measurement records)
runs on the CPU."""
import numpy as np
import pytest

from inputs import circuits as C


class _FakeState:
    def __init__(self, capacity):
        self.h, self.wmax, self.capacity = 1, 4, capacity
        self.free = list(range(capacity - 1, -1, -1))
        self.live = set()

    def alloc(self, k=1):
        from paper_2609_26516_amd import capi
        if len(self.free) < k:
            raise capi.DcsError(capi.DCS_ECAPACITY, "no free branch slot")
        out = [self.free.pop() for _ in range(k)]
        self.live.update(out)
        return out

    def release(self, ids):
        for i in ids:
            self.live.discard(int(i))
            self.free.append(int(i))

    # the driver-facing operations, routed to the (replaced) library calls
    bond_rule = True

    def _capi(self):
        from paper_2609_26516_amd import capi
        return capi

    def chunk(self, circ, op_ids):
        return 1

    def init_zero(self, ids, chis):
        self._capi().dcs_branch_init_zero(self.h, ids, chis, 0)

    def set_chi(self, ids, chis):
        self._capi().dcs_branch_set_chi(self.h, ids, chis)

    def compress(self, ids, chunks, n_sweeps):
        return self._capi().dcs_compress_step(self.h, ids, chunks, n_sweeps, 0)

    def measure(self, ids, qubits):
        return self._capi().dcs_measure_prob(self.h, ids, qubits, 0)

    def collapse(self, src, qubits, outcomes, dst, eps):
        return self._capi().dcs_collapse(self.h, src, qubits, outcomes, dst, eps, 0)


class _FakeEngine:
    def stream(self):
        return 0

    def chunk(self, circ, op_ids):
        return 1

    def span(self, circ, li):
        g = circ.ops[li].gate if isinstance(circ.ops[li], C.CGate) else circ.ops[li]
        return None if len(g.qubits) == 1 else (min(g.qubits), max(g.qubits), 4)


@pytest.fixture
def fake_lib(monkeypatch):
    E = pytest.importorskip("paper_2609_26516_amd.engine")
    capi = E.capi
    calls = {"compress": 0}
    monkeypatch.setattr(capi, "dcs_branch_init_zero", lambda *a: None)
    monkeypatch.setattr(capi, "dcs_branch_set_chi", lambda *a: None)

    def compress(h, ids, hs, s, stream):
        calls["compress"] += 1
        return np.full(len(ids), 0.9)

    monkeypatch.setattr(capi, "dcs_compress_step", compress)
    monkeypatch.setattr(capi, "dcs_measure_prob",
                        lambda h, ids, q, stream: np.full(len(ids), 0.25))
    monkeypatch.setattr(capi, "dcs_collapse",
                        lambda h, src, q, m, dst, eps, stream:
                        np.array([0.25 if x == 0 else 0.75 for x in m]))
    return E, calls


def test_multi_path_records_p0_per_measurement(fake_lib):
    E, _ = fake_lib
    circ, _ = C.workload("cfg3_n32_mp64", n=6, depth=4, chi=4)
    st = _FakeState(64)
    res = E.run_multi_path(_FakeEngine(), st, circ, 4, 100, 2, max_branches=3)
    nm = circ.n_measurements()
    assert len(res["branches"]) == 3
    for b in res["branches"]:
        assert b["p0s"] == [0.25] * nm
        pm = np.prod([0.25 if m == 0 else 0.75 for m in b["path"]])
        assert abs(b["p"] - pm) < 1e-15
    assert st.live == {b["id"] for b in res["branches"]}


def test_multi_path_releases_every_slot_on_error(fake_lib):
    """A host-side failure in the middle of a run (here the bond-cap draw of
    the children) releases the live branches and the children allocated so
    far before the exception propagates."""
    E, calls = fake_lib
    circ, _ = C.workload("cfg3_n32_mp64", n=6, depth=6, chi=4)
    st = _FakeState(64)
    seen = []

    def chi_of(path):
        seen.append(path)
        if len(path) == 3:
            raise RuntimeError("planted failure")
        return 4

    with pytest.raises(RuntimeError, match="planted failure"):
        E.run_multi_path(_FakeEngine(), st, circ, 4, 100, 2, chi_of=chi_of)
    assert calls["compress"] > 0 and any(len(p) == 3 for p in seen)
    assert st.live == set()
    assert sorted(st.free) == list(range(64))


def test_multi_path_releases_on_capacity_error(fake_lib):
    E, _ = fake_lib
    circ, _ = C.workload("cfg3_n32_mp64", n=6, depth=6, chi=4)
    st = _FakeState(5)
    from paper_2609_26516_amd import capi
    with pytest.raises(capi.DcsError):
        E.run_multi_path(_FakeEngine(), st, circ, 4, 100, 2)
    assert st.live == set() and sorted(st.free) == list(range(5))
