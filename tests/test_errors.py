"""Error paths of dfa_create that are decided before any device is touched
(Section 2.1: the automaton (Q, Sigma, delta, q0, F) must have a total delta
into Q, q0 in Q and F a subset of Q): each invalid automaton is refused with
DFA_E_INVAL and no handle.  Runs without a GPU."""
import ctypes

import numpy as np
import pytest

import paper_1210_5093_amd as dfa


def create(delta, nq, nsym, q0, acc, b2s):
    L = dfa.lib()
    h = ctypes.c_void_p()
    d = None if delta is None else np.ascontiguousarray(delta, dtype=np.uint32)
    a = None if acc is None else np.ascontiguousarray(acc, dtype=np.uint32)
    m = None if b2s is None else np.ascontiguousarray(b2s, dtype=np.uint8)
    rc = L.dfa_create(None if d is None else d.ctypes.data, nq, nsym, q0,
                      None if a is None else a.ctypes.data, 0 if a is None else int(a.size),
                      None if m is None else m.ctypes.data, ctypes.byref(h))
    return rc, h.value, dfa.lib().dfa_last_error().decode()


GOOD = np.array([[1, 0], [1, 1]], dtype=np.uint32)       # 2 states, 2 symbols
MAP = np.full(256, 0xFF, dtype=np.uint8)
MAP[ord("a")], MAP[ord("b")] = 0, 1


@pytest.mark.parametrize("case,args,msg", [
    ("null delta", (None, 2, 2, 0, [1], MAP), "delta is NULL"),
    ("no states", (GOOD, 0, 2, 0, [1], MAP), "num_states"),
    ("too many states", (np.zeros((32768, 1), np.uint32), 32768, 1, 0, [0], MAP), "num_states"),
    ("no symbols", (GOOD, 2, 0, 0, [1], MAP), "num_symbols"),
    ("too many symbols", (np.zeros((2, 257), np.uint32), 2, 257, 0, [1], MAP), "num_symbols"),
    ("q0 outside Q", (GOOD, 2, 2, 2, [1], MAP), "q0"),
    ("delta leaves Q", (np.array([[1, 2], [0, 1]]), 2, 2, 0, [1], MAP), "delta entry"),
    ("F not in Q", (GOOD, 2, 2, 0, [5], MAP), "accepting state"),
    ("identity map needs 256 symbols", (GOOD, 2, 2, 0, [1], None), "byte_to_symbol"),
])
def test_dfa_create_rejects_invalid_automata(case, args, msg):
    rc, h, err = create(*args)
    assert rc == dfa.DFA_E_INVAL, case
    assert h is None, case
    assert msg in err, (case, err)


def test_null_accepting_with_a_count():
    L = dfa.lib()
    h = ctypes.c_void_p()
    d = GOOD.copy()
    rc = L.dfa_create(d.ctypes.data, 2, 2, 0, None, 3, MAP.ctypes.data, ctypes.byref(h))
    assert rc == dfa.DFA_E_INVAL and h.value is None


def test_null_out_pointer():
    L = dfa.lib()
    d = GOOD.copy()
    assert L.dfa_create(d.ctypes.data, 2, 2, 0, None, 0, MAP.ctypes.data, None) == dfa.DFA_E_INVAL


def test_binding_raises_with_the_status():
    with pytest.raises(dfa.DFAError) as e:
        dfa.DFA(np.array([[0, 3]], dtype=np.uint32), 0, [0], MAP)
    assert e.value.status == dfa.DFA_E_INVAL


def test_status_strings():
    L = dfa.lib()
    for st, text in [(dfa.DFA_E_INVAL, b"invalid argument"),
                     (dfa.DFA_E_TOOBIG, b"exceeds a device limit"),
                     (dfa.DFA_E_SPECULATION, b"speculation invariant violated"),
                     (dfa.DFA_E_SYMBOL, b"input byte outside the alphabet")]:
        assert L.dfa_strerror(st) == text
