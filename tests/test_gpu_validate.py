"""GPU parity of the read-only validation entry points (b64_validate,
b64_validate_async) against the oracle: the same decoded length or first
invalid offset as decoding, bit-exact, without writing any output."""
import numpy as np
import pytest

import workloads
from gpu_util import say, to_dev, to_host

pytestmark = pytest.mark.gpu

STD = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789+/"
URL = b"ABCDEFGHIJKLMNOPQRSTUVWXYZabcdefghijklmnopqrstuvwxyz0123456789-_"


@pytest.fixture(scope="module")
def b64():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    import paper_1910_05109_amd as b64
    b64.load()
    return b64


def _dev(a):
    import torch
    return to_dev(a) if a.size else torch.empty(0, dtype=torch.uint8, device="cuda")


def _check(b64, oracle, text, alpha=STD, label=""):
    say("validate", label, "n =", text.size)
    ref = oracle.decode_raw(text, alpha)
    length, bad = b64.validate(_dev(text), alpha)
    got = length if bad is None else ~bad
    assert got == ref, (label, got, ref)
    return got


def test_3mib_and_its_invalid_copy(b64, oracle):
    x = workloads.random_bytes(workloads.SEED_BASE + 1, workloads.SINGLE_3MIB)
    text = oracle.encode(x)
    assert _check(b64, oracle, text, label="3MiB") == x.size
    bad, pos = workloads.plant_invalid(text, workloads.SEED_BASE + 1, STD)
    assert _check(b64, oracle, bad, label="3MiB invalid") == ~pos
    st = to_host(b64.validate_async(to_dev(bad)))
    assert st.tolist() == [-1, pos]
    st = to_host(b64.validate_async(to_dev(text)))
    assert st.tolist() == [x.size, -1]


@pytest.mark.parametrize("alpha", [STD, URL], ids=["std", "url"])
def test_lengths_and_truncations(b64, oracle, alpha):
    data = workloads.random_bytes(workloads.SEED_BASE + 150, 2 * 1500)
    for n in range(0, 1500, 7):
        text = oracle.encode(data[n: 2 * n], alpha)
        _check(b64, oracle, text, alpha, f"len {n}")
        for cut in (1, 2, 3):
            if text.size >= cut:
                _check(b64, oracle, text[: text.size - cut], alpha, f"len {n} cut {cut}")


@pytest.mark.parametrize("where", ["first", "body", "final"])
def test_invalid_bytes_and_pads(b64, oracle, where):
    x = workloads.random_bytes(workloads.SEED_BASE + 151, 3 * 1500)
    text = oracle.encode(x)                          # 6000 characters
    q = {"first": 0, "body": 4 * 777, "final": 5996}[where]
    outside = [c for c in range(256) if c not in STD]
    for c in outside[::5] + [ord("="), ord("\n")]:
        for p in range(4):
            s = text.copy()
            s[q + p] = c
            _check(b64, oracle, s, label=f"{where} {c} {p}")
    for pattern in (b"AA==", b"AAA=", b"A===", b"AB==", b"AA=A", b"QQ==AAAA"):
        for qq in (0, 3, 4, 63, 64, 1400, (text.size - len(pattern)) // 4):
            s = text.copy()
            s[4 * qq: 4 * qq + len(pattern)] = np.frombuffer(pattern, dtype=np.uint8)
            _check(b64, oracle, s, label=f"{pattern!r} at {qq}")
            _check(b64, oracle, s[: 4 * qq + len(pattern)], label=f"{pattern!r} final at {qq}")


def test_misaligned_source(b64, oracle):
    x = workloads.random_bytes(workloads.SEED_BASE + 152, 30_000)
    t = oracle.encode(x)
    for so in range(16):
        hb = np.concatenate([np.zeros(so, np.uint8), t, np.zeros(16, np.uint8)])
        length, bad = b64.validate(to_dev(hb)[so: so + t.size])
        assert bad is None and length == x.size, so


def test_agrees_with_decode_on_random_damage(b64, oracle):
    """Random single-byte damage anywhere: validate and decode report the same."""
    x = workloads.random_bytes(workloads.SEED_BASE + 153, 9000)
    text = oracle.encode(x)
    g = workloads.rng(workloads.SEED_BASE + 154)
    for k in range(300):
        s = text.copy()
        s[g.integers(0, s.size)] = g.integers(0, 256)
        dec, dbad = b64.decode(to_dev(s))
        length, vbad = b64.validate(to_dev(s))
        assert vbad == dbad, k
        if dbad is None:
            assert length == dec.numel()


def test_1gib(b64, oracle):
    n = workloads.SINGLE_1GIB[0]
    say("validate 1GiB")
    x = workloads.random_bytes(workloads.SEED_BASE + 2, n)
    text = to_dev(oracle.encode(x))
    length, bad = b64.validate(text)
    assert bad is None and length == n
    pos = 1_000_000_007
    text[pos] = ord("!")
    length, bad = b64.validate(text)
    assert length is None and bad == pos
