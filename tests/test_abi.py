"""C ABI checks that need no GPU: the library loads, exports every declared
entry point, and its host copy of the hash equals the oracle's."""
import ctypes
import os
import re

import numpy as np
import pytest

import datagen
import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_entry_points():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(bht_\w+)\s*\(", text))
    return sorted(names)


def test_library_exports_every_declared_symbol():
    import paper_2108_07232_amd as bht
    lib = ctypes.CDLL(bht.LIB_PATH)
    missing = [n for n in declared_entry_points() if not hasattr(lib, n)]
    assert not missing, missing
    assert set(declared_entry_points()) <= set(bht.EXPORTED)


def test_status_strings():
    import paper_2108_07232_amd as bht
    assert bht.bht_status_string(bht.BHT_OK) == "ok"
    assert "failed" in bht.bht_status_string(bht.BHT_ERR_BUILD_FAILED)


EDGE_K = [0, 1, 2, 5, 4294967290, 4294967291, 4294967292, 4294967294, 0xFFFFFFFF, 123456789]
EDGE_M = [1, 2, 3, 16, 72818, 18641352, 9320676, (1 << 31) - 1, 0xFFFFFFFF]


def test_library_hash32_equals_oracle():
    import paper_2108_07232_amd as bht
    P = 4294967291
    consts = [(1, 0), (P - 1, P - 1), (2, 3), (P - 1, 0), (1, P - 1)]
    consts += list(zip(*datagen.hash_constants(4, 4)))
    for a, c in consts:
        for k in EDGE_K:
            for m in EDGE_M:
                assert bht.bht_hash32(a, c, k, m) == oracle.hash32(a, c, k, m), (a, c, k, m)
    rng = np.random.default_rng(0)
    for _ in range(3000):
        a, c = int(rng.integers(1, P)), int(rng.integers(0, P))
        k, m = int(rng.integers(0, 1 << 32)), int(rng.integers(1, 1 << 32))
        assert bht.bht_hash32(a, c, k, m) == oracle.hash32(a, c, k, m)


def test_library_hash32_quotient_boundaries():
    """The bucket reduction takes r mod m from a fixed-point reciprocal of m
    (no division); a wrong quotient would first show at multiples of m.
    With a = 1, c = 0 the residue r equals the key (k < p), so keys at
    q m - 1, q m, q m + 1 and q m + m - 1 probe those boundaries for
    divisors of every size, powers of two and the two sides of 2^31 among
    them."""
    import paper_2108_07232_amd as bht
    P = 4294967291
    rng = np.random.default_rng(7)
    ms = [1, 2, 3, 5, 7, 16, 1000, 72818, 9320676, 18641352, 167772160, (1 << 30) + 3,
          (1 << 31) - 1, 1 << 31, (1 << 31) + 1, 3000000019, 0xFFFFFFFE, 0xFFFFFFFF]
    ms += [1 << s for s in range(1, 32)]
    ms += [int(x) for x in rng.integers(1, 1 << 32, 40)]
    for m in ms:
        qmax = (P - 1) // m
        qs = {0, 1, qmax, max(qmax - 1, 0)} | {int(x) for x in rng.integers(0, qmax + 1, 30)}
        for q in qs:
            for r in (q * m - 1, q * m, q * m + 1, q * m + m - 1):
                if 0 <= r < P:
                    assert bht.bht_hash32(1, 0, r, m) == r % m, (r, m)


def test_diagnostics_reject_bad_buffers_before_touching_the_device():
    import paper_2108_07232_amd as bht
    lib = bht._lib
    sink = ctypes.c_void_p(256)
    assert lib.bht_diag_stream(None, None, 1 << 20, sink, None) == bht.BHT_ERR_INVALID_ARG
    assert lib.bht_diag_stream(ctypes.c_void_p(256), None, 8, sink, None) == bht.BHT_ERR_INVALID_ARG
    assert lib.bht_diag_stream(ctypes.c_void_p(264), None, 1 << 20, sink, None) == bht.BHT_ERR_INVALID_ARG
    assert lib.bht_diag_stream(ctypes.c_void_p(256), ctypes.c_void_p(260), 1 << 20, sink,
                               None) == bht.BHT_ERR_INVALID_ARG
    assert lib.bht_diag_stream(ctypes.c_void_p(256), None, 1 << 20, None, None) == bht.BHT_ERR_INVALID_ARG


def test_library_hash64_equals_oracle():
    import paper_2108_07232_amd as bht
    Q = (1 << 61) - 1
    rng = np.random.default_rng(1)
    edge_k = [0, 1, Q - 1, Q, Q + 1, (1 << 64) - 2, (1 << 63), 0x123456789ABCDEF]
    edge_m = [1, 2, 8, 18641352, (1 << 32) - 1, (1 << 40) + 7]
    for a, c in [(1, 0), (Q - 1, Q - 1), (2, 3)] + list(zip(*datagen.hash_constants64(2, 3))):
        for k in edge_k:
            for m in edge_m:
                assert bht.bht_hash64(a, c, k, m) == oracle.hash64(a, c, k, m), (a, c, k, m)
    for _ in range(2000):
        a, c = int(rng.integers(1, Q)), int(rng.integers(0, Q))
        k = int(rng.integers(0, 1 << 63)) * 2 + int(rng.integers(0, 2))
        m = int(rng.integers(1, 1 << 40))
        assert bht.bht_hash64(a, c, k, m) == oracle.hash64(a, c, k, m)


def test_product_path_never_imports_the_oracle():
    pkg = os.path.join(ROOT, "paper_2108_07232_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                for banned in ("import oracle", "from oracle", "liboracle", "oracle.h",
                               "import datagen", "from datagen"):
                    assert banned not in text, (fn, banned)


def test_create_rejects_bad_parameters_before_touching_the_device():
    import paper_2108_07232_amd as bht
    a, c = datagen.hash_constants(1, 3)
    cases = [
        ("bcht", 16, dict(a=a, b=c, key_bits=16)),         # key width
        ("bcht", 12, dict(a=a, b=c)),                       # bucket size
        ("cht1", 4, dict(a=a, b=c)),                        # single-slot scheme
        ("bp2ht", 16, dict(a=a, b=c)),                      # needs two hashes
        ("iht", 8, dict(a=a, b=c)),                         # bucket size
        ("iht", 16, dict(a=a, b=c, iht_threshold=17)),      # threshold above b
        ("iht", 16, dict(a=a, b=c, iht_secondary_b=4, iht_secondary_m=10)),
        ("bcht", 16, dict(a=[0, 1, 2], b=[0, 0, 0])),       # a must be >= 1
        ("bcht", 16, dict(a=[4294967291, 1, 2], b=[0, 0, 0])),  # a must be < p
    ]
    for scheme, bsz, kw in cases:
        p = bht.make_params(**kw)
        with pytest.raises(bht.BhtError) as e:
            bht.bht_create(1000, bsz, scheme, p)
        assert e.value.status in (bht.BHT_ERR_INVALID_ARG, bht.BHT_ERR_UNSUPPORTED), (scheme, bsz, kw)


def _splitmix64(state):
    """Steele, Lea and Flood's splitmix64 step on a Python integer state."""
    state = (state + 0x9E3779B97F4A7C15) & (2**64 - 1)
    z = state
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & (2**64 - 1)
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & (2**64 - 1)
    return state, z ^ (z >> 31)


def test_splitmix64_reference_value():
    # first output of splitmix64 from state 0, as published with the generator
    assert _splitmix64(0)[1] == 0xE220A8397B1DCDAF


def test_params_from_seed_draws_in_range_and_is_deterministic():
    import paper_2108_07232_amd as bht
    P32, P61 = 4294967291, (1 << 61) - 1
    seen = set()
    for seed in range(200):
        for scheme, h in (("bcht", 3), ("bp2ht", 2), ("iht", 3), ("cht1", 3)):
            for bits, prime in ((32, P32), (64, P61)):
                p = bht.bht_params_from_seed(seed, scheme, bits)
                assert p.num_hashes == h and p.key_bits == bits and p.max_chain == 128
                assert p.rng_seed != 0 and p.iht_secondary_b == 0
                for i in range(4):
                    assert 1 <= p.a[i] < prime and 0 <= p.b[i] < prime
                q = bht.bht_params_from_seed(seed, scheme, bits)
                assert list(p.a) == list(q.a) and list(p.b) == list(q.b)
                seen.add((bits, p.a[0]))
    assert len(seen) == 400                 # distinct seeds give distinct constants
    with pytest.raises(bht.BhtError):
        bht.bht_params_from_seed(1, "bcht", 16)


def test_params_from_seed_follows_rejection_from_splitmix64():
    """The constants are the accepted draws of the documented stream:
    32-bit draws (top half) for p = 2^32 - 5, 61-bit draws for 2^61 - 1."""
    import paper_2108_07232_amd as bht
    for bits, prime, shift in ((32, 4294967291, 32), (64, (1 << 61) - 1, 3)):
        for seed in (0, 1, 12345, 2**64 - 1):
            st = seed ^ 0x5EEDC0457A27
            a, c = [], []
            for _ in range(4):
                while True:
                    st, x = _splitmix64(st)
                    x >>= shift
                    if 1 <= x < prime:
                        break
                a.append(x)
                while True:
                    st, x = _splitmix64(st)
                    x >>= shift
                    if x < prime:
                        break
                c.append(x)
            p = bht.bht_params_from_seed(seed, "bcht", bits)
            assert list(p.a) == a and list(p.b) == c


def test_build_retry_rejects_bad_arguments_on_the_host():
    import paper_2108_07232_amd as bht
    st = bht._lib.bht_build_retry(None, None, None, 0, 0, 1, None, None)
    assert st == bht.BHT_ERR_INVALID_ARG
