"""The Python binding on the CPU: an output or plan buffer of the wrong shape or
word size is refused with ValueError before the library is called (the C ABI
carries no buffer sizes, so such a buffer would be written past its end)."""
import pytest
import torch

import paper_2307_06554_amd as pm


def t32(*shape):
    return torch.zeros(shape, dtype=torch.int32)


def t64(*shape):
    return torch.zeros(shape, dtype=torch.int64)


Q = 3329
QS = [3329, 7681]

# (call, a valid-shaped out, a wrong one): the wrong ones are one word short or the wrong word size
CASES = [
    ("negacyclic", lambda out: pm.polymul_negacyclic(t32(3, 64), t32(3, 64), Q, out=out)),
    ("plain", lambda out: pm.polymul_negacyclic_plain(t32(3, 64), t32(3, 64), Q, out=out)),
    ("u64", lambda out: pm.polymul_negacyclic_u64(t64(3, 64), t64(3, 64), Q, out=out)),
    ("cyclic", lambda out: pm.polymul_cyclic(t32(3, 64), t32(3, 64), Q, out=out)),
    ("cyclic_u64", lambda out: pm.polymul_cyclic_u64(t64(3, 64), t64(3, 64), Q, out=out)),
    ("rns", lambda out: pm.polymul_negacyclic_rns(t32(3, 2, 64), t32(3, 2, 64), QS, out=out)),
    ("crt", lambda out: pm.polymul_negacyclic_crt(t32(3, 64), t32(3, 64), Q, out=out)),
    ("rns_crt", lambda out: pm.polymul_negacyclic_rns_crt(t32(3, 2, 64), t32(3, 2, 64), QS, out=out)),
    ("shared", lambda out: pm.polymul_negacyclic_shared(t32(3, 64), t32(64), Q, out=out)),
    ("u64_shared", lambda out: pm.polymul_negacyclic_u64_shared(t64(3, 64), t64(64), Q, out=out)),
    ("rns_shared", lambda out: pm.polymul_negacyclic_rns_shared(t32(3, 2, 64), t32(2, 64), QS, out=out)),
    ("rns_karatsuba", lambda out: pm.polymul_negacyclic_rns_karatsuba(t32(3, 2, 64), t32(3, 2, 64), QS, 2,
                                                                        out=out)),
    ("u64_karatsuba", lambda out: pm.polymul_negacyclic_u64_karatsuba(t64(3, 64), t64(3, 64), Q, 2, out=out)),
]
SHAPES = {"negacyclic": (3, 64), "plain": (3, 64), "u64": (3, 64), "cyclic": (3, 64), "cyclic_u64": (3, 64),
          "rns": (3, 2, 64), "crt": (3, 64), "rns_crt": (3, 2, 64), "shared": (3, 64), "u64_shared": (3, 64),
          "rns_shared": (3, 2, 64), "rns_karatsuba": (3, 2, 64), "u64_karatsuba": (3, 64)}
WIDE = {"u64", "cyclic_u64", "u64_shared", "u64_karatsuba"}


@pytest.mark.parametrize("name,call", CASES, ids=[c[0] for c in CASES])
def test_short_output_refused(name, call):
    shape = list(SHAPES[name])
    shape[-1] -= 1
    out = torch.zeros(shape, dtype=torch.int64 if name in WIDE else torch.int32)
    with pytest.raises(ValueError, match="shape"):
        call(out)


@pytest.mark.parametrize("name,call", CASES, ids=[c[0] for c in CASES])
def test_flat_output_refused(name, call):
    # the right number of words in the wrong shape is refused too
    shape = SHAPES[name]
    numel = 1
    for s in shape:
        numel *= s
    out = torch.zeros((numel,), dtype=torch.int64 if name in WIDE else torch.int32)
    with pytest.raises(ValueError, match="shape"):
        call(out)


@pytest.mark.parametrize("name,call", CASES, ids=[c[0] for c in CASES])
def test_wrong_word_size_refused(name, call):
    out = torch.zeros(SHAPES[name], dtype=torch.int32 if name in WIDE else torch.int64)
    with pytest.raises(ValueError, match="bit integer words"):
        call(out)


def test_plan_group_buffers_checked():
    a = t32(4, 256)
    with pytest.raises(ValueError, match="same shape"):
        pm.polymul_plan_create([(a, t32(4, 256), t32(3, 256), 256, Q)])
    with pytest.raises(ValueError, match="same shape"):
        pm.polymul_plan_create([(a, t32(4, 128), t32(4, 256), 256, Q)])
    with pytest.raises(ValueError, match="same size"):
        pm.polymul_plan_create([(a, t32(4, 256), torch.zeros((4, 256), dtype=torch.int16), 256, Q)])
    with pytest.raises(ValueError, match="whole polynomials"):
        pm.polymul_plan_create([(t32(5, 100), t32(5, 100), t32(5, 100), 256, Q)])
    with pytest.raises(ValueError, match="32 or 64 bits"):
        h = torch.zeros((4, 256), dtype=torch.int16)
        pm.polymul_plan_create([(h, h, h, 256, Q)])
