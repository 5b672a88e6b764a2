"""The product path has no CPU fallback: without the built HIP library it
raises, and host tensors are rejected instead of being computed on the CPU."""
import numpy as np
import pytest
import torch

from paper_1912_10024_amd import _lib, sse
from paper_1912_10024_amd.inputs import CONFIGS, generate


def test_missing_library_raises(monkeypatch, tmp_path):
    monkeypatch.setattr(_lib, "LIB_PATH", str(tmp_path / "absent" / "libsse.so"))
    monkeypatch.setattr(_lib, "_lib", None)
    with pytest.raises(RuntimeError, match="missing"):
        _lib.load()


@pytest.mark.parametrize("call", ["forward", "forward_signed", "backward", "phonon_forward"])
def test_host_tensors_are_rejected(call):
    d = CONFIGS["tiny"]
    inp = {k: torch.from_numpy(v) for k, v in generate(d, 0, which=("nbr", "G<", "D<", "dH", "W")).items()}
    G, D, dH, nbr = inp["G<"], inp["D<"], inp["dH"], inp["nbr"]
    with pytest.raises(ValueError, match="HIP device"):
        if call == "forward":
            sse.forward(G, D, dH, nbr)
        elif call == "forward_signed":
            sse.forward_signed(G, D, D.clone(), dH, nbr)
        elif call == "backward":
            sse.backward(G, D, dH, nbr, inp["W"].conj().transpose(-1, -2).contiguous())
        else:
            sse.phonon_forward(G, G, dH, nbr, d.nqz, d.nw)
