"""The streaming-copy probes behind the roofline ceilings (pflbm_hbm_copy):
every form copies its whole buffer bit for bit, ragged sizes included (a
partial last block; a row length that is not a multiple of the block)."""
import ctypes as C

import pytest
import torch

from gpu_util import say

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("form, nbytes", [
    ("w4", 4 * 2048 * 3 + 16), ("w16", 16 * 1024 * 5 + 48), ("w16_cached", 16 * 1024 + 16),
    ("soa43", 43 * 4 * 1000), ("soa43_nt", 43 * 4 * 260),
    ("soa43_f64", 43 * 8 * 1000), ("soa43_f64_nt", 43 * 8 * 300)])
def test_copy_probe_copies_every_byte(form, nbytes):
    from paper_2206_11637_amd import _lib
    lib = _lib.load()
    say(f"case: copy probe {form} {nbytes} B")
    g = torch.Generator().manual_seed(nbytes)
    src = torch.randint(0, 256, (nbytes,), dtype=torch.uint8, generator=g).to("cuda")
    dst = torch.zeros_like(src)
    stream = torch.cuda.current_stream()
    _lib.check(lib.pflbm_hbm_copy(C.c_void_p(src.data_ptr()), C.c_void_p(dst.data_ptr()), nbytes,
                                  _lib.COPY_FORMS[form], C.c_void_p(stream.cuda_stream)), None, "pflbm_hbm_copy")
    torch.cuda.synchronize()
    assert torch.equal(src, dst)
