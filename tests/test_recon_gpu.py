"""What the trained network gains (clinical case, held-out phantom, Poisson
I0 = 1e5): the committed multiscale primal-dual net (8 iterations, FDK start)
against CGLS on the same FP32 projector pair and against the same net with
its blocks zeroed (only the output convolutions act).

Pass criteria: the net's final PSNR is at least CGLS's best over 50
iterations (a CGLS stopped by an oracle that knows the truth); it reaches that
PSNR in less wall time than CGLS; and its blocks add at least 5 dB over the
zero-block net.  The net's quality itself is not pinned to any reference
(there are no reference weights)."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def setup():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    torch.cuda.set_device(0)
    from paper_2512_21180_amd import compare
    return compare, compare.Setup(compare.DEFAULT_WEIGHTS)


def test_learned_net_beats_cgls_and_its_zero_block_version(setup):
    compare, S = setup
    print("[recon] held-out phantom 50001", flush=True)
    r = compare.compare_one(S, 50_001, log=lambda m: print(m, flush=True))
    learned = r["learned_psnr_db"][-1]
    assert learned >= r["target_psnr_db"], r
    assert r["learned_time_to_target_s"] is not None
    assert r["learned_time_to_target_s"] < r["cgls_time_to_target_s"], r
    assert learned >= r["zero_block_psnr_db"][-1] + 5.0, r
    # PSNR rises over the iterations of each resolution level
    assert r["learned_psnr_db"][-1] > r["learned_psnr_db"][0]
