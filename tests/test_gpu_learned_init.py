"""What the learned initialisation gains over the plain heuristic (an
empirical claim, parity unpinned): trained by the project's kernels on
converged parameters the plain mapper produced on three training scenes, it
reaches on held-out scenes the PSNR the heuristic needs many more window
iterations for, and ends a fixed iteration budget ahead."""
import pytest

from paper_2504_02437_amd import init_mlp as IM

pytestmark = pytest.mark.gpu


def test_learned_initialisation_beats_heuristic_on_held_out_scenes():
    print("case learned init", flush=True)
    res, net = IM.experiment(train_seeds=range(3), eval_seeds=(2000, 2001),
                             n_kf=20, epochs=10, log=print)
    assert res["pairs"] > 20000
    assert res["train_loss"][-1] < 0.5 * res["train_loss"][0]
    for ev in res["evals"]:
        h, m = ev["heuristic"], ev["learned"]
        it0, p0 = m[0]
        # The heuristic needs more iterations to reach the learned start.
        need = IM.iterations_to_reach(h, p0)
        assert need is None or need > it0, (ev["seed"], need, it0)
        # And ends the same budget at least 1 dB lower.
        assert m[-1][1] > h[-1][1] + 1.0, (ev["seed"], m[-1], h[-1])
