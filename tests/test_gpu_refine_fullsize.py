"""The refined benchmark forms at their full size, in the configuration the
benchmark times (the same levels, fields and refine_tree_step calls):
properties that hold at any size.  Over 10 coarsest steps the mass over all
levels, sum of M / 8^depth, is conserved (the scheme conserves it exactly;
FP32 storage within 1e-6), every level stays finite, and a second run from
the same start gives the same populations bit for bit.  Element-wise parity
of the exchange against the oracle is covered at small sizes."""
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

import bench  # noqa: E402


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    yield
    torch.cuda.empty_cache()


def _mass(tree, nodes):
    return sum(lat.totals()[0] / 8.0 ** cfg["depth"] for (lat, _, _), cfg in zip(tree, nodes))


def _checksums(tree):
    out = []
    for lat, _, _ in tree:
        bits = lat.get_pdfs().view(torch.int64)
        out.append((int(bits.sum()), int((bits * 3 + 7).sum())))
    return out


@pytest.mark.parametrize("key", list(bench.REFINED_FORMS))
def test_refined_form_conserves_mass_and_repeats_at_full_size(key):
    from paper_2305_09910_amd import lbm
    nodes = bench.refined_nodes(*bench.REFINED_FORMS[key])
    print(f"[case] {key}: " + ", ".join(f"{c['name']} {c['shape']}" for c in nodes), flush=True)
    runs = []
    for _ in range(2):
        tree = bench.make_refined(nodes)
        m0 = _mass(tree, nodes)
        lbm.refine_tree_step(tree, 10)
        m1 = _mass(tree, nodes)
        runs.append(_checksums(tree))
        for (lat, _, _), cfg in zip(tree, nodes):
            assert lat.time == 10 * 2 ** cfg["depth"]
            assert bool(torch.isfinite(lat.moments()[1]).all())
        del tree
        torch.cuda.empty_cache()
        print(f"{key}: mass {m0:.10e} -> {m1:.10e}, relative drift {abs(m1 - m0) / m0:.2e}")
        assert abs(m1 - m0) / m0 < 1e-6
    assert runs[0] == runs[1]
