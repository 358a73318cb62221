"""Host-side normalisation of the pair histograms into g_ab(r) (engine)
against the oracle's, on counts the oracle computed.  CPU only."""
import numpy as np

from paper_2409_04430_amd import inputs as I


def test_engine_normalisation_matches_oracle(orc):
    from paper_2409_04430_amd.engine import rdf_normalise
    rng = np.random.default_rng(9)
    p0, types, box = I.rocksalt(3, 4.2)
    types = np.asarray(types)
    pos = p0[None] + rng.normal(0.0, 0.1, (3,) + p0.shape)
    c = orc.rdf_counts(pos, types, box, 5.0, 50, 2)
    n_sp = [int((types == a).sum()) for a in range(2)]
    V = float(np.prod(box))
    r1, g1 = rdf_normalise(c, n_sp, V, 5.0, 2, 3)
    r2, g2 = orc.rdf_normalise(c, n_sp, V, 5.0, frames=2, P=3)
    np.testing.assert_allclose(r1, r2, rtol=1e-14)
    np.testing.assert_allclose(g1, g2, rtol=1e-12)
    assert g1[0, 1].max() > 1.0
