"""kw_create_static (the spectral scratch arrays in the library's static
array) against kw_create (the same arrays in the caller's workspace), through
the C ABI: two set-ups in a row, the second on a smaller grid, every recorded
output equal bit for bit (the same kernels run in the same order on the same
values; only the scratch addresses differ)."""
import numpy as np
import pytest

from paper_1408_4675_amd import scenarios as sc

pytestmark = pytest.mark.gpu


def _outputs(sim, scen):
    from paper_1408_4675_amd import _abi as A
    whats = [A.KW_REC_P_FINAL, A.KW_REC_U_FINAL, A.KW_REC_P_MAX, A.KW_REC_P_RMS]
    if scen.sensor.record & sc.REC_P_SERIES:
        whats.append(A.KW_REC_P_SERIES)
    return {w: sim.gather(w, device=False) for w in whats}


def test_static_scratch_matches_workspace_scratch():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_1408_4675_amd import _abi as A
    from paper_1408_4675_amd.simulation import Simulation, static_workspace_size, workspace_size
    cases = [sc.small_case(96, 96, 96, seed=3, steps=12, sensor_mask=True, n_elements=2),
             sc.small_case(40, 36, 30, seed=4, steps=10)]
    for scen in cases:
        print("\n[case] static scratch %s" % scen.name, flush=True)
        ref = Simulation(scen)
        ref.step(scen.steps)
        want = _outputs(ref, scen)
        ref.close()
        st = Simulation(scen, static_scratch=True)
        assert st.stats()["workspace_bytes"] == static_workspace_size(scen) < workspace_size(scen)
        st.step(scen.steps)
        got = _outputs(st, scen)
        st.close()
        for w in want:
            assert np.array_equal(got[w], want[w]), (scen.name, w)
    # a grid whose six spectra exceed the static array is refused before any device work
    big = sc.small_case(256, 256, 256, seed=1, steps=1, heterogeneous=False)
    with pytest.raises(A.KwError) as e:
        Simulation(big, static_scratch=True)
    assert e.value.code == A.KW_EUNSUPPORTED
