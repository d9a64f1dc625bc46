"""Host side of the registration checkpoint: the state file round trip
(parameters, Adam moments, step count and pyramid level), read back with
numpy's loader that executes nothing from the file."""
import numpy as np

from paper_1806_09907_amd.registration import RegistrationState


def test_state_round_trip(tmp_path):
    rng = np.random.default_rng(5)
    th = rng.normal(size=(2, 11, 11)).astype(np.float32)
    st = RegistrationState(theta=th, m=0.1 * th, v=th * th, step=123, level=2)
    path = str(tmp_path / "s.npz")
    st.save(path)
    back = RegistrationState.load(path)
    assert back.step == 123 and back.level == 2
    for a, b in ((back.theta, th), (back.m, 0.1 * th), (back.v, th * th)):
        assert a.dtype == np.float32 and np.array_equal(a, b.astype(np.float32))
