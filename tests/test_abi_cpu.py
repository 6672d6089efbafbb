"""Host-side checks of the C ABI that need no GPU: the library loads, exports every function
declared in include/handtrack.h, validates model tables and rejects bad arguments."""
import ctypes as C

import numpy as np
import pytest

import paper_2005_07068_amd as ht
from paper_2005_07068_amd import binding
from workload import make_hand_model


def test_library_exports_every_declared_function():
    lib = ht.load_library()
    names = ht.header_functions()
    assert len(names) >= 15
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing
    assert lib.ht_version().decode().startswith("handtrack")


@pytest.mark.parametrize("n_hands", [1, 2])
@pytest.mark.parametrize("prims", ["cylinders", "paper"])
def test_model_tables_validate(n_hands, prims):
    binding.check_model(make_hand_model(3, n_hands, prims))


@pytest.mark.parametrize("kind,index", [("cone", 2), ("ecyl", 0), ("ecyl", 2)])
def test_paper_primitive_sizes_validated(kind, index):
    """A truncated cone needs both radii and the length, an elliptic cylinder both semi-axes
    and the length, all positive."""
    from workload import CONE, ECYLINDER
    m = make_hand_model(4, 1, "paper")
    m = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in m.items()}
    k = int(np.nonzero(m["prim_type"] == (CONE if kind == "cone" else ECYLINDER))[0][0])
    m["prim_size"][k, index] = 0.0
    with pytest.raises(binding.HandtrackError):
        binding.check_model(m)


def _broken(mutate):
    m = make_hand_model(4)
    m = {k: (v.copy() if isinstance(v, np.ndarray) else v) for k, v in m.items()}
    mutate(m)
    return m


@pytest.mark.parametrize("mutate", [
    lambda m: m["seg_parent"].__setitem__(2, 5),               # parent after child
    lambda m: m["seg_joint_axis"].__setitem__((3, 0), [1.0, 1.0, 0.0]),   # not unit
    lambda m: m["seg_joint_dof"].__setitem__((3, 0), 99),       # dof out of range
    lambda m: m["prim_size"].__setitem__((7, 0), 0.0),          # zero radius
    lambda m: m["prim_type"].__setitem__(5, 7),                 # unknown type
    lambda m: m["prim_seg"].__setitem__(5, 40),                 # segment out of range
    lambda m: m["bounds_lo"].__setitem__(3, 9.0),               # lo > hi
    lambda m: m["kc_pairs"].__setitem__((0, 1), -3),            # bad pair
    lambda m: m["seg_joint_dof"].__setitem__((4, 1), 0),        # dof 0 drives two joints
])
def test_model_validation_rejects(mutate):
    with pytest.raises(binding.HandtrackError) as e:
        binding.check_model(_broken(mutate))
    assert e.value.status == binding.HT_ERR_ARG
    assert len(str(e.value)) > 12


def test_null_arguments_and_destroy_null():
    lib = ht.load_library()
    lib.ht_destroy(None)
    assert lib.ht_check_model(None) == binding.HT_ERR_ARG
    assert lib.ht_create(None, 0) == binding.HT_ERR_ARG
    assert lib.ht_set_model(None, None) == binding.HT_ERR_ARG
    assert lib.ht_eval_particles(None, 1, None, 1, None, None, None, None) == binding.HT_ERR_ARG
    assert lib.ht_pso_step(None, None, None, None) == binding.HT_ERR_ARG
    assert b"NULL" in lib.ht_last_error()
    lc = binding.LaunchConfig()
    assert lib.ht_get_launch_config(None, C.byref(lc)) == binding.HT_ERR_ARG


def test_create_without_device_fails_cleanly():
    torch = pytest.importorskip("torch")
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = C.c_void_p()
    st = ht.load_library().ht_create(C.byref(h), 0)
    assert st in (binding.HT_ERR_ARG, binding.HT_ERR_HIP)
    assert not h.value
