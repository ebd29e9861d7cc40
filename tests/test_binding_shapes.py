"""The binding rejects tensors whose shapes disagree with the sizes it passes
to the library, before any device check or library call (no GPU needed:
the tensors here are host tensors, so a call that got past the shape checks
stops at the device check instead)."""
import pytest
import torch

import paper_1705_07272_amd as rrt

N = 8
V = 5
NNZ = 70            # two 64-value scale blocks
K = 16


def z(*shape, dtype=torch.float32):
    return torch.zeros(shape, dtype=dtype)


def base(**over):
    a = dict(n=N, light_idx=z(K, dtype=torch.int32), light_val=z(K), vert_rot=z(V, 3, 3),
             t_idx=z(V, NNZ, dtype=torch.int32), t_val=z(V, NNZ))
    a.update(over)
    return a


def shape_error(fn, *args, **kw):
    with pytest.raises(ValueError) as e:
        fn(*args, **kw)
    assert "device" not in str(e.value), str(e.value)
    return str(e.value)


def reaches_device_check(fn, *args, **kw):
    with pytest.raises(ValueError, match="device tensor"):
        fn(*args, **kw)


def test_relight_well_formed_reaches_device_check():
    reaches_device_check(rrt.relight, **base())
    reaches_device_check(rrt.relight, **base(t_val=z(V, NNZ, dtype=torch.uint8),
                                              block_scale=z(V, 2)))
    reaches_device_check(rrt.relight, **base(t_idx=z(3, NNZ, dtype=torch.int32),
                                              cluster=z(V, dtype=torch.int32)))
    reaches_device_check(rrt.relight, **base(frame_rot=z(4, 3, 3), out=z(4, V)))


@pytest.mark.parametrize("over", [
    dict(t_val=z(V + 1, NNZ)),                                   # rows != vertices
    dict(t_idx=z(V, NNZ - 1, dtype=torch.int32)),                # idx / val row length
    dict(t_idx=z(V - 1, NNZ, dtype=torch.int32)),                # idx rows
    dict(t_val=z(V, NNZ, dtype=torch.uint8)),                    # codes without scales
    dict(t_val=z(V, NNZ, dtype=torch.int16), block_scale=z(V, 1)),   # too few blocks
    dict(t_val=z(V, NNZ, dtype=torch.uint8), block_scale=z(V - 1, 2)),
    dict(light_val=z(K - 1)),                                    # lighting lengths
    dict(light_idx=z(2, K // 2, dtype=torch.int32), light_val=z(2, K // 2)),
    dict(vert_rot=z(V, 3, 2)),                                   # not 3x3
    dict(frame_rot=z(4, 8)),
    dict(frame_rot=z(4, 3, 3), out=z(1, V)),                     # out for one frame
    dict(out=z(V + 1)),
    dict(cluster=z(V - 1, dtype=torch.int32)),                   # cluster length
    dict(cluster=z(V, dtype=torch.int32), t_idx=z(3, NNZ + 1, dtype=torch.int32)),
    dict(order=z(V + 2, dtype=torch.int32)),
    dict(brdf=z(2, 6, N, N // 2)),                               # brdf not [M, 6, n, n]
    dict(brdf=z(2, 6, N, N), material=z(V - 1, dtype=torch.int32)),
])
def test_relight_rejects_mis_shaped(over):
    shape_error(rrt.relight, **base(**over))


def test_relight_prepared_checks_shapes():
    prep = rrt.PreparedLighting(N, z(K, dtype=torch.int32), z(K), z(1, dtype=torch.uint8))
    shape_error(rrt.relight_prepared, prep, z(V, 3, 3), z(V, NNZ, dtype=torch.int32), z(V + 1, NNZ))
    shape_error(rrt.relight_prepared, prep, z(V, 3, 3), z(V, NNZ, dtype=torch.int32), z(V, NNZ),
                out=z(2, V))


def test_latlong_shapes():
    args = dict(H=N, light_idx=z(K, dtype=torch.int32), light_val=z(K), elev=z(V, 2),
                shift=z(V, 2, dtype=torch.int32), t_idx=z(V, NNZ, dtype=torch.int32), t_val=z(V, NNZ))
    reaches_device_check(rrt.relight_latlong, **args)
    shape_error(rrt.relight_latlong, **{**args, "shift": z(V - 1, 2, dtype=torch.int32)})
    shape_error(rrt.relight_latlong, **{**args, "elev": z(V, 3)})
    shape_error(rrt.relight_latlong, **{**args, "out": z(V - 1)})
    shape_error(rrt.relight_latlong, **{**args, "t_val": z(V, NNZ, dtype=torch.int16),
                                        "block_scale": z(V, 3)})


def test_relight_mlp_shapes():
    C = 3
    args = dict(n=N, light_idx=z(K, dtype=torch.int32), light_val=z(K), vert_rot=z(V, 3, 3),
                weights=z(rrt.RRT_MLP_WEIGHT_COUNT, dtype=torch.bfloat16),
                bias=z(rrt.RRT_MLP_BIAS_COUNT), supports=z(C, 256, dtype=torch.int32),
                scales=z(C, 256), pos_nrm=z(V, 6), cluster=z(V, dtype=torch.int32))
    reaches_device_check(rrt.relight_mlp, **args)
    for key, bad in [("weights", z(100, dtype=torch.bfloat16)), ("bias", z(1279)),
                     ("supports", z(C, 128, dtype=torch.int32)), ("scales", z(C + 1, 256)),
                     ("pos_nrm", z(V, 5)), ("pos_nrm", z(V + 1, 6)),
                     ("cluster", z(V + 1, dtype=torch.int32)), ("out", z(2, V))]:
        shape_error(rrt.relight_mlp, **{**args, key: bad})


def test_small_calls_shapes():
    shape_error(rrt.haar_forward, z(6, 8, 4))
    shape_error(rrt.haar_forward, z(6, 8, 8), out=z(6, 8, 4))
    shape_error(rrt.haar_inverse, z(6, 8, 8), out=z(5, 8, 8))
    shape_error(rrt.topk, z(3, 10), 4, out=(z(3, 3, dtype=torch.int32), z(3, 4)))
    shape_error(rrt.topk, z(3, 10), 11)
    shape_error(rrt.topk, z(30), 4)
    shape_error(rrt.haar_phase_shift, z(5, 8, 8), z(2, 3, 3))
    shape_error(rrt.haar_phase_shift, z(6, 8, 8), z(2, 3, 4))
    shape_error(rrt.relight_order, N, z(V, NNZ, dtype=torch.int32), out=z(V - 1, dtype=torch.int32))
    shape_error(rrt.relight_order, N, None)
    shape_error(rrt.convert, z(10), "bf16")
    shape_error(rrt.mlp_encode, z(4, 7))
    w = z(rrt.RRT_MLP_WEIGHT_COUNT, dtype=torch.bfloat16)
    b = z(rrt.RRT_MLP_BIAS_COUNT)
    shape_error(rrt.mlp_forward, w, b, z(4, 120, dtype=torch.bfloat16))
    shape_error(rrt.mlp_forward, w[:-1], b, z(4, 128, dtype=torch.bfloat16))
    shape_error(rrt.mlp_forward, w, b, z(4, 128, dtype=torch.bfloat16), out=z(4, 255))
    shape_error(rrt.mlp_backward, w, z(4, 128, dtype=torch.bfloat16), z(4, 200), None)
    shape_error(rrt.mlp_backward, w, z(4, 128, dtype=torch.bfloat16), z(4, 256), None, dw=z(10))
    shape_error(rrt.mse, z(10), z(9))
    shape_error(rrt.adam_step, z(10), z(10), z(9), z(10), 1, 1e-3)
