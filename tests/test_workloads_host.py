"""The synthetic workloads' layer chains (no GPU): every layer's input is the previous
layer's output, directly or after 2x2 pooling, so the products the bench and the tests run
have the shapes of the networks they stand for."""
import pytest

workloads = pytest.importorskip("paper_2411_09287_amd.workloads")


def out_shape(layer):
    if layer[0] == "fc":
        return (layer[2],)
    oh, ow = workloads.conv_out_hw(layer)
    return (oh, ow, layer[4])


def in_shape(layer):
    if layer[0] == "fc":
        return (layer[1],)
    return tuple(layer[6]) + (layer[3],)


def follows(prev, nxt):
    """nxt's input is prev's output, or prev's output 2x2-pooled, flattened for a dense layer."""
    cands = [prev]
    if len(prev) == 3 and prev[0] % 2 == 0 and prev[1] % 2 == 0:
        cands.append((prev[0] // 2, prev[1] // 2, prev[2]))
    for c in cands:
        if len(nxt) == 1:
            n = 1
            for v in c:
                n *= v
            if n == nxt[0]:
                return True
        elif c == nxt:
            return True
    return False


@pytest.mark.parametrize("name", sorted(workloads.MODELS))
def test_layer_chain(name):
    spec = workloads.MODELS[name]
    layers = spec["layers"]
    assert in_shape(layers[0]) == tuple(spec["input"]) or (
        len(in_shape(layers[0])) == 1 and in_shape(layers[0])[0] == spec["input"][0])
    for a, b in zip(layers, layers[1:]):
        assert follows(out_shape(a), in_shape(b)), (name, a, b)


def test_vgg_products():
    # batch 32, 32 x 32 x 3: the shapes the bench's step runs (first convolution K = 27)
    assert workloads.model_shapes("vgg") == [(32768, 27, 64), (32768, 576, 64), (8192, 576, 128),
                                             (8192, 1152, 128), (2048, 1152, 256), (2048, 2304, 256),
                                             (32, 4096, 256), (32, 256, 10)]


def test_strided_convolution_size():
    # the S-NN convolution: 5 x 5, pad 1, stride 2 on 28 x 28 -> 13 x 13 (845 = 13 13 5 features)
    layer = workloads.MODELS["snn"]["layers"][0]
    assert workloads.conv_stride(layer) == 2
    assert workloads.conv_out_hw(layer) == (13, 13)
