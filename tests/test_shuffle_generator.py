"""The host copy of the training shuffle's generator against the value the C++
standard fixes for it: the 10000th output of a default-constructed
std::mt19937_64 (seed 5489) is 9981545732273789042."""
import itertools

from tests.mt64 import mt19937_64, shuffled_epochs


def test_mt19937_64_ten_thousandth_output():
    g = mt19937_64(5489)
    assert next(itertools.islice(g, 9999, None)) == 9981545732273789042


def test_shuffles_are_permutations():
    for order in shuffled_epochs(37, 3, 11):
        assert sorted(order) == list(range(37))
